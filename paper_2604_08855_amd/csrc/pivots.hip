// pivots.hip -- shared pivots (approximate): one pivot per occupied pivot cell (gfx950).
//
// The paper speeds its sweep up by letting spatially close pivots share one neighbour list, with
// closeness set by a pivot length scale that defaults to the mean separation (Implementation
// section). Here that is made concrete: pivots are grouped by a cubic grid of pivot cells of Hq
// lattice units, and each occupied cell contributes one pivot at the rounded mean lattice position
// of its members, carrying their summed weight; every point stays a secondary. The sweep kernel
// then runs over these pivots instead of the points.
//
//   k_group_accum : per point (sorted records): member count, lattice-coordinate sums (64-bit
//                   integer atomics) and weight sum (FP64 atomics) of its pivot cell.
//   k_group_flag  : 1 for occupied cells (scanned into the pivots' output slots).
//   k_group_emit  : per occupied cell: pivot record (X << sh, FP32 weight) and FP64 weight, with
//                   X = (2 sum q + n) div (2 n) per axis (round half up of the mean).
#include "tpcf_internal.h"

namespace tpcf {

__global__ void k_group_accum(const uint4* __restrict__ rec, const double* __restrict__ w64, uint32_t n, int sh,
                              uint64_t Hq, uint32_t ng, uint32_t* __restrict__ count,
                              unsigned long long* __restrict__ sum, double* __restrict__ wsum) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint4 r = rec[s];
  const uint32_t qx = r.x >> sh, qy = r.y >> sh, qz = r.z >> sh;
  const uint32_t g = (uint32_t)((((uint64_t)qz / Hq) * ng + (uint64_t)qy / Hq) * ng + (uint64_t)qx / Hq);
  atomicAdd(&count[g], 1u);
  atomicAdd(&sum[3 * (size_t)g + 0], (unsigned long long)qx);
  atomicAdd(&sum[3 * (size_t)g + 1], (unsigned long long)qy);
  atomicAdd(&sum[3 * (size_t)g + 2], (unsigned long long)qz);
  atomicAdd(&wsum[g], w64[s]);
}

__global__ void k_group_flag(const uint32_t* __restrict__ count, uint32_t* __restrict__ flag, uint32_t ncell) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ncell) flag[g] = count[g] ? 1u : 0u;
}

__global__ void k_group_emit(const uint32_t* __restrict__ count, const unsigned long long* __restrict__ sum,
                             const double* __restrict__ wsum, const uint32_t* __restrict__ slot, uint32_t ncell,
                             int sh, uint4* __restrict__ prim_rec, double* __restrict__ prim_w) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncell) return;
  const uint32_t c = count[g];
  if (!c) return;
  const uint32_t i = slot[g];
  const unsigned long long c2 = 2ull * c;
  const uint32_t X = (uint32_t)((2ull * sum[3 * (size_t)g + 0] + c) / c2);
  const uint32_t Y = (uint32_t)((2ull * sum[3 * (size_t)g + 1] + c) / c2);
  const uint32_t Z = (uint32_t)((2ull * sum[3 * (size_t)g + 2] + c) / c2);
  const double W = wsum[g];
  prim_rec[i] = make_uint4(X << sh, Y << sh, Z << sh, __float_as_uint((float)W));
  prim_w[i] = W;
}

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void fill_f64(double* p, double v, size_t n, hipStream_t s);
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* block_sum, hipStream_t s);

static inline unsigned blocks_of(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// Builds the pivots of the ng^3 pivot cells of Hq lattice units over the n sorted records:
// prim_rec[0..G), prim_w[0..G) and slot[ng^3] (its entry ng^3 receives G). Buffers: count[ng^3],
// sum[3 ng^3], wsum[ng^3], flag[ng^3], slot[ng^3 + 1], block_sum[scan blocks].
hipError_t build_pivots(const uint4* rec, const double* w64, uint32_t n, int sh, uint64_t Hq, uint32_t ng,
                        uint32_t* count, unsigned long long* sum, double* wsum, uint32_t* flag, uint32_t* slot,
                        uint32_t* block_sum, uint4* prim_rec, double* prim_w, hipStream_t s) {
  const uint32_t ncell = ng * ng * ng;
  fill_u32(count, 0u, ncell, s);
  fill_u32(reinterpret_cast<uint32_t*>(sum), 0u, (size_t)ncell * 6, s);
  fill_f64(wsum, 0.0, ncell, s);
  if (n)
    hipLaunchKernelGGL(k_group_accum, dim3(blocks_of(n, 256)), dim3(256), 0, s, rec, w64, n, sh, Hq, ng, count, sum,
                       wsum);
  hipLaunchKernelGGL(k_group_flag, dim3(blocks_of(ncell, 256)), dim3(256), 0, s, count, flag, ncell);
  hipError_t e = exclusive_scan_u32(flag, slot, ncell, block_sum, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_emit, dim3(blocks_of(ncell, 256)), dim3(256), 0, s, count, sum, wsum, slot, ncell, sh,
                     prim_rec, prim_w);
  return hipGetLastError();
}

}  // namespace tpcf
