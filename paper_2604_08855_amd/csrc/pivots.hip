// pivots.hip -- shared pivots (approximate): one pivot per occupied pivot cell (gfx950).
//
// The paper speeds its sweep up by letting spatially close pivots share one neighbour list, with
// closeness set by a pivot length scale that defaults to the mean separation (Implementation
// section). Here that is made concrete: pivots are grouped by a cubic grid of pivot cells of Hq
// lattice units, and each occupied cell contributes one pivot at the rounded mean lattice position
// of its members, carrying their summed weight; every point stays a secondary. The sweep kernel
// then runs over these pivots instead of the points.
//
// The cells are found by sorting, so only occupied cells cost anything (points on the sphere fill
// a thin shell of the cube):
//   k_pivot_keys : per point (cell-sorted records): its catalogue index above the Morton code of
//                  its pivot cell (gx, gy, gz), B bits per axis (B = 21 for one catalogue; fewer
//                  for batches, so that the key fits 63 bits). Cells of different catalogues
//                  never merge. Any one-to-one key groups the same cells; the Z order also makes
//                  the pivots, which the sweep takes in key order, come in compact patches, so
//                  the waves in flight have overlapping neighbourhoods.
//   radix sort   : rocPRIM, stable, so a cell's members stay in sorted-record order.
//   k_pivot_heads: 1 where a cell starts; an exclusive scan numbers the cells.
//   k_pivot_emit : one thread per cell start walks its members: pivot record (X << sh, FP32
//                  weight) and FP64 weight, X = (2 sum q + n) div (2 n) per axis (round half up of
//                  the mean), weights summed in member order.
//   k_pivot_starts: first pivot of every catalogue (keys are catalogue-major, so catalogue k's
//                  points hold sorted positions [point_base_k, point_base_k + n_k)).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "tpcf_internal.h"

namespace tpcf {

constexpr int kPivotAxisBits = 21;

// Bits of the catalogue index and per axis for a batch of ncat catalogues: 3 B + C <= 63.
__host__ __device__ inline int pivot_cat_bits(int ncat) {
  int c = 0;
  while ((1 << c) < ncat) ++c;
  return c;
}
int pivot_axis_bits(int ncat) {
  const int b = (63 - pivot_cat_bits(ncat)) / 3;
  return b < kPivotAxisBits ? b : kPivotAxisBits;
}

// The 21 low bits of v moved to bits 0, 3, 6, ..., 60 (masked shift-or spreading).
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__global__ void k_pivot_keys(const uint4* __restrict__ rec, uint32_t n, const CatDesc* __restrict__ cats, int ncat,
                             const unsigned long long* __restrict__ hq, int axis_bits,
                             unsigned long long* __restrict__ key, uint32_t* __restrict__ idx) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int c = catalogue_of(cats, ncat, s);
  const int sh = cats[c].sh;
  const uint64_t Hq = hq[c];
  const uint4 r = rec[s];
  const uint64_t gx = (uint64_t)(r.x >> sh) / Hq, gy = (uint64_t)(r.y >> sh) / Hq, gz = (uint64_t)(r.z >> sh) / Hq;
  key[s] = ((uint64_t)c << (3 * axis_bits)) | spread3(gx) | (spread3(gy) << 1) | (spread3(gz) << 2);
  idx[s] = s;
}

__global__ void k_pivot_heads(const unsigned long long* __restrict__ key, uint32_t n, uint32_t* __restrict__ head) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = (i == 0 || key[i] != key[i - 1]) ? 1u : 0u;
}

__global__ void k_pivot_emit(const unsigned long long* __restrict__ key, const uint32_t* __restrict__ idx,
                             const uint32_t* __restrict__ head, const uint32_t* __restrict__ slot,
                             const uint4* __restrict__ rec, const double* __restrict__ w64, uint32_t n,
                             const CatDesc* __restrict__ cats, int axis_bits, uint4* __restrict__ prim_rec,
                             double* __restrict__ prim_w) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !head[i]) return;
  const unsigned long long k = key[i];
  const int sh = cats[k >> (3 * axis_bits)].sh;
  unsigned long long sx = 0, sy = 0, sz = 0;
  double W = 0.0;
  uint32_t j = i;
  for (; j < n && key[j] == k; ++j) {
    const uint32_t s = idx[j];
    const uint4 r = rec[s];
    sx += r.x >> sh;
    sy += r.y >> sh;
    sz += r.z >> sh;
    W += w64[s];
  }
  const unsigned long long c = j - i, c2 = 2ull * c;
  const uint32_t X = (uint32_t)((2ull * sx + c) / c2), Y = (uint32_t)((2ull * sy + c) / c2),
                 Z = (uint32_t)((2ull * sz + c) / c2);
  const uint32_t g = slot[i];
  prim_rec[g] = make_uint4(X << sh, Y << sh, Z << sh, __float_as_uint((float)W));
  prim_w[g] = W;
}

__global__ void k_pivot_starts(const CatDesc* __restrict__ cats, int ncat, const uint32_t* __restrict__ slot,
                               uint32_t n, uint32_t* __restrict__ start) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ncat) start[k] = slot[cats[k].point_base];
  else if (k == ncat) start[k] = slot[n];
}

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* block_sum, hipStream_t s);

static inline unsigned blocks_of(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// Temporary bytes of the key sort for n points (the sort covers at most 63 key bits).
size_t pivot_sort_bytes(uint32_t n) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs(nullptr, bytes, (unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                  (uint32_t*)nullptr, (uint32_t*)nullptr, n, 0, 63);
  return bytes;
}

// Pivots of the cells of hq[k] lattice units (device, one per catalogue) over the n sorted
// records of ncat catalogues (cells per axis must stay below 2^pivot_axis_bits(ncat)):
// prim_rec[0..G), prim_w[0..G), catalogue-major; slot[n] receives G and start[0..ncat] the first
// pivot of every catalogue. Buffers: key_a, key_b (n), idx_a, idx_b, head (n), slot (n + 1),
// block_sum (scan blocks of n), sort_tmp (sort_bytes).
hipError_t build_pivots(const uint4* rec, const double* w64, uint32_t n, const CatDesc* cats, int ncat,
                        const unsigned long long* hq, unsigned long long* key_a, unsigned long long* key_b,
                        uint32_t* idx_a, uint32_t* idx_b, uint32_t* head, uint32_t* slot, uint32_t* block_sum,
                        void* sort_tmp, size_t sort_bytes, uint4* prim_rec, double* prim_w, uint32_t* start,
                        hipStream_t s) {
  const int B = pivot_axis_bits(ncat);
  const int bits = 3 * B + pivot_cat_bits(ncat);
  if (n) {
    hipLaunchKernelGGL(k_pivot_keys, dim3(blocks_of(n, 256)), dim3(256), 0, s, rec, n, cats, ncat, hq, B, key_a,
                       idx_a);
    size_t bytes = sort_bytes;
    hipError_t e = rocprim::radix_sort_pairs(sort_tmp, bytes, key_a, key_b, idx_a, idx_b, n, 0, bits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pivot_heads, dim3(blocks_of(n, 256)), dim3(256), 0, s, key_b, n, head);
  }
  hipError_t e = exclusive_scan_u32(head, slot, n, block_sum, s);
  if (e != hipSuccess) return e;
  if (n)
    hipLaunchKernelGGL(k_pivot_emit, dim3(blocks_of(n, 256)), dim3(256), 0, s, key_b, idx_b, head, slot, rec, w64, n,
                       cats, B, prim_rec, prim_w);
  hipLaunchKernelGGL(k_pivot_starts, dim3(blocks_of((size_t)ncat + 1, 64)), dim3(64), 0, s, cats, ncat, slot, n,
                     start);
  return hipGetLastError();
}

}  // namespace tpcf
