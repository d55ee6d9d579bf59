// grid.hip -- lattice snap and counting-sort cell grid for one or many catalogues (gfx950).
//
// The paper finds neighbours with an octree / kd-tree pruned into balls (Implementation
// section); here neighbours come from a uniform cubic cell grid built by a counting sort, which
// is what a wide GPU wants: every stencil row is a contiguous range of the cell-sorted records.
//
//   k_snap      : FP64 positions -> lattice coordinates q (FP64 multiply by 2^K/L, floor, wrap
//                 or clamp), stored shifted as q << sh; cell id; cell histogram (atomics);
//                 validation flags for non-finite values and non-periodic points outside the box.
//                 Points on the sphere are unit vectors, shifted by +2 into the cube [0, 4)^3.
//   k_scan_*    : exclusive scan of the histogram -> cell_start (three small kernels).
//   k_scatter   : each point claims a slot of its cell (atomic, so the order inside a cell is
//                 arbitrary at this point).
//   k_cellsort  : restores input order inside every cell, so the sorted layout (catalogue, cell,
//                 input index) and hence every summation order is reproducible: cells of up to
//                 64 points by a one-wave rank count, up to kCellSortMax by a bitonic sort in
//                 LDS, larger ones by a rank count of the whole workgroup.
//   k_gather    : writes the cell-sorted records (Qx, Qy, Qz, float w), FP64 weights and the
//                 permutation back to input order, then one zero-weight sentinel record.
#include "tpcf_internal.h"

namespace tpcf {

constexpr int kCellSortMax = 4096;

// Points on the sphere must be unit vectors to within 1e-6 in |v|^2 (flag bit 8).
__device__ __forceinline__ int unit_norm_flag(double px, double py, double pz) {
  const double r2 = px * px + py * py + pz * pz;
  return (r2 >= 1.0 - 1e-6 && r2 <= 1.0 + 1e-6) ? 0 : 8;
}

// Lattice coordinate of one position (periodic: mod 2^K; else clamped to [0, 2^K)).
__device__ __forceinline__ uint32_t snap_coord(double x, double scale, int K, int periodic) {
  const int64_t t = (int64_t)floor(x * scale);
  const int64_t M = (int64_t)1 << K;
  int64_t q;
  if (periodic) {
    q = t & (M - 1);
  } else {
    q = t < 0 ? 0 : (t > M - 1 ? M - 1 : t);
  }
  return (uint32_t)q;
}

__global__ void k_snap(const double* __restrict__ x, const double* __restrict__ y,
                       const double* __restrict__ z, const double* __restrict__ w, uint32_t n,
                       const CatDesc* __restrict__ cats, int ncat, uint4* __restrict__ qtmp,
                       uint32_t* __restrict__ cell, uint32_t* __restrict__ hist, int* __restrict__ err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = catalogue_of(cats, ncat, i);
  const CatDesc& cd = cats[c];
  double px = x[i], py = y[i], pz = z[i];
  const double pw = w ? w[i] : 1.0;
  int bad = 0;
  if (!isfinite(px) || !isfinite(py) || !isfinite(pz) || !isfinite(pw)) bad |= 1;
  if (cd.sphere) {
    bad |= unit_norm_flag(px, py, pz);
    px += 2.0;
    py += 2.0;
    pz += 2.0;
  }
  if (cd.periodic) {
    const double lim = cd.box * 1048576.0;
    if (fabs(px) > lim || fabs(py) > lim || fabs(pz) > lim) bad |= 4;
  } else if (px < 0.0 || px >= cd.box || py < 0.0 || py >= cd.box || pz < 0.0 || pz >= cd.box) {
    bad |= 2;
  }
  if (bad) {
    atomicOr(err, bad);
    px = py = pz = 0.0;
  }
  const uint32_t qx = snap_coord(px, cd.scale, cd.K, cd.periodic);
  const uint32_t qy = snap_coord(py, cd.scale, cd.K, cd.periodic);
  const uint32_t qz = snap_coord(pz, cd.scale, cd.K, cd.periodic);
  const uint64_t nc = (uint64_t)cd.nc, nx = (uint64_t)cd.nx;
  const uint32_t cx = (uint32_t)(((uint64_t)qx * nx) >> cd.K);
  const uint32_t cy = (uint32_t)(((uint64_t)qy * nc) >> cd.K);
  const uint32_t cz = (uint32_t)(((uint64_t)qz * nc) >> cd.K);
  const uint32_t id = cd.cell_base + (cz * (uint32_t)nc + cy) * (uint32_t)nx + cx;
  cell[i] = id;
  qtmp[i] = make_uint4(qx << cd.sh, qy << cd.sh, qz << cd.sh, __float_as_uint((float)pw));
  atomicAdd(&hist[id], 1u);
}

// Exclusive scan, stage 1: each block of 1024 threads scans 4096 entries.
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                             uint32_t* __restrict__ block_sum, uint32_t n) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? in[base + k] : 0u;
    s += v[k];
  }
  // inclusive scan of per-thread sums within the wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t incl = s;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
      uint32_t t = wsum[k];
      wsum[k] = run;
      run += t;
    }
    block_sum[blockIdx.x] = run;
  }
  __syncthreads();
  uint32_t excl = incl - s + wsum[wv];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = excl;
    excl += v[k];
  }
}

// Stage 2: one block scans the block sums (any count) in place, exclusive.
__global__ __launch_bounds__(64) void k_scan_sums(uint32_t* __restrict__ sums, uint32_t nblocks) {
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nblocks; base += 64) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < nblocks ? sums[i] : 0u;
    uint32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
      uint32_t t = __shfl_up(incl, off);
      if ((int)threadIdx.x >= off) incl += t;
    }
    if (i < nblocks) sums[i] = carry + incl - v;
    carry += __shfl(incl, 63);
  }
}

// Stage 3: add block offsets; the entry past the last cell receives the total.
__global__ void k_scan_add(uint32_t* __restrict__ out, const uint32_t* __restrict__ block_off, uint32_t n,
                           uint32_t total) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += block_off[i / kScanTile];
  if (i == 0) out[n] = total;
}

__global__ void k_scatter(const uint32_t* __restrict__ cell, const uint32_t* __restrict__ cell_start,
                          uint32_t* __restrict__ hist, uint32_t* __restrict__ slot_idx, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = cell[i];
  const uint32_t k = atomicSub(&hist[c], 1u) - 1u;
  slot_idx[cell_start[c] + k] = i;
}

// Cells are visited in chunks strided over the grid: a sparsely filled grid (a map on the sphere
// occupies a thin shell of its cube) has far more cells than points, so each chunk first reads the
// sizes of many cells at once and only the cells that need work are then processed one by one.
// Small cells: one wavefront per chunk of 64 cells; each cell of 2 to 64 points is sorted by the
// whole wave, each lane ranking its entry by input index (a one-point cell is copied).
constexpr uint32_t kCellSortGrid = 65536;
constexpr uint32_t kCellSortSmall = 64;

__global__ __launch_bounds__(64) void k_cellsort(const uint32_t* __restrict__ cell_start,
                                                 const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                 uint32_t ncell) {
  const uint32_t lane = threadIdx.x;
  for (uint32_t c0 = blockIdx.x * 64u; c0 < ncell; c0 += gridDim.x * 64u) {
    const uint32_t c = c0 + lane;
    uint32_t beg = 0, n = 0;
    if (c < ncell) {
      beg = cell_start[c];
      n = cell_start[c + 1] - beg;
    }
    uint64_t todo = __ballot(n > 0 && n <= kCellSortSmall);
    while (todo) {
      const int k = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1;
      const uint32_t b = __builtin_amdgcn_readlane(beg, k);
      const uint32_t m = __builtin_amdgcn_readlane(n, k);
      if (lane < m) {
        const uint32_t v = in[b + lane];
        uint32_t rank = 0;
        for (uint32_t q = 0; q < m; ++q) rank += in[b + q] < v ? 1u : 0u;
        out[b + rank] = v;
      }
    }
  }
}

// Larger cells, one workgroup of 256 per chunk of 256 cells: the chunk's cells above 64 points are
// listed in LDS, then each is sorted in turn by the whole workgroup: a bitonic sort of the cell's
// input indices in LDS (padded with 0xFFFFFFFF to a power of two) up to kCellSortMax entries,
// beyond that a rank count over the cell.
__global__ __launch_bounds__(256) void k_cellsort_large(const uint32_t* __restrict__ cell_start,
                                                        const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                        uint32_t ncell) {
  __shared__ uint32_t buf[kCellSortMax];
  __shared__ uint32_t list[256];
  __shared__ uint32_t nlist;
  const uint32_t tid = threadIdx.x;
  for (uint32_t c0 = blockIdx.x * 256u; c0 < ncell; c0 += gridDim.x * 256u) {
    if (tid == 0) nlist = 0;
    __syncthreads();
    const uint32_t cc = c0 + tid;
    if (cc < ncell && cell_start[cc + 1] - cell_start[cc] > kCellSortSmall) list[atomicAdd(&nlist, 1u)] = cc;
    __syncthreads();
    const uint32_t cnt = nlist;
    for (uint32_t q = 0; q < cnt; ++q) {
      const uint32_t c = list[q];
      const uint32_t beg = cell_start[c], end = cell_start[c + 1];
      const uint32_t n = end - beg;
      if (n > (uint32_t)kCellSortMax) {
        for (uint32_t k = tid; k < n; k += 256) {
          const uint32_t v = in[beg + k];
          uint32_t rank = 0;
          for (uint32_t m = 0; m < n; ++m) rank += in[beg + m] < v ? 1u : 0u;
          out[beg + rank] = v;
        }
        continue;
      }
      uint32_t P = 1;
      while (P < n) P <<= 1;
      for (uint32_t k = tid; k < P; k += 256) buf[k] = k < n ? in[beg + k] : 0xFFFFFFFFu;
      __syncthreads();
      for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
          for (uint32_t t = tid; t < (P >> 1); t += 256) {
            const uint32_t i = 2 * t - (t & (stride - 1));  // lower index of the pair
            const uint32_t j = i + stride;
            const uint32_t a = buf[i], b = buf[j];
            const bool up = (i & size) == 0;
            if ((a > b) == up) {
              buf[i] = b;
              buf[j] = a;
            }
          }
          __syncthreads();
        }
      }
      for (uint32_t k = tid; k < n; k += 256) out[beg + k] = buf[k];
      __syncthreads();
    }
    __syncthreads();  // every thread has read nlist and list before the next chunk resets them
  }
}

__global__ void k_gather(const uint32_t* __restrict__ order, const uint4* __restrict__ qtmp,
                         const double* __restrict__ w, uint4* __restrict__ rec, double* __restrict__ w64,
                         uint32_t* __restrict__ perm, uint32_t n) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > n) return;
  if (s == n) {  // sentinel record after the last point: weight 0, read by padding entries
    rec[n] = make_uint4(0u, 0u, 0u, 0u);
    w64[n] = 0.0;
    return;
  }
  const uint32_t i = order[s];
  rec[s] = qtmp[i];
  w64[s] = w ? w[i] : 1.0;
  perm[s] = i;
}

// Validation of device-resident inputs: bit 1 non-finite value, bit 2 non-periodic point outside
// [0, box), bit 4 periodic coordinate beyond 2^20 box sides, bit 8 a point on the sphere that is
// not a unit vector.
__global__ void k_validate(const double* __restrict__ x, const double* __restrict__ y,
                           const double* __restrict__ z, const double* __restrict__ w, uint32_t n,
                           const CatDesc* __restrict__ cats, int ncat, int* __restrict__ err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const CatDesc& cd = cats[catalogue_of(cats, ncat, i)];
  const double px = x[i], py = y[i], pz = z[i], pw = w ? w[i] : 1.0;
  int bad = 0;
  if (!isfinite(px) || !isfinite(py) || !isfinite(pz) || !isfinite(pw)) bad |= 1;
  else if (cd.sphere) {
    bad |= unit_norm_flag(px, py, pz);
  } else if (cd.periodic) {
    const double lim = cd.box * 1048576.0;
    if (fabs(px) > lim || fabs(py) > lim || fabs(pz) > lim) bad |= 4;
  } else if (px < 0.0 || px >= cd.box || py < 0.0 || py >= cd.box || pz < 0.0 || pz >= cd.box) {
    bad |= 2;
  }
  if (bad) atomicOr(err, bad);
}

// Records and FP64 weights with each weight squared (the secondaries of the degenerate-term
// sweep); the FP32 weight bits hold the rounded FP64 square.
__global__ void k_square_weights(const uint4* __restrict__ rec, const double* __restrict__ w64, uint32_t n,
                                 uint4* __restrict__ out, double* __restrict__ w2) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = w64[i] * w64[i];
  uint4 r = rec[i];
  r.w = __float_as_uint((float)v);
  out[i] = r;
  w2[i] = v;
}

// FP32 inputs widened to the FP64 staging arrays (exact).
__global__ void k_widen_f32(const float* __restrict__ in, double* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* __restrict__ p, double v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------------------------------
// Host launchers (stream-ordered, no synchronisation, no memset nodes: safe under capture).
// ------------------------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
}
void widen_f32(const float* in, double* out, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_widen_f32, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
}
void fill_f64(double* p, double v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
}

void validate_inputs(const double* x, const double* y, const double* z, const double* w, uint32_t n,
                     const CatDesc* cats, int ncat, int* err, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_validate, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, z, w, n, cats, ncat, err);
}

hipError_t square_weights(const uint4* rec, const double* w64, uint32_t n, uint4* out, double* w2, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_square_weights, dim3(blocks_for(n, 256)), dim3(256), 0, s, rec, w64, n, out, w2);
  return hipGetLastError();
}

size_t scan_block_count(uint32_t ncell) { return (ncell + kScanTile - 1) / kScanTile; }

// out[n] = out[n-1] + in[n-1] (the total), after the exclusive scan of in[0..n).
__global__ void k_scan_total(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, uint32_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = n ? out[n - 1] + in[n - 1] : 0u;
}

// Exclusive scan of in[0..n) into out[0..n], out[n] = total. block_sum holds scan_block_count(n)
// entries.
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* block_sum, hipStream_t s) {
  const uint32_t nb = (uint32_t)scan_block_count(n);
  if (n) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kScanThreads), 0, s, in, out, block_sum, n);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(64), 0, s, block_sum, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, block_sum, n, 0u);
  }
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, s, in, out, n);
  return hipGetLastError();
}

// Builds the cell-sorted layout. Buffers: qtmp[n], cell[n], hist[ncell], idx_a[n], idx_b[n],
// block_sum[scan_block_count(ncell)], err[1] (all device). Outputs: cell_start[ncell+1],
// rec[n], w64[n], perm[n].
hipError_t build_grid(const double* x, const double* y, const double* z, const double* w, uint32_t n,
                      const CatDesc* cats, int ncat, uint32_t ncell, uint4* qtmp, uint32_t* cell,
                      uint32_t* hist, uint32_t* idx_a, uint32_t* idx_b, uint32_t* block_sum, int* err,
                      uint32_t* cell_start, uint4* rec, double* w64, uint32_t* perm, hipStream_t s) {
  fill_u32(hist, 0u, ncell, s);
  if (n)
    hipLaunchKernelGGL(k_snap, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, z, w, n, cats, ncat, qtmp,
                       cell, hist, err);
  const uint32_t nb = (uint32_t)scan_block_count(ncell);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kScanThreads), 0, s, hist, cell_start, block_sum, ncell);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(64), 0, s, block_sum, nb);
  hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(ncell + 1, 256)), dim3(256), 0, s, cell_start, block_sum,
                     ncell, n);
  if (n) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, cell, cell_start, hist, idx_a, n);
    const uint32_t g_small = std::min<uint32_t>(kCellSortGrid, (ncell + 63) / 64);
    const uint32_t g_large = std::min<uint32_t>(kCellSortGrid, (ncell + 255) / 256);
    hipLaunchKernelGGL(k_cellsort, dim3(g_small), dim3(64), 0, s, cell_start, idx_a, idx_b, ncell);
    hipLaunchKernelGGL(k_cellsort_large, dim3(g_large), dim3(256), 0, s, cell_start, idx_a, idx_b, ncell);
  }
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, idx_b, qtmp, w, rec, w64, perm, n);
  return hipGetLastError();
}

// Primary ranges: the sorted positions s whose input index perm[s] lies in [lo, hi), in sorted
// order (flags, an exclusive scan, a compacting scatter), so that a range sweep keeps the cell
// order of its primaries.
__global__ void k_range_flags(const uint32_t* __restrict__ perm, uint32_t n, uint32_t lo, uint32_t hi,
                              uint32_t* __restrict__ flag) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) flag[s] = (perm[s] - lo < hi - lo) ? 1u : 0u;  // lo <= perm[s] < hi
}
__global__ void k_range_emit(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos, uint32_t n,
                             uint32_t* __restrict__ list) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n && flag[s]) list[pos[s]] = s;
}

// Task list of the primaries with input index in [lo, hi) into list (n entries); pos[n] receives
// their count. Buffers: flag (n), pos (n + 1), block_sum (scan_block_count(n)).
hipError_t range_tasks(const uint32_t* perm, uint32_t n, uint32_t lo, uint32_t hi, uint32_t* flag, uint32_t* pos,
                       uint32_t* block_sum, uint32_t* list, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_range_flags, dim3(blocks_for(n, 256)), dim3(256), 0, s, perm, n, lo, hi, flag);
  hipError_t e = exclusive_scan_u32(flag, pos, n, block_sum, s);
  if (e != hipSuccess) return e;
  if (n) hipLaunchKernelGGL(k_range_emit, dim3(blocks_for(n, 256)), dim3(256), 0, s, flag, pos, n, list);
  return hipGetLastError();
}

// Copies per-primary debug rows from sorted to input order and widens them to int64 / FP64.
__global__ void k_unsort_counts(const int32_t* __restrict__ in, const uint32_t* __restrict__ perm,
                                int64_t* __restrict__ out, uint32_t n, int nb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n * nb) return;
  const uint32_t s = (uint32_t)(i / nb);
  const int b = (int)(i % nb);
  out[(size_t)perm[s] * nb + b] = in[i];
}
template <class T>
__global__ void k_unsort_alm(const T* __restrict__ in, const uint32_t* __restrict__ perm,
                             double* __restrict__ out, uint32_t n, int row) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n * row) return;
  const uint32_t s = (uint32_t)(i / row);
  const int k = (int)(i % row);
  out[(size_t)perm[s] * row + k] = (double)in[i];
}

void unsort_counts(const int32_t* in, const uint32_t* perm, int64_t* out, uint32_t n, int nb, hipStream_t s) {
  const size_t tot = (size_t)n * nb;
  if (tot) hipLaunchKernelGGL(k_unsort_counts, dim3(blocks_for(tot, 256)), dim3(256), 0, s, in, perm, out, n, nb);
}
void unsort_alm(const void* in, bool f64, const uint32_t* perm, double* out, uint32_t n, int row, hipStream_t s) {
  const size_t tot = (size_t)n * row;
  if (!tot) return;
  if (f64)
    hipLaunchKernelGGL(k_unsort_alm<double>, dim3(blocks_for(tot, 256)), dim3(256), 0, s,
                       (const double*)in, perm, out, n, row);
  else
    hipLaunchKernelGGL(k_unsort_alm<float>, dim3(blocks_for(tot, 256)), dim3(256), 0, s,
                       (const float*)in, perm, out, n, row);
}

}  // namespace tpcf
