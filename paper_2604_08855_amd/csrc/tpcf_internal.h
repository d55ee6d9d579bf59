// tpcf_internal.h -- structures shared by the host side of the library and its gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpcf {

constexpr int kMaxBins = 32;   // bucket layout and the 32x32 MFMA output tile
constexpr int kMaxLmax = 10;
constexpr int kBlock = 64;       // secondaries per scratch block = one wavefront round
constexpr int kBatch = 4;        // pass rounds evaluated together (one batch of loads in flight)
// A bin's region takes new entries until it is within one batch of being full; the batch that
// crosses that soft limit still fits, then the shells are replayed and the region emptied.
constexpr int kSoftReserve = kBatch * kBlock;
constexpr int kMinRegionBlocks = kBatch + 1;
// Blocks after a wave's regions: the shell replay may read (and discard) up to four blocks past
// a region's last block.
constexpr int kScratchTail = 4;
constexpr int kQueueSegments = 8;  // task-queue segments, one per XCD
constexpr int kTileF32 = 32;        // primaries per contraction tile, mixed precision
constexpr int kTileF32Sphere = 64;  // the same on the sphere (few components, many primaries)
constexpr int kTileF64 = 16;        // primaries per contraction tile, FP64
__host__ __device__ constexpr int tile_primaries(bool f64, bool sphere) {
  return f64 ? kTileF64 : (sphere ? kTileF32Sphere : kTileF32);
}

// One catalogue as the kernels see it. Points of catalogue c occupy sorted positions
// [point_base, point_base + npoints) of the concatenated arrays; its cells occupy
// [cell_base, cell_base + nc^3] of cell_start (cell_start has one extra end entry per catalogue).
struct CatDesc {
  uint32_t point_base;
  uint32_t npoints;
  uint32_t cell_base;    // index of this catalogue's first cell_start entry
  int32_t nc;            // cells per axis in y and z
  int32_t nx;            // cells along x: a multiple of nc (thinner slabs clip stencil rows closer
                         // to the r_max sphere at no cost, a row being one contiguous run)
  int32_t K;             // lattice bits: coordinates are integers in [0, 2^K)
  int32_t sh;            // stored coordinate = q << sh (32-K when periodic, else 0)
  int32_t periodic;
  int32_t row_lo;        // stencil rows: offsets (dy, dz) in [row_lo, row_lo + row_w)^2
  int32_t row_w;
  int32_t sphere;        // 1: unit vectors on the sphere, stored shifted by +2 in a cube of side 4
  double box;
  double scale;          // 2^K / box
  double T[kMaxBins + 1];  // exact integer squared-separation thresholds (lattice units)
  // FP32 quantities of the per-primary stencil and of the fast bin decision (lattice units)
  float cs;              // cell side 2^K / nc
  float inv_cs;
  float inv_csx;         // nx / 2^K
  float span;            // 2^K
  float reach;           // r_max + margin
  float margin;
  float inv_delta_l;     // 2^-sh / bin width: bin position per unit of stored coordinate difference
  float u0;              // -r_min / bin width
  float eps;             // fast bin decisions need a fractional bin position in [eps, 1 - eps]
  float one_minus_eps;   // 1 - eps in FP32
  float half_inv_scale;  // sphere: 0.5 / scale, so that sqrt(R^2) * half_inv_scale = sin(theta / 2)
  int32_t asin_small;    // sphere: sin(theta_max / 2) <= 0.06, the three-term arcsine suffices
};

// Arguments of the persistent sweep kernel.
struct SweepArgs {
  const uint4* rec;             // sorted records: (Qx, Qy, Qz, float bits of w), then the sentinel
  const double* w64;            // sorted FP64 weights, then the sentinel's 0
  uint32_t sentinel;            // index of the zero-weight sentinel record (total points)
  const uint32_t* cell_start;   // per catalogue nc^3 + 1 entries
  const CatDesc* cats;
  int32_t ncat;
  int32_t nb;
  const uint32_t* task_list;    // NULL: task t is sorted position t
  const uint4* prim_rec;        // optional: task t is the pivot prim_rec[t] (shared pivots), not a point
  const double* prim_w64;       // FP64 weights of those pivots
  const uint32_t* prim_cat_start;  // with pivots: catalogue k owns pivots [start[k], start[k+1])
  uint32_t ntask;
  int32_t phase_rows;           // 1: each wave starts its stencil at the row matching its ticket's phase
  uint32_t* queue;              // [kQueueSegments] ticket counters, one per segment of the task list
  uint32_t* scratch;            // per wave: scratch_blocks + kScratchTail blocks of 64 sorted positions
  int32_t scratch_blocks;       // blocks per wave in bin regions
  const uint32_t* regions;      // [nb + 1]: bin b owns scratch blocks [regions[b], regions[b+1])
  void* tile;                   // per-wave a_lm tile area
  double* zeta;                 // [ncat][(lmax+1)][nb][nb]
  int32_t* counts;              // optional [total points][nb], by sorted position
  void* alm_debug;              // optional [total points][nb][NC] (float or double), by sorted position
  unsigned long long* stats;    // [0] pairs, [1] candidates
  unsigned long long* bin_pairs;  // [ncat][nb] ordered pairs per bin
  double* bin_dd;               // [ncat][nb] sum over pairs of w_p w_j per bin
  // moments -> a_lm, spread over the lanes: entry (q, lane), q < conv_q, adds
  // conv_coef[q * 64 + lane] * moment[m] to component c, with conv_idx[q * 64 + lane] =
  // m | c << 7 | last << 14 (last: the component is complete)
  const int16_t* conv_idx;
  const float* conv_coef32;
  const double* conv_coef64;
  int32_t conv_q;
  // deterministic form (NULL det_tiles: off): tile k covers tasks [det_tiles[k].x, det_tiles[k].y)
  // of one catalogue; its zeta contraction and weight sums go to det_out + k * det_stride
  const uint2* det_tiles;
  uint32_t ndet;
  double* det_out;
};

constexpr int kConvTerms = 6;

// Index k of the range [start(k), start(k+1)) holding i, for non-decreasing starts with start(0) = 0
// (binary search; empty ranges are skipped).
template <class Start>
__host__ __device__ __forceinline__ int range_of(Start start, int n, uint32_t i) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start(mid) <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Catalogue of sorted point i.
__device__ __forceinline__ int catalogue_of(const CatDesc* cats, int ncat, uint32_t i) {
  return range_of([&](int k) { return cats[k].point_base; }, ncat, i);
}

// Components per primary and bin: (lmax+1)^2 real numbers in 3D; on the sphere 2 m_max + 1
// (Re a_0, then Re and Im of a_m for m = 1..m_max).
__host__ __device__ constexpr int ncomp(int lmax, bool sphere = false) {
  return sphere ? 2 * lmax + 1 : (lmax + 1) * (lmax + 1);
}

}  // namespace tpcf
