// sweep.hip -- the persistent pair sweep: cell-grid neighbour scan, exact radial binning,
// spherical-harmonic shells a_lm(p, b) accumulated in registers, and the bin-pair contraction
// zeta_l(b1, b2) += w_p sum_m a_lm(b1) a*_lm(b2) on MFMA, for gfx950 (wave64).
//
// Method (paper, Implementation section): for each pivot (primary), find every neighbour in
// the search range and fill the multipole bins; the per-multipole work uses a recurrence
// instead of trigonometric functions. Nearby pivots share neighbour lists: here every primary
// of a grid cell scans the same stencil of cells.
//
// One wavefront owns one primary at a time (tasks come from a global atomic queue):
//   pass    : the wave walks the primary's stencil in rounds of 64 candidates, decides each
//             candidate's bin exactly (integer lattice separation, FP64 squared distance against
//             integer thresholds) and appends it to a per-bin LDS bucket. A bucket that reaches
//             64 entries is written as one block of 64 sorted positions to the wave's scratch
//             area, so every block holds 64 secondaries of a single bin.
//   shells  : bin by bin, the wave replays that bin's blocks. Each lane evaluates the
//             (l_max+1)^2 real harmonic components of its pair with a register recurrence
//             (powers of (x - i y) times monic associated-Legendre polynomials in z) and adds them
//             into register accumulators. Every <= 64 rounds the 64 lanes are reduced with a
//             transpose-reduction (permlane32/16 swaps, then DPP) and added into the shell with a
//             compensated (Kahan) sum (mixed precision) or plain FP64.
//   contract: every 32 (mixed) or 16 (FP64) primaries, the wave multiplies its tile of shells on
//             MFMA: per l, zeta_l += X_l diag(f w) X_l^T with X_l the [bins x (primaries*(2l+1))]
//             matrix of real components. Mixed: three-piece BF16 split, six products, FP32
//             accumulation within the tile. FP64: v_mfma_f64_16x16x4. Tile results are added into
//             a per-wave FP64 partial; partials are added into zeta (FP64 atomics) when the wave
//             changes catalogue and when it finishes.
#include <type_traits>

#include "tpcf_internal.h"

namespace tpcf {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int I>
using ic = std::integral_constant<int, I>;

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(ic<B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr uint16_t kEnd = 0xFFFFu;

// ------------------------------------------------------------------------------------------
// Harmonic plan: which m-chains a group holds and where each real component lives.
//
// Real component layout (l-major): index l*l for Re a_l0, l*l + 2m - 1 for Re a_lm and
// l*l + 2m for Im a_lm (m = 1..l). The FP64 sweep with more than 64 components splits the
// m-chains into two groups (two passes over a bin) to stay within the register file.
// ------------------------------------------------------------------------------------------
template <int LMAX, bool F64>
struct Plan {
  static constexpr int NC = (LMAX + 1) * (LMAX + 1);
  static constexpr bool TWO = F64 && NC > 64;
  static constexpr int NG = TWO ? 2 : 1;
  static constexpr int chain(int m) { return m == 0 ? LMAX + 1 : 2 * (LMAX - m + 1); }
  // Greedy balance of the chains over two groups, largest chain first.
  static constexpr int group_of(int m) {
    if (!TWO) return 0;
    int tot[2] = {0, 0};
    bool done[LMAX + 1] = {};
    int result = 0;
    for (int it = 0; it <= LMAX; ++it) {
      int best = -1;
      for (int mm = 0; mm <= LMAX; ++mm)
        if (!done[mm] && (best < 0 || chain(mm) > chain(best))) best = mm;
      done[best] = true;
      int g = tot[1] < tot[0] ? 1 : 0;
      tot[g] += chain(best);
      if (best == m) result = g;
    }
    return result;
  }
  static constexpr int gsize(int g) {
    int s = 0;
    for (int m = 0; m <= LMAX; ++m)
      if (group_of(m) == g) s += chain(m);
    return s;
  }
  // Register slots per lane before the reduction: a multiple of 64.
  static constexpr int slots(int g) { return gsize(g) <= 64 ? 64 : 128; }
  // Position of component (l, m, part) inside its group (part 0 = Re, 1 = Im).
  static constexpr int loc(int l, int m, int part) {
    int off = 0;
    for (int mm = 0; mm < m; ++mm)
      if (group_of(mm) == group_of(m)) off += chain(mm);
    return off + (m == 0 ? (l - m) : 2 * (l - m) + part);
  }
  // Global real-component index of group-local slot s (-1 for padding).
  __host__ __device__ static constexpr int global_of(int g, int s) {
    int off = 0;
    for (int m = 0; m <= LMAX; ++m) {
      if (group_of(m) != g) continue;
      int c = chain(m);
      if (s < off + c) {
        int r = s - off;
        if (m == 0) return r * r;  // l = r
        int l = m + r / 2, part = r % 2;
        return l * l + 2 * m - 1 + part;
      }
      off += c;
    }
    return -1;
  }
};

// Recurrence coefficient of the monic associated-Legendre polynomials in z:
// H_mm = 1, H_{m+1,m} = z, H_lm = z H_{l-1,m} - beta_lm H_{l-2,m}.
__host__ __device__ constexpr double beta(int l, int m) {
  return double((l + m - 1) * (l - 1 - m)) / double((2 * l - 1) * (2 * l - 3));
}

// Adds the group-G components of w * conj(Y_lm(x,y,z)) / C_lm into acc (unnormalised: the
// constant C_lm is applied when a shell is stored). (x, y, z) is a unit vector.
template <int LMAX, bool F64, int G, class real, int S>
__device__ __forceinline__ void add_harmonics(real (&acc)[S], real x, real y, real z, real w) {
  using P = Plan<LMAX, F64>;
  real pr = w, pi = real(0);  // w (x - i y)^m
  const real zz = z * z;
  static_for<0, LMAX + 1>([&](auto M) {
    constexpr int m = M;
    if constexpr (m > 0) {
      real nr = pr * x + pi * y;
      real ni = pi * x - pr * y;
      pr = nr;
      pi = ni;
    }
    if constexpr (P::group_of(m) == G) {
      acc[P::loc(m, m, 0)] += pr;
      if constexpr (m > 0) acc[P::loc(m, m, 1)] += pi;
      if constexpr (m + 1 <= LMAX) {
        acc[P::loc(m + 1, m, 0)] += z * pr;
        if constexpr (m > 0) acc[P::loc(m + 1, m, 1)] += z * pi;
      }
      real h2 = real(1), h1 = z;
      static_for<m + 2, LMAX + 1>([&](auto L) {
        constexpr int l = L;
        constexpr real bt = real(beta(l, m));
        real h = (l == m + 2) ? (zz - bt) : (z * h1 - bt * h2);
        acc[P::loc(l, m, 0)] += h * pr;
        if constexpr (m > 0) acc[P::loc(l, m, 1)] += h * pi;
        h2 = h1;
        h1 = h;
      });
    }
  });
}

// ------------------------------------------------------------------------------------------
// Cross-lane transpose-reduction. Input: S values per lane (S = 64 or 128). Output: slot k of
// lane L (k < S/64) holds the wave-wide sum of component (S/64)*L + k.
// Stage pairs: lanes 32 apart (permlane32 swap), 16 apart (permlane16 swap), then within rows
// of 16 by DPP row_mirror, row_half_mirror and quad permutations. At each stage a lane keeps
// the half of its values selected by one lane-index bit and receives the partner's copy of it.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float pair32(float a, float b) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair16(float a, float b) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double pair32(double a, double b) {
  uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)ua, (uint32_t)ub, false, false);
  auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
  double na = __longlong_as_double((int64_t)(((uint64_t)hi[0] << 32) | lo[0]));
  double nb = __longlong_as_double((int64_t)(((uint64_t)hi[1] << 32) | lo[1]));
  return na + nb;
}
__device__ __forceinline__ double pair16(double a, double b) {
  uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ua, (uint32_t)ub, false, false);
  auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
  double na = __longlong_as_double((int64_t)(((uint64_t)hi[0] << 32) | lo[0]));
  double nb = __longlong_as_double((int64_t)(((uint64_t)hi[1] << 32) | lo[1]));
  return na + nb;
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  uint64_t u = __double_as_longlong(v);
  uint32_t lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
  uint32_t hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}
template <int CTRL, class real>
__device__ __forceinline__ real dpp_pair(real a, real b, bool upper) {
  real send = upper ? a : b;
  real keep = upper ? b : a;
  return keep + dpp<CTRL>(send);
}

constexpr int kRowMirror = 0x140, kHalfMirror = 0x141, kQuadXor2 = 0x4E, kQuadXor1 = 0xB1;

template <int S, class real>
__device__ __forceinline__ void transpose_reduce(real (&v)[S], int lane) {
  static_for<0, S / 2>([&](auto k) { v[k] = pair32(v[k], v[k + S / 2]); });
  static_for<0, S / 4>([&](auto k) { v[k] = pair16(v[k], v[k + S / 4]); });
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
  static_for<0, S / 8>([&](auto k) { v[k] = dpp_pair<kRowMirror>(v[k], v[k + S / 8], b3); });
  static_for<0, S / 16>([&](auto k) { v[k] = dpp_pair<kHalfMirror>(v[k], v[k + S / 16], b2); });
  static_for<0, S / 32>([&](auto k) { v[k] = dpp_pair<kQuadXor2>(v[k], v[k + S / 32], b1); });
  static_for<0, S / 64>([&](auto k) { v[k] = dpp_pair<kQuadXor1>(v[k], v[k + S / 64], b0); });
}

// ------------------------------------------------------------------------------------------
// Pair geometry.
// ------------------------------------------------------------------------------------------
struct Primary {
  uint32_t qx, qy, qz;  // stored lattice coordinates (shifted)
  int sh;
};

// Lattice displacement of a secondary from the primary: the shifted coordinates wrap modulo
// 2^32, so the arithmetic shift back gives the minimum image when periodic.
__device__ __forceinline__ void displacement(const Primary& P, uint4 r, int& dx, int& dy, int& dz) {
  dx = (int)(r.x - P.qx) >> P.sh;
  dy = (int)(r.y - P.qy) >> P.sh;
  dz = (int)(r.z - P.qz) >> P.sh;
}

// Unit vector of a lattice displacement.
__device__ __forceinline__ void unit(int dx, int dy, int dz, float& x, float& y, float& z) {
  float fx = (float)dx, fy = (float)dy, fz = (float)dz;
  float r2 = fx * fx + fy * fy + fz * fz;
  float ri = __builtin_amdgcn_rsqf(r2);
  x = fx * ri;
  y = fy * ri;
  z = fz * ri;
}
__device__ __forceinline__ void unit(int dx, int dy, int dz, double& x, double& y, double& z) {
  double fx = (double)dx, fy = (double)dy, fz = (double)dz;
  double r2 = fma(fx, fx, fma(fy, fy, fz * fz));
  double ri = __builtin_amdgcn_rsq(r2);
  // two Newton steps from the hardware estimate
  double h = r2 * ri;
  ri = fma(ri * 0.5, fma(-h, ri, 1.0), ri);
  h = r2 * ri;
  ri = fma(ri * 0.5, fma(-h, ri, 1.0), ri);
  x = fx * ri;
  y = fy * ri;
  z = fz * ri;
}

// ------------------------------------------------------------------------------------------
// Contraction of one tile of shells on MFMA.
// tile: [TP][nb][NC] normalised a_lm (real components), wt: [TP] weights in LDS, nt valid
// primaries. Adds zeta_l(b1, b2) of the tile into part[(l*nb + b1)*nb + b2] (FP64, per wave).
// ------------------------------------------------------------------------------------------
template <int LMAX>
__device__ __noinline__ void contract_tile(const float* __restrict__ tile, const float* wt, int nt,
                                           int nb, double* __restrict__ part, int lane) {
  constexpr int NC = (LMAX + 1) * (LMAX + 1);
  const int b = lane & 31;
  const int kh = (lane >> 5) * 8;
  const bool brow = b < nb;
#pragma unroll 1
  for (int l = 0; l <= LMAX; ++l) {
    const int n2 = 2 * l + 1;
    const int K = nt * n2;
    floatx16 acc = {};
    // (t, cc) of this lane's first k, advanced incrementally
    int t0 = kh / n2, c0 = kh - (kh / n2) * n2;
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += 16) {
      bf16x8 a0, a1, a2, b0, b1, b2;
      int t = t0, cc = c0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + kh + j;
        float xv = 0.f, wv = 0.f;
        if (brow && k < K) {
          xv = tile[(t * nb + b) * NC + l * l + cc];
          wv = wt[t] * (cc == 0 ? 1.f : 2.f);
        }
        const float yv = xv * wv;
        // three-piece BF16 split: v = v0 + v1 + v2 to within 2^-27 |v|
        const __bf16 x0 = (__bf16)xv;
        const float xr = xv - (float)x0;
        const __bf16 x1 = (__bf16)xr;
        const __bf16 x2 = (__bf16)(xr - (float)x1);
        const __bf16 y0 = (__bf16)yv;
        const float yr = yv - (float)y0;
        const __bf16 y1 = (__bf16)yr;
        const __bf16 y2 = (__bf16)(yr - (float)y1);
        a0[j] = x0;
        a1[j] = x1;
        a2[j] = x2;
        b0[j] = y0;
        b1[j] = y1;
        b2[j] = y2;
        if (++cc == n2) {
          cc = 0;
          ++t;
        }
      }
      // advance the first (t, cc) by 16
      c0 += 16;
      while (c0 >= n2) {
        c0 -= n2;
        ++t0;
      }
      // every product of total order <= 2, smallest first
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b2, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
    }
    const int col = lane & 31;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
      if (row < nb && col < nb) part[(l * nb + row) * nb + col] += (double)acc[r];
    }
  }
}

template <int LMAX>
__device__ __noinline__ void contract_tile(const double* __restrict__ tile, const double* wt, int nt,
                                           int nb, double* __restrict__ part, int lane) {
  constexpr int NC = (LMAX + 1) * (LMAX + 1);
  const int rl = lane & 15;
  const int kq = lane >> 4;
  const bool two = nb > 16;
#pragma unroll 1
  for (int l = 0; l <= LMAX; ++l) {
    const int n2 = 2 * l + 1;
    const int K = nt * n2;
    doublex4 acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
    int t = kq / n2, cc = kq - (kq / n2) * n2;  // (primary, component) of k = k0 + kq
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + kq;
      double x0 = 0.0, x1 = 0.0, y0 = 0.0, y1 = 0.0;
      if (k < K) {
        const double wf = wt[t] * (cc == 0 ? 1.0 : 2.0);
        const double* src = tile + (size_t)t * nb * NC + l * l + cc;
        if (rl < nb) {
          x0 = src[rl * NC];
          y0 = x0 * wf;
        }
        if (two && 16 + rl < nb) {
          x1 = src[(16 + rl) * NC];
          y1 = x1 * wf;
        }
      }
      acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc00, 0, 0, 0);
      if (two) {
        acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc01, 0, 0, 0);
        acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc10, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc11, 0, 0, 0);
      }
      cc += 4;
      while (cc >= n2) {
        cc -= n2;
        ++t;
      }
    }
    // D[i][j] of a 16x16 block: lane j + 16*(i%4), register i/4.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = kq + 4 * r;
      if (row < nb && rl < nb) part[(l * nb + row) * nb + rl] += acc00[r];
      if (two) {
        if (row < nb && 16 + rl < nb) part[(l * nb + row) * nb + 16 + rl] += acc01[r];
        if (16 + row < nb && rl < nb) part[(l * nb + 16 + row) * nb + rl] += acc10[r];
        if (16 + row < nb && 16 + rl < nb) part[(l * nb + 16 + row) * nb + 16 + rl] += acc11[r];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// The persistent sweep kernel.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int find_cat(const CatDesc* cats, int ncat, uint32_t p) {
  int lo = 0, hi = ncat - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cats[mid].point_base <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class T>
__device__ __forceinline__ T uniform(T v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// LDS layout (bytes), one wavefront per workgroup.
struct Lds {
  static constexpr int T = 0;                    // double[kMaxBins + 1]
  static constexpr int WT = 272;                 // real[32]
  static constexpr int BCNT = WT + 256;          // uint32[32]
  static constexpr int BTOT = BCNT + 128;        // uint32[32]
  static constexpr int HEAD = BTOT + 128;        // uint16[32]
  static constexpr int TAIL = HEAD + 64;         // uint16[32]
  static constexpr int NEXT = TAIL + 64;         // uint16[S]
  static __host__ __device__ int bucket(int S) { return (NEXT + 2 * S + 15) & ~15; }
  static __host__ __device__ int bytes(int S, int nb) { return bucket(S) + nb * kBucketCap * 4; }
};

template <int LMAX, bool F64>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void sweep_kernel(SweepArgs a) {
  using real = std::conditional_t<F64, double, float>;
  using P = Plan<LMAX, F64>;
  constexpr int NC = P::NC;
  constexpr int TP = F64 ? kTileF64 : kTileF32;

  extern __shared__ __align__(16) unsigned char smem[];
  double* sT = reinterpret_cast<double*>(smem + Lds::T);
  real* swt = reinterpret_cast<real*>(smem + Lds::WT);
  uint32_t* bcnt = reinterpret_cast<uint32_t*>(smem + Lds::BCNT);
  uint32_t* btot = reinterpret_cast<uint32_t*>(smem + Lds::BTOT);
  uint16_t* head = reinterpret_cast<uint16_t*>(smem + Lds::HEAD);
  uint16_t* tail = reinterpret_cast<uint16_t*>(smem + Lds::TAIL);
  uint16_t* nxt = reinterpret_cast<uint16_t*>(smem + Lds::NEXT);
  const int S = a.scratch_blocks;
  uint32_t* bucket = reinterpret_cast<uint32_t*>(smem + Lds::bucket(S));

  const int lane = threadIdx.x;
  const int nb = a.nb;
  const uint32_t wave = blockIdx.x;
  uint32_t* scratch = a.scratch + (size_t)wave * S * kBlock;
  real* tile = reinterpret_cast<real*>(a.tile) + (size_t)wave * (TP * nb * NC + (LMAX + 1) * nb * nb * (F64 ? 1 : 2));
  // per-wave FP64 zeta partial follows the tile area
  double* part = reinterpret_cast<double*>(tile + TP * nb * NC);

  // Component index and normalisation of the slots this lane holds after a reduction.
  int comp[P::NG][2];
  real cs[P::NG][2];
  static_for<0, P::NG>([&](auto G) {
    constexpr int per = P::slots(G) / 64;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      int c = k < per ? P::global_of(G, per * lane + k) : -1;
      comp[G][k] = c;
      cs[G][k] = c >= 0 ? (F64 ? (real)a.cscale64[c] : (real)a.cscale32[c]) : real(0);
    }
  });

  for (int i = lane; i < (LMAX + 1) * nb * nb; i += 64) part[i] = 0.0;

  int tile_n = 0, tile_cat = -1, part_cat = -1, cur_cat = -1;
  unsigned long long my_pairs = 0, my_cand = 0;

  // Catalogue parameters (wave-uniform).
  int sh = 0, K = 0, nc = 0, periodic = 0, st_base = 0, nst = 0;
  uint32_t cell_base = 0;
  float rmin_l = 0.f, inv_dl = 0.f;

  auto flush_part = [&]() {
    if (part_cat >= 0) {
      double* z = a.zeta + (size_t)part_cat * (LMAX + 1) * nb * nb;
      for (int i = lane; i < (LMAX + 1) * nb * nb; i += 64) {
        double v = part[i];
        if (v != 0.0) atomicAdd(&z[i], v);
        part[i] = 0.0;
      }
    }
  };
  auto do_contract = [&]() {
    if (tile_n == 0) return;
    if (part_cat != tile_cat) {
      flush_part();
      part_cat = tile_cat;
    }
    __syncthreads();
    contract_tile<LMAX>(tile, swt, tile_n, nb, part, lane);
    __syncthreads();
    tile_n = 0;
  };

  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(a.queue, 1u);
    t = uniform(t);
    if (t >= a.ntask) break;
    const uint32_t p = uniform(a.task_list ? a.task_list[t] : t);
    const int cat = uniform(find_cat(a.cats, a.ncat, p));
    if (cat != tile_cat) {
      do_contract();
      tile_cat = cat;
    }
    if (cat != cur_cat) {
      const CatDesc& cd = a.cats[cat];
      sh = uniform(cd.sh);
      K = uniform(cd.K);
      nc = uniform(cd.nc);
      periodic = uniform(cd.periodic);
      st_base = uniform(cd.stencil_base);
      nst = uniform(cd.nstencil);
      cell_base = uniform(cd.cell_base);
      rmin_l = cd.rmin_l;
      inv_dl = cd.inv_delta_l;
      if (lane <= nb) sT[lane] = cd.T[lane];
      cur_cat = cat;
      __syncthreads();
    }
    const double T0 = sT[0], Tn = sT[nb];

    // ---- primary
    const uint4 rp = a.rec[p];
    Primary P0;
    P0.qx = uniform(rp.x);
    P0.qy = uniform(rp.y);
    P0.qz = uniform(rp.z);
    P0.sh = sh;
    const real wp = F64 ? (real)a.w64[p] : (real)__uint_as_float(uniform(rp.w));
    const int cx = (int)(((uint64_t)(P0.qx >> sh) * (uint64_t)nc) >> K);
    const int cy = (int)(((uint64_t)(P0.qy >> sh) * (uint64_t)nc) >> K);
    const int cz = (int)(((uint64_t)(P0.qz >> sh) * (uint64_t)nc) >> K);

    if (lane < 32) {
      bcnt[lane] = 0;
      btot[lane] = 0;
      head[lane] = kEnd;
      tail[lane] = kEnd;
    }
    __syncthreads();
    int nblk = 0;
    uint32_t written = 0;  // bins whose shell already holds a stored value

    real* slot = tile + (size_t)tile_n * nb * NC;

    // ---- replay the blocks of every bin and store the shells
    auto process_blocks = [&](bool final_pass) {
      for (int b = 0; b < nb; ++b) {
        const int first = uniform((int)head[b]);
        if (first == kEnd) continue;
        static_for<0, P::NG>([&](auto G) {
          constexpr int SG = P::slots(G);
          constexpr int per = SG / 64;
          real acc[SG];
#pragma unroll
          for (int i = 0; i < SG; ++i) acc[i] = real(0);
          real hi[2] = {real(0), real(0)}, lo[2] = {real(0), real(0)};
          auto flush_acc = [&]() {
            transpose_reduce<SG>(acc, lane);
#pragma unroll
            for (int k = 0; k < per; ++k) {
              if constexpr (F64) {
                hi[k] += acc[k];
              } else {  // Kahan: hi holds the sum, lo the negated lost low part
                real yk = acc[k] - lo[k];
                real tk = hi[k] + yk;
                lo[k] = (tk - hi[k]) - yk;
                hi[k] = tk;
              }
            }
#pragma unroll
            for (int i = 0; i < SG; ++i) acc[i] = real(0);
          };
          // Software pipeline: the record of the next round and the index of the round after
          // it are in flight while the current round is evaluated.
          uint32_t j = scratch[first * kBlock + lane];
          int kn = uniform((int)nxt[first]);
          uint32_t jn = kn != kEnd ? scratch[kn * kBlock + lane] : kInvalid;
          uint4 r = a.rec[j != kInvalid ? j : p];
          double wd = (F64 && j != kInvalid) ? a.w64[j] : 0.0;
          int rounds = 0;
          for (;;) {
            uint4 rn = r;
            double wdn = 0.0;
            int knn = kEnd;
            uint32_t jnn = kInvalid;
            if (kn != kEnd) {
              rn = a.rec[jn != kInvalid ? jn : p];
              if constexpr (F64) wdn = jn != kInvalid ? a.w64[jn] : 0.0;
              knn = uniform((int)nxt[kn]);
              if (knn != kEnd) jnn = scratch[knn * kBlock + lane];
            }
            int dx, dy, dz;
            displacement(P0, r, dx, dy, dz);
            real w;
            if (j != kInvalid) {
              w = F64 ? (real)wd : (real)__uint_as_float(r.w);
            } else {
              dx = 1;
              dy = 0;
              dz = 0;
              w = real(0);
            }
            real ux, uy, uz;
            unit(dx, dy, dz, ux, uy, uz);
            add_harmonics<LMAX, F64, G>(acc, ux, uy, uz, w);
            if (++rounds == 64) {
              flush_acc();
              rounds = 0;
            }
            if (kn == kEnd) break;
            r = rn;
            wd = wdn;
            j = jn;
            jn = jnn;
            kn = knn;
          }
          if (rounds) flush_acc();
          // store this group's components of the shell (normalised)
#pragma unroll
          for (int kk = 0; kk < per; ++kk) {
            const int c = comp[G][kk];
            if (c >= 0 && c < NC) {
              real v = F64 ? hi[kk] : (hi[kk] - lo[kk]);
              v *= cs[G][kk];
              real* dst = slot + b * NC + c;
              if (written & (1u << b)) v += *dst;
              *dst = v;
            }
          }
        });
        written |= 1u << b;
      }
      if (lane < 32) {
        head[lane] = kEnd;
        tail[lane] = kEnd;
      }
      __syncthreads();
      (void)final_pass;
    };

    // Appends bucket b (64 entries, or the final partial bucket padded with kInvalid) as one
    // scratch block.
    auto emit_block = [&](int b, uint32_t n) {
      const uint32_t v = lane < (int)n ? bucket[b * kBucketCap + lane] : kInvalid;
      scratch[nblk * kBlock + lane] = v;
      const uint32_t c = bcnt[b];
      const uint32_t rem = c - n;
      const uint32_t carry = lane < (int)rem ? bucket[b * kBucketCap + n + lane] : 0u;
      __syncthreads();
      if (lane < (int)rem) bucket[b * kBucketCap + lane] = carry;
      if (lane == 0) {
        bcnt[b] = rem;
        btot[b] += n;
        nxt[nblk] = kEnd;
        if (head[b] == kEnd) head[b] = (uint16_t)nblk;
        else nxt[tail[b]] = (uint16_t)nblk;
        tail[b] = (uint16_t)nblk;
      }
      __syncthreads();
      ++nblk;
    };

    // ---- pass over the stencil
    for (int e = 0; e < nst; ++e) {
      const StencilRow row = a.stencil[st_base + e];
      const int ry = uniform(row.dy), rz = uniform(row.dz), half = uniform(row.half), full = uniform(row.full);
      int y = cy + ry, z = cz + rz;
      if (periodic) {
        y = y < 0 ? y + nc : (y >= nc ? y - nc : y);
        z = z < 0 ? z + nc : (z >= nc ? z - nc : z);
      } else if (y < 0 || y >= nc || z < 0 || z >= nc) {
        continue;
      }
      const uint32_t rowbase = cell_base + (uint32_t)((z * nc + y) * nc);
      int xa[2], xb[2], nint = 0;
      if (periodic && full) {
        xa[0] = 0;
        xb[0] = nc - 1;
        nint = 1;
      } else {
        int x0 = cx - half, x1 = cx + half;
        if (periodic) {
          if (x0 < 0) {
            xa[0] = x0 + nc; xb[0] = nc - 1; xa[1] = 0; xb[1] = x1; nint = 2;
          } else if (x1 >= nc) {
            xa[0] = x0; xb[0] = nc - 1; xa[1] = 0; xb[1] = x1 - nc; nint = 2;
          } else {
            xa[0] = x0; xb[0] = x1; nint = 1;
          }
        } else {
          xa[0] = x0 < 0 ? 0 : x0;
          xb[0] = x1 >= nc ? nc - 1 : x1;
          nint = 1;
        }
      }
      for (int s = 0; s < nint; ++s) {
        const uint32_t beg = uniform(a.cell_start[rowbase + xa[s]]);
        const uint32_t end = uniform(a.cell_start[rowbase + xb[s] + 1]);
        // Rounds of 64 candidates, with the records of up to four rounds loaded ahead.
        for (uint32_t o4 = beg; o4 < end; o4 += 4 * kBlock) {
          uint4 rr[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t j = o4 + u * kBlock + lane;
            rr[u] = a.rec[j < end ? j : beg];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t o = o4 + u * kBlock;
            if (o >= end) break;
            const uint32_t j = o + lane;
            const bool ok = j < end;
            int dx, dy, dz;
            displacement(P0, rr[u], dx, dy, dz);
            const double ddx = dx, ddy = dy, ddz = dz;
            const double R2 = fma(ddx, ddx, fma(ddy, ddy, ddz * ddz));
            if (ok && R2 > 0.0 && R2 >= T0 && R2 < Tn) {
              int bb = (int)((sqrtf((float)R2) - rmin_l) * inv_dl);
              bb = bb < 0 ? 0 : (bb >= nb ? nb - 1 : bb);
              while (R2 < sT[bb]) --bb;
              while (bb + 1 < nb && R2 >= sT[bb + 1]) ++bb;
              const uint32_t pos = atomicAdd(&bcnt[bb], 1u);
              bucket[bb * kBucketCap + pos] = j;
            }
            my_cand += (end - o < (uint32_t)kBlock) ? (end - o) : (uint32_t)kBlock;
            __syncthreads();
            uint64_t full_mask = __ballot(lane < nb && bcnt[lane] >= (uint32_t)kBlock);
            while (full_mask) {
              const int b = __ffsll((unsigned long long)full_mask) - 1;
              full_mask &= full_mask - 1;
              emit_block(b, kBlock);
              if (nblk + nb >= S) {
                process_blocks(false);
                nblk = 0;
              }
            }
          }
        }
      }
    }
    // final partial buckets
    {
      uint64_t part_mask = __ballot(lane < nb && bcnt[lane] > 0);
      while (part_mask) {
        const int b = __ffsll((unsigned long long)part_mask) - 1;
        part_mask &= part_mask - 1;
        emit_block(b, bcnt[b]);
      }
    }
    process_blocks(true);
    nblk = 0;
    // bins without any pair: zero shells
    for (int b = 0; b < nb; ++b)
      if (!(written & (1u << b)))
        for (int c = lane; c < NC; c += 64) slot[b * NC + c] = real(0);

    uint32_t pairs_p = lane < nb ? btot[lane] : 0u;
    if (a.counts && lane < nb) a.counts[(size_t)p * nb + lane] = (int32_t)pairs_p;
    for (int off = 32; off > 0; off >>= 1) pairs_p += __shfl_xor(pairs_p, off);
    my_pairs += pairs_p;
    if (a.alm_debug) {
      real* dbg = reinterpret_cast<real*>(a.alm_debug) + (size_t)p * nb * NC;
      for (int i = lane; i < nb * NC; i += 64) dbg[i] = slot[i];
    }
    if (lane == 0) swt[tile_n] = wp;
    __syncthreads();
    ++tile_n;
    if (tile_n == TP) do_contract();
  }
  do_contract();
  flush_part();
  if (lane == 0) {
    atomicAdd(&a.stats[0], my_pairs);
    atomicAdd(&a.stats[1], my_cand);
  }
}

// ------------------------------------------------------------------------------------------
// Host-side launch table.
// ------------------------------------------------------------------------------------------
typedef void (*SweepFn)(SweepArgs);

template <int LMAX, bool F64>
static void launch_one(SweepArgs args, int waves, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((sweep_kernel<LMAX, F64>), dim3(waves), dim3(64), lds, stream, args);
}

template <int LMAX, bool F64>
static hipError_t set_lds(size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&sweep_kernel<LMAX, F64>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

size_t sweep_lds_bytes(int scratch_blocks, int nb) { return (size_t)Lds::bytes(scratch_blocks, nb); }

// Doubles (FP64) or floats (mixed) of per-wave tile area, including the FP64 zeta partial.
size_t sweep_tile_bytes_per_wave(int lmax, int nb, bool f64) {
  const int NC = (lmax + 1) * (lmax + 1);
  const size_t tp = f64 ? kTileF64 : kTileF32;
  const size_t elem = f64 ? 8 : 4;
  return tp * nb * NC * elem + (size_t)(lmax + 1) * nb * nb * 8;
}

hipError_t launch_sweep(int lmax, bool f64, const SweepArgs& args, int waves, hipStream_t stream) {
  const size_t lds = sweep_lds_bytes(args.scratch_blocks, args.nb);
  hipError_t err = hipSuccess;
#define TPCF_CASE(L)                                   \
  case L:                                              \
    if (f64) {                                         \
      err = set_lds<L, true>(lds);                     \
      if (err == hipSuccess) launch_one<L, true>(args, waves, lds, stream); \
    } else {                                           \
      err = set_lds<L, false>(lds);                    \
      if (err == hipSuccess) launch_one<L, false>(args, waves, lds, stream); \
    }                                                  \
    break;
  switch (lmax) {
    TPCF_CASE(0)
    TPCF_CASE(1)
    TPCF_CASE(2)
    TPCF_CASE(3)
    TPCF_CASE(4)
    TPCF_CASE(5)
    TPCF_CASE(6)
    TPCF_CASE(7)
    TPCF_CASE(8)
    TPCF_CASE(9)
    TPCF_CASE(10)
    default:
      return hipErrorInvalidValue;
  }
#undef TPCF_CASE
  if (err != hipSuccess) return err;
  return hipGetLastError();
}

// Group plan query for the host (normalisation constants are per global component).
int plan_groups(int lmax, bool f64) { return (f64 && (lmax + 1) * (lmax + 1) > 64) ? 2 : 1; }

}  // namespace tpcf
