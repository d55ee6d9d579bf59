// sweep.hip -- the persistent pair sweep: cell-grid neighbour scan, exact radial binning,
// spherical-harmonic shells a_lm(p, b) accumulated in registers, and the bin-pair contraction
// zeta_l(b1, b2) += w_p sum_m a_lm(b1) a*_lm(b2) on MFMA, for gfx950 (wave64).
//
// Method (paper, Implementation section): for each pivot (primary), find every neighbour in
// the search range and fill the multipole bins, with Chebyshev polynomials in place of
// trigonometric functions. Here the Chebyshev polynomials are those of the polar cosine z:
// every a_lm of a bin is a fixed linear combination of the moments
//     M_{m,k} = sum_j w_j T_k(z_j) (x_j - i y_j)^m,   0 <= k <= l_max - m,
// because d^m P_l / dz^m is a polynomial of degree l - m in z. T_k costs one FMA each
// (T_k = 2 z T_{k-1} - T_{k-2}) and is shared by all m, so a pair costs about one FMA per real
// moment plus the powers of (x - i y).
//
// One wavefront owns one primary at a time; persistent waves take tasks from an atomic queue cut
// into one segment per XCD (a wave starts on its own XCD's segment and moves on when it is empty):
//   stencil : the primary's own stencil: every (y, z) row of cells whose slab comes within
//             r_max of the primary, clipped in x to the chord of the r_max sphere (cells are up
//             to four times thinner in x, so the clip is tighter). Rows are built 64 at a time,
//             one per lane; each row's cells are one contiguous run of the cell-sorted records.
//             For large neighbourhoods the rows are taken in a rotated order, phase-aligned
//             across the waves in flight (L2 sharing).
//   pass    : batches of four rounds of 64 consecutive candidates, packed across runs. Each
//             candidate's bin is decided in FP32 when its fractional bin position is farther than
//             a proven error bound from a bin edge, and otherwise exactly (FP64 squared lattice
//             separation against integer thresholds). An accepted candidate takes the next entry
//             of its bin's region in the wave's scratch (one LDS cursor increment) and stores its
//             sorted position there.
//   shells  : when a region is nearly full or the stencil is done, the wave replays bin by bin:
//             each lane adds its pair's moments into register accumulators; every <= 64 rounds
//             the 64 lanes are combined with a transpose-reduction (permlane32/16 swaps, then DPP)
//             into a compensated (Kahan) shell sum (mixed precision) or a plain FP64 sum. At the
//             end of the bin the moments are turned into normalised a_lm through LDS.
//   contract: every 32 (mixed) or 16 (FP64) primaries, the wave multiplies its tile of shells on
//             MFMA: per l, zeta_l += X_l diag(f w) X_l^T with X_l the [bins x (primaries*(2l+1))]
//             matrix of real components. Mixed: three-piece BF16 split, six products, FP32
//             accumulation within the tile. FP64: v_mfma_f64_16x16x4. Tile results are added into
//             a per-wave FP64 partial; partials are added into zeta (FP64 atomics) when the wave
//             changes catalogue and when it finishes. In the deterministic form each tile of
//             consecutive primaries writes a slot of its own instead, and a second kernel adds the
//             slots in tile order.
//
// Projected fields on the unit sphere (the paper's own geometry, Statement of need, Features and
// Performance sections) run through the same skeleton with 2D multipoles of the position angle:
// points are unit vectors shifted into a cube of side 4, bins are linear in the angle theta
// (integer thresholds on the squared chord 2 sin(theta/2)), and per pair the displacement is
// projected on a tangent basis (e1, e2) of the primary, (c, s) = unit(d.e1, d.e2), so that
//     a_m = sum_j w_j exp(-i m phi_j) = sum_j w_j (T_m(c_j) - i s_j U_(m-1)(c_j)),  0 <= m <= m_max,
// with the Chebyshev recurrence in place of trigonometric calls, as the paper does (two FMAs per
// m); zeta_m(b1, b2) = sum_p w_p Re[a_m(b1) conj(a_m(b2))].
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

// Adds (WRITE: stores) the group-G moments w T_k(z) (x - i y)^m of one pair into acc. Moment
// (m, k) occupies the register slot of component (l = m + k, m) of the plan.
template <int LMAX, bool F64, int G, bool WRITE, class real, int S>
__device__ __forceinline__ void add_moments(real (&acc)[S], real x, real y, real z, real w) {
  using P = Plan<LMAX, F64>;
  real T[LMAX + 1];
  T[0] = real(1);
  if constexpr (LMAX >= 1) T[1] = z;
  const real z2 = z + z;
  static_for<2, LMAX + 1>([&](auto K) { T[K] = z2 * T[K - 1] - T[K - 2]; });
  real pr = w, pi = real(0);  // w (x - i y)^m
  static_for<0, LMAX + 1>([&](auto M) {
    constexpr int m = M;
    if constexpr (m == 1) {  // pi is still 0
      pi = -(pr * y);
      pr = pr * x;
    } else if constexpr (m > 1) {
      real nr = pr * x + pi * y;
      real ni = pi * x - pr * y;
      pr = nr;
      pi = ni;
    }
    if constexpr (P::group_of(m) == G) {
      static_for<0, LMAX - m + 1>([&](auto Kk) {
        constexpr int k = Kk;
        if constexpr (WRITE) {
          if constexpr (k == 0) {
            acc[P::loc(m, m, 0)] = pr;
            if constexpr (m > 0) acc[P::loc(m, m, 1)] = pi;
          } else {
            acc[P::loc(m + k, m, 0)] = T[k] * pr;
            if constexpr (m > 0) acc[P::loc(m + k, m, 1)] = T[k] * pi;
          }
        } else {
          if constexpr (k == 0) {
            acc[P::loc(m, m, 0)] += pr;
            if constexpr (m > 0) acc[P::loc(m, m, 1)] += pi;
          } else {
            acc[P::loc(m + k, m, 0)] += T[k] * pr;
            if constexpr (m > 0) acc[P::loc(m + k, m, 1)] += T[k] * pi;
          }
        }
      });
    }
  });
}

// Sphere plan: component 0 is Re a_0, components 2m - 1 and 2m are Re a_m and Im a_m; one group
// of 32 reduction slots (2 m_max + 1 <= 21 are used).
template <int M>
struct PlanSph {
  static constexpr int NC = 2 * M + 1;
  static constexpr int NG = 1;
  static constexpr int slots(int) { return 32; }
  static constexpr int gsize(int) { return NC; }
  __host__ __device__ static constexpr int global_of(int, int s) { return s < NC ? s : -1; }
};

// Adds (WRITE: stores) w exp(-i m phi) = w (cos m phi - i sin m phi), m = 0..M, of one pair into
// acc, from (c, s) = (cos phi, sin phi) with the Chebyshev recurrence the paper uses in place of
// trigonometric calls: A_m = w T_m(c) = w cos m phi and B_m = w s U_(m-1)(c) = w sin m phi both
// obey X_m = 2c X_(m-1) - X_(m-2), so each m costs two FMAs and two adds.
template <int M, bool WRITE, class real, int S>
__device__ __forceinline__ void add_moments_sph(real (&acc)[S], real c, real s, real w) {
  auto put = [&](int k, real v) {
    if constexpr (WRITE) acc[k] = v;
    else acc[k] += v;
  };
  auto put_neg = [&](int k, real v) {
    if constexpr (WRITE) acc[k] = -v;
    else acc[k] -= v;
  };
  put(0, w);
  if constexpr (M >= 1) {
    const real c2 = c + c;
    real Ap = w, A = w * c;         // A_0, A_1
    real Bp = real(0), B = w * s;   // B_0, B_1
    put(1, A);
    put_neg(2, B);
    static_for<2, M + 1>([&](auto Mi) {
      constexpr int m = Mi;
      const real An = c2 * A - Ap;
      const real Bn = c2 * B - Bp;
      Ap = A;
      A = An;
      Bp = B;
      B = Bn;
      put(2 * m - 1, A);
      put_neg(2 * m, B);
    });
  }
}

// ------------------------------------------------------------------------------------------
// Cross-lane transpose-reduction. Input: S values per lane (S = 32, 64 or 128). Output: slot k of
// lane L (k < S/64) holds the wave-wide sum of component (S/64)*L + k; for S = 32, slot 0 of
// lanes 2c and 2c + 1 both hold the sum of component c.
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
  if constexpr (S >= 64) {
    static_for<0, S / 64>([&](auto k) { v[k] = dpp_pair<kQuadXor1>(v[k], v[k + S / 64], b0); });
  } else {
    // the stages so far summed over the 32 lanes of equal (bit 2 xor bit 0); the neighbour
    // (lane bit 0 flipped) holds the other half of the same component
    v[0] = v[0] + dpp<kQuadXor1>(v[0]);
  }
}

// ------------------------------------------------------------------------------------------
// Pair geometry.
// ------------------------------------------------------------------------------------------
struct Primary {
  uint32_t qx, qy, qz;  // stored lattice coordinates (shifted)
  int sh;
};

// Stored-coordinate difference of a secondary and the primary: the lattice displacement times
// 2^sh. Stored coordinates wrap modulo 2^32, so when periodic the signed difference is the
// minimum image; an arithmetic shift by sh gives the lattice displacement itself.
__device__ __forceinline__ int sdiff(uint32_t a, uint32_t b) { return (int)(a - b); }

// Unit vector of a secondary's displacement, from the scaled difference (the scale cancels).
// The tiny addend keeps the zero-weight sentinel record finite when it sits on the primary;
// it cannot change the squared length of a real pair (>= 1 in lattice units).
template <class Rec>
__device__ __forceinline__ void unit(const Primary& P, Rec r, float& x, float& y, float& z) {
  const float fx = (float)sdiff(r.x, P.qx), fy = (float)sdiff(r.y, P.qy), fz = (float)sdiff(r.z, P.qz);
  const float r2 = __builtin_fmaf(fx, fx, __builtin_fmaf(fy, fy, __builtin_fmaf(fz, fz, 0x1p-100f)));
  const float ri = __builtin_amdgcn_rsqf(r2);
  x = fx * ri;
  y = fy * ri;
  z = fz * ri;
}
template <class Rec>
__device__ __forceinline__ void unit(const Primary& P, Rec r, double& x, double& y, double& z) {
  const double fx = (double)sdiff(r.x, P.qx), fy = (double)sdiff(r.y, P.qy), fz = (double)sdiff(r.z, P.qz);
  const double r2 = fma(fx, fx, fma(fy, fy, fma(fz, fz, 0x1p-100)));
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

// Tangent basis at a primary on the sphere: n = unit(q s - 2) from its lattice position (s = 1 /
// scale), e1 = unit(z x n) (unit(x x n) within 1e-6 of the poles), e2 = n x e1. zeta_m does not
// depend on the choice: turning the basis by alpha multiplies every a_m of the primary by
// exp(i m alpha).
template <class real>
struct Tangent {
  real e1x, e1y, e1z, e2x, e2y, e2z;
};

// Orders LDS accesses between the lanes of the wavefront: a workgroup is one wavefront, whose LDS
// operations complete in issue order, so only the compiler must not move accesses across this
// point (no wait on outstanding global memory operations, unlike a workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float uniform_f(float v) {
  return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}

__device__ __forceinline__ double uniform_d(double v) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

template <class real>
__device__ __forceinline__ Tangent<real> tangent_basis(uint32_t ux, uint32_t uy, uint32_t uz, double inv_scale) {
  double nx = (double)ux * inv_scale - 2.0, ny = (double)uy * inv_scale - 2.0, nz = (double)uz * inv_scale - 2.0;
  const double nn = sqrt(nx * nx + ny * ny + nz * nz);
  nx /= nn;
  ny /= nn;
  nz /= nn;
  double ax = -ny, ay = nx, az = 0.0;
  double l1 = sqrt(ax * ax + ay * ay);
  if (l1 < 1e-6) {
    ax = 0.0;
    ay = -nz;
    az = ny;
    l1 = sqrt(ay * ay + az * az);
  }
  ax /= l1;
  ay /= l1;
  az /= l1;
  Tangent<real> t;
  t.e1x = (real)uniform_d(ax);
  t.e1y = (real)uniform_d(ay);
  t.e1z = (real)uniform_d(az);
  t.e2x = (real)uniform_d(ny * az - nz * ay);
  t.e2y = (real)uniform_d(nz * ax - nx * az);
  t.e2z = (real)uniform_d(nx * ay - ny * ax);
  return t;
}

// Position angle of a secondary around the primary as (c, s) = (cos phi, sin phi): the lattice
// displacement projected on the tangent basis, normalised.
template <class Rec>
__device__ __forceinline__ void unit_sph(const Primary& P, const Tangent<float>& tb, Rec r, float& c, float& s) {
  const float fx = (float)sdiff(r.x, P.qx), fy = (float)sdiff(r.y, P.qy), fz = (float)sdiff(r.z, P.qz);
  const float t1 = __builtin_fmaf(fx, tb.e1x, __builtin_fmaf(fy, tb.e1y, fz * tb.e1z));
  const float t2 = __builtin_fmaf(fx, tb.e2x, __builtin_fmaf(fy, tb.e2y, fz * tb.e2z));
  const float r2 = __builtin_fmaf(t1, t1, __builtin_fmaf(t2, t2, 0x1p-100f));
  const float ri = __builtin_amdgcn_rsqf(r2);
  c = t1 * ri;
  s = t2 * ri;
}
template <class Rec>
__device__ __forceinline__ void unit_sph(const Primary& P, const Tangent<double>& tb, Rec r, double& c, double& s) {
  const double fx = (double)sdiff(r.x, P.qx), fy = (double)sdiff(r.y, P.qy), fz = (double)sdiff(r.z, P.qz);
  const double t1 = fma(fx, tb.e1x, fma(fy, tb.e1y, fz * tb.e1z));
  const double t2 = fma(fx, tb.e2x, fma(fy, tb.e2y, fz * tb.e2z));
  const double r2 = fma(t1, t1, fma(t2, t2, 0x1p-100));
  double ri = __builtin_amdgcn_rsq(r2);
  double h = r2 * ri;
  ri = fma(ri * 0.5, fma(-h, ri, 1.0), ri);
  h = r2 * ri;
  ri = fma(ri * 0.5, fma(-h, ri, 1.0), ri);
  c = t1 * ri;
  s = t2 * ri;
}

// Direction of a pair and its moments, for either geometry (3D: unit vector; sphere: (c, s)).
template <bool SPH, class real, class Rec>
__device__ __forceinline__ void direction(const Primary& P, const Tangent<real>& tb, Rec r, real& x, real& y,
                                          real& z) {
  if constexpr (SPH) {
    unit_sph(P, tb, r, x, y);
    z = real(0);
  } else {
    unit(P, r, x, y, z);
  }
}
template <int LMAX, bool F64, bool SPH, int G, bool WRITE, class real, int S>
__device__ __forceinline__ void accumulate(real (&acc)[S], real x, real y, real z, real w) {
  if constexpr (SPH) add_moments_sph<LMAX, WRITE>(acc, x, y, w);
  else add_moments<LMAX, F64, G, WRITE>(acc, x, y, z, w);
}

// Arcsine of x in [0, 1] in FP32 for the fast angular bin decision: the Taylor series about 0,
// asin y = sum_n c_n y^(2n+1), c_0 = 1, c_n = c_(n-1) (2n-1)^2 / (2n (2n+1)), through n = 10 for
// y <= 1/2 (truncation below 2^-28 relative), and asin x = pi/2 - 2 asin(sqrt((1 - x) / 2)) above
// 1/2. Relative error below 16 * 2^-24 for exact x (rounding of the Horner steps, the square root
// and the final subtraction).
__device__ __forceinline__ float asin01(float x) {
  const bool up = x > 0.5f;
  const float y = up ? __builtin_amdgcn_sqrtf((1.0f - x) * 0.5f) : x;
  const float y2 = y * y;
  float p = 8.390335810e-03f;
  p = __builtin_fmaf(p, y2, 9.761609529e-03f);
  p = __builtin_fmaf(p, y2, 1.155180090e-02f);
  p = __builtin_fmaf(p, y2, 1.396484375e-02f);
  p = __builtin_fmaf(p, y2, 1.735276442e-02f);
  p = __builtin_fmaf(p, y2, 2.237215909e-02f);
  p = __builtin_fmaf(p, y2, 3.038194444e-02f);
  p = __builtin_fmaf(p, y2, 4.464285714e-02f);
  p = __builtin_fmaf(p, y2, 7.500000000e-02f);
  p = __builtin_fmaf(p, y2, 1.666666667e-01f);
  const float a = __builtin_fmaf(y * y2, p, y);
  return up ? __builtin_fmaf(-2.0f, a, 1.5707963268f) : a;
}

// The same series through n = 2 (x + x^3/6 + 3 x^5/40), for x <= 0.06: the truncation is below
// c_3 x^6 / (1 - x^2) < 2.1e-9 (about 2^-28.8) relative.
__device__ __forceinline__ float asin_small(float x) {
  const float x2 = x * x;
  return __builtin_fmaf(x * x2, __builtin_fmaf(x2, 7.500000000e-02f, 1.666666667e-01f), x);
}

// ------------------------------------------------------------------------------------------
// Contraction of one tile of shells on MFMA.
// tile: [TP][nb][NC] normalised a_lm (real components), wt: [TP] weights in LDS, nt valid
// primaries. Adds zeta_l(b1, b2) of the tile into part[(l*nb + b1)*nb + b2] (FP64, per wave).
// 3D: the 2l+1 components of l start at l*l; components m != 0 stand for +m and -m (factor 2).
// Sphere: the components of m start at 0 (m = 0, Re only) or 2m - 1 (Re, Im), factor 1.
// ------------------------------------------------------------------------------------------
template <bool SPH>
__device__ __forceinline__ int comp_base(int l) { return SPH ? (l == 0 ? 0 : 2 * l - 1) : l * l; }
template <bool SPH>
__device__ __forceinline__ int comp_count(int l) { return SPH ? (l == 0 ? 1 : 2) : 2 * l + 1; }
template <bool SPH, class real>
__device__ __forceinline__ real comp_factor(int cc) { return (SPH || cc == 0) ? real(1) : real(2); }

template <int LMAX, bool SPH>
__device__ __noinline__ void contract_tile(const float* __restrict__ tile, const float* wt, int nt,
                                           int nb, double* __restrict__ part, int lane) {
  constexpr int NC = ncomp(LMAX, SPH);
  const int b = lane & 31;
  const int kh = (lane >> 5) * 8;
  const bool brow = b < nb;
#pragma unroll 1
  for (int l = 0; l <= LMAX; ++l) {
    const int n2 = comp_count<SPH>(l);
    const int lb = comp_base<SPH>(l);
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
          xv = tile[(t * nb + b) * NC + lb + cc];
          wv = wt[t] * comp_factor<SPH, float>(cc);
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

template <int LMAX, bool SPH>
__device__ __noinline__ void contract_tile(const double* __restrict__ tile, const double* wt, int nt,
                                           int nb, double* __restrict__ part, int lane) {
  constexpr int NC = ncomp(LMAX, SPH);
  const int rl = lane & 15;
  const int kq = lane >> 4;
  const bool two = nb > 16;
#pragma unroll 1
  for (int l = 0; l <= LMAX; ++l) {
    const int n2 = comp_count<SPH>(l);
    const int lb = comp_base<SPH>(l);
    const int K = nt * n2;
    doublex4 acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
    int t = kq / n2, cc = kq - (kq / n2) * n2;  // (primary, component) of k = k0 + kq
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + kq;
      double x0 = 0.0, x1 = 0.0, y0 = 0.0, y1 = 0.0;
      if (k < K) {
        const double wf = wt[t] * comp_factor<SPH, double>(cc);
        const double* src = tile + (size_t)t * nb * NC + lb + cc;
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

template <class T>
__device__ __forceinline__ T uniform(T v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// LDS layout (bytes), one wavefront per workgroup.
struct Lds {
  static constexpr int T = 0;                    // double[kMaxBins + 1] thresholds
  static constexpr int WT = 272;                 // real[<= 64] tile weights (256 bytes)
  static constexpr int BTOT = WT + 256;          // uint32[32] pairs per bin (this primary)
  static constexpr int BBLK = BTOT + 128;        // uint32[32] filled scratch blocks per bin
  static constexpr int REG = BBLK + 128;         // uint32[33] scratch region start per bin (blocks)
  static constexpr int MOM = REG + 144;          // real[128] moments of one bin
  static constexpr int RUNS = MOM + 1024;        // uint2[128] non-empty runs of one row chunk
  static constexpr int CUR = RUNS + 1024;        // uint64[kMaxBins]: bin cursors
  static constexpr int PARK = CUR + 8 * kMaxBins;  // uint4[kBatch][64] records, uint32[kBatch][64] ids
  static constexpr int END = PARK + kBatch * 64 * 20;
  // 3D only: the moment -> a_lm conversion spread over the lanes, real coef[kConvTerms][64] then
  // int16 meta[kConvTerms][64]
  static constexpr int CONV = END;
  static __host__ __device__ constexpr int conv_bytes(int lmax, bool f64, bool sph) {
    return sph ? 0 : ((kConvTerms * 64 * ((f64 ? 8 : 4) + 2) + 15) & ~15) + 0 * lmax;
  }
  static __host__ __device__ constexpr int bytes(int lmax, bool f64, bool sph) {
    return END + conv_bytes(lmax, f64, sph);
  }
};

// One row of the per-primary stencil: up to two runs [b, e) of sorted positions.
struct Row {
  uint32_t b0, e0, b1, e1;
};

// Wave-uniform catalogue parameters.
struct CatU {
  int sh, K, nc, nx, periodic, row_lo, row_w;
  uint32_t cell_base;
  float cs, inv_cs, inv_csx, span, inv_span, reach, margin, inv_dl, u0, eps, one_me, inv_w, hinv;
  int asin_small;
};

// Builds row t of the primary's stencil (rows are offsets (dy, dz) from the primary's cell):
// the x cells (nx per row, thinner than the y-z cells) whose slab intersects the chord of the
// r_max sphere through that row.
__device__ __forceinline__ Row make_row(const uint32_t* __restrict__ cell_start, const CatU& c, int t, int cx,
                                        int cy, int cz, float qx, float qy, float qz) {
  Row r = {0u, 0u, 0u, 0u};
  const int W = c.row_w;
  if (t >= W * W) return r;
  const int tz = (int)(((float)t + 0.5f) * c.inv_w);
  const int ty = t - tz * W;
  const int y = cy + c.row_lo + ty, z = cz + c.row_lo + tz;
  const int nc = c.nc;
  float dyf, dzf;
  int yw = y, zw = z;
  if (c.periodic) {
    float oy = ((float)y + 0.5f) * c.cs - qy;
    float oz = ((float)z + 0.5f) * c.cs - qz;
    oy -= c.span * rintf(oy * c.inv_span);
    oz -= c.span * rintf(oz * c.inv_span);
    dyf = fmaxf(fabsf(oy) - 0.5f * c.cs, 0.f);
    dzf = fmaxf(fabsf(oz) - 0.5f * c.cs, 0.f);
    yw = y % nc;
    yw += yw < 0 ? nc : 0;
    zw = z % nc;
    zw += zw < 0 ? nc : 0;
  } else {
    if (y < 0 || y >= nc || z < 0 || z >= nc) return r;
    dyf = fmaxf(fmaxf((float)y * c.cs - qy, qy - (float)(y + 1) * c.cs), 0.f);
    dzf = fmaxf(fmaxf((float)z * c.cs - qz, qz - (float)(z + 1) * c.cs), 0.f);
  }
  const float rr = c.reach * c.reach;
  const float d2 = dyf * dyf + dzf * dzf;
  if (d2 >= rr) return r;
  const float h = __builtin_amdgcn_sqrtf(rr - d2) + c.margin;
  const int nx = c.nx;
  const int xa = (int)floorf((qx - h) * c.inv_csx);
  const int xb = (int)floorf((qx + h) * c.inv_csx);
  const uint32_t rowbase = c.cell_base + (uint32_t)((zw * nc + yw) * nx);
  int a0, b0, a1 = 0, b1 = -1;
  if (c.periodic) {
    if (xb - xa + 1 >= nx) {
      a0 = 0;
      b0 = nx - 1;
    } else {
      int aw = xa % nx;
      aw += aw < 0 ? nx : 0;
      const int bw = aw + (xb - xa);
      a0 = aw;
      if (bw < nx) {
        b0 = bw;
      } else {
        b0 = nx - 1;
        b1 = bw - nx;
      }
    }
  } else {
    a0 = xa < 0 ? 0 : xa;
    b0 = xb > nx - 1 ? nx - 1 : xb;
    if (a0 > b0) return r;
  }
  r.b0 = cell_start[rowbase + a0];
  r.e0 = cell_start[rowbase + b0 + 1];
  if (b1 >= a1) {
    r.b1 = cell_start[rowbase + a1];
    r.e1 = cell_start[rowbase + b1 + 1];
  }
  return r;
}

// Compiler-only ordering point for LDS data exchanged between lanes of the one wavefront of a
// workgroup: the hardware executes a wavefront's LDS instructions in order.
__device__ __forceinline__ void lds_order() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// Inclusive prefix sum over the 64 lanes of the wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(v, (unsigned)d);
    if (lane >= d) v += u;
  }
  return v;
}

__device__ __forceinline__ uint32_t row_len(const Row& r) { return (r.e0 - r.b0) + (r.e1 - r.b1); }

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Waves per SIMD the register allocation targets: three for the FP32 sweeps (the mixed 3D shells
// fit in 168 VGPRs while the pass state is parked in LDS during the replay), two for FP64.
template <bool F64>
constexpr int kSweepWaves = F64 ? 2 : 3;

// DET: deterministic form. Tickets hand out whole tiles of consecutive tasks (a tile never spans
// two catalogues), each tile's contraction and 2PCF weight sums go to the tile's own slot of
// a.det_out, and a second kernel adds the slots in tile order; with every primary's shells fixed
// by its stencil order, the result no longer depends on scheduling.
template <int LMAX, bool F64, bool SPH, bool DET>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kSweepWaves<F64>))) void sweep_kernel(SweepArgs a) {
  using real = std::conditional_t<F64, double, float>;
  using P = std::conditional_t<SPH, PlanSph<LMAX>, Plan<LMAX, F64>>;
  constexpr int NC = P::NC;
  constexpr int TP = tile_primaries(F64, SPH);

  extern __shared__ __align__(16) unsigned char smem[];
  double* sT = reinterpret_cast<double*>(smem + Lds::T);
  real* swt = reinterpret_cast<real*>(smem + Lds::WT);
  uint32_t* btot = reinterpret_cast<uint32_t*>(smem + Lds::BTOT);
  uint32_t* bblk = reinterpret_cast<uint32_t*>(smem + Lds::BBLK);
  uint32_t* reg = reinterpret_cast<uint32_t*>(smem + Lds::REG);
  real* mom = reinterpret_cast<real*>(smem + Lds::MOM);
  uint2* runs = reinterpret_cast<uint2*>(smem + Lds::RUNS);
  unsigned long long* cur = reinterpret_cast<unsigned long long*>(smem + Lds::CUR);
  real* scoef = reinterpret_cast<real*>(smem + Lds::CONV);
  int16_t* smeta = reinterpret_cast<int16_t*>(smem + Lds::CONV + kConvTerms * 64 * sizeof(real));

  const int lane = threadIdx.x;
  // The conversion table stays in LDS for the whole sweep (the epilogue of every bin reads it).
  if constexpr (!SPH) {
    for (int i = lane; i < a.conv_q * 64; i += 64) {
      smeta[i] = a.conv_idx[i];
      scoef[i] = F64 ? (real)a.conv_coef64[i] : (real)a.conv_coef32[i];
    }
  }
  const int nb = a.nb;
  const int S = a.scratch_blocks;
  const uint32_t wave = blockIdx.x;
  uint32_t* scratch = a.scratch + (size_t)wave * (S + kScratchTail) * kBlock;
  // Scratch accesses as a wave-uniform address plus a 32-bit byte offset per lane (a wave's
  // scratch is far below 4 GiB), which the loads and stores take in their scalar-base form:
  // no 64-bit address arithmetic on the VALU.
  uint32_t lane4 = (uint32_t)lane * 4u;
  auto entry = [&](const uint32_t* blk) -> uint32_t {  // this lane's entry of a block
    asm volatile("" : "+v"(lane4));  // keeps the per-lane part apart from the uniform address
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(blk) + lane4);
  };
  auto put = [&](uint32_t k, uint32_t v) {  // entry k of the wave's scratch
    *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(scratch) + (k << 2)) = v;
  };
  real* tile = reinterpret_cast<real*>(a.tile) + (size_t)wave * (TP * nb * NC + (LMAX + 1) * nb * nb * (F64 ? 1 : 2));
  double* part = reinterpret_cast<double*>(tile + TP * nb * NC);
  // DET: slot of the current tile, [(LMAX+1) nb nb] zeta then [nb] weight sums
  const size_t det_stride = (size_t)(LMAX + 1) * nb * nb + nb;

  // Scratch regions: bin b owns blocks [reg[b], reg[b+1]).
  if (lane <= nb) reg[lane] = a.regions[lane];

  // Moment index held by each of this lane's reduction slots, per group (32 slots: the even
  // lane of each pair writes).
  int mslot[P::NG][2];
  static_for<0, P::NG>([&](auto G) {
    constexpr int SG = P::slots(G);
    constexpr int per = SG >= 64 ? SG / 64 : 1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      int ms = -1;
      if (k < per) ms = SG >= 64 ? P::global_of(G, per * lane + k) : ((lane & 1) ? -1 : P::global_of(G, lane >> 1));
      mslot[G][k] = ms;
    }
  });

  for (int i = lane; i < (LMAX + 1) * nb * nb; i += 64) part[i] = 0.0;

  int tile_n = 0, tile_cat = -1, part_cat = -1, cur_cat = -1;
  unsigned long long my_pairs = 0, my_cand = 0;
  // Two-point by-product, per wave (lane b < nb: bin b) for catalogue bins_cat: ordered pairs
  // and sum of w_p w_j. sdd (lane b): sum of w_j of bin b for the current primary.
  unsigned long long bins_np = 0;
  double bins_dd = 0.0, sdd = 0.0;
  int bins_cat = -1;
  auto flush_bins = [&]() {
    if (bins_cat >= 0 && lane < nb) {
      if (bins_np) atomicAdd(&a.bin_pairs[(size_t)bins_cat * nb + lane], bins_np);
      if (!DET && bins_dd != 0.0) atomicAdd(&a.bin_dd[(size_t)bins_cat * nb + lane], bins_dd);
    }
    bins_np = 0;
    bins_dd = 0.0;
  };
  CatU cu = {};

  auto flush_part = [&]() {
    if (!DET && part_cat >= 0) {
      double* zt = a.zeta + (size_t)part_cat * (LMAX + 1) * nb * nb;
      for (int i = lane; i < (LMAX + 1) * nb * nb; i += 64) {
        const double v = part[i];
        if (v != 0.0) atomicAdd(&zt[i], v);
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
    contract_tile<LMAX, SPH>(tile, swt, tile_n, nb, part, lane);
    __syncthreads();
    tile_n = 0;
  };

  // XCD-aware tickets: the task list is cut into kQueueSegments contiguous segments, one counter
  // each. Workgroups are dispatched round-robin over the 8 XCDs, so wave w starts on segment
  // w mod 8, the one of its own XCD: each XCD's L2 then serves a compact run of primaries rather
  // than every eighth one. A wave moves on to the next segment when its own is exhausted and
  // leaves after it has found all of them exhausted.
  int seg = (int)(blockIdx.x % (uint32_t)kQueueSegments), seg_left = kQueueSegments;
  const uint32_t seg_waves = max(1u, gridDim.x / (uint32_t)kQueueSegments);  // waves in flight per segment
  uint32_t j = 0;  // ticket within its segment
  // Next ticket of [0, n): segment base + j; false once every segment is exhausted.
  auto next_ticket = [&](uint32_t n, uint32_t& ticket) -> bool {
    for (;;) {
      const uint32_t lo = (uint32_t)((uint64_t)n * (uint32_t)seg / kQueueSegments);
      const uint32_t hi = (uint32_t)((uint64_t)n * (uint32_t)(seg + 1) / kQueueSegments);
      uint32_t jj = 0;
      if (lane == 0) jj = atomicAdd(a.queue + seg, 1u);
      j = uniform(jj);
      if (j < hi - lo) {
        ticket = lo + j;
        return true;
      }
      if (--seg_left == 0) return false;
      seg = (seg + 1) % kQueueSegments;
    }
  };
  uint32_t det_t = 0, det_end = 0;
  // DET: closes the current tile (contraction into its slot, weight sums) and opens the next.
  auto det_next_tile = [&]() -> bool {
    do_contract();
    if (det_end > 0 && lane < nb) part[(size_t)(LMAX + 1) * nb * nb + lane] = bins_dd;
    bins_dd = 0.0;
    uint32_t tk;
    if (!next_ticket(a.ndet, tk)) return false;
    const uint2 tr = a.det_tiles[tk];
    det_t = uniform(tr.x);
    det_end = uniform(tr.y);
    part = a.det_out + (size_t)tk * det_stride;
    for (size_t i = lane; i < det_stride; i += 64) part[i] = 0.0;
    __syncthreads();
    return true;
  };
  for (;;) {
    uint32_t t;
    if constexpr (DET) {
      if (det_t == det_end && !det_next_tile()) break;
      t = det_t++;
    } else {
      if (!next_ticket(a.ntask, t)) break;
    }
    const uint32_t p = uniform(a.task_list ? a.task_list[t] : t);
    const int cat = uniform(a.prim_cat_start ? range_of([&](int k) { return a.prim_cat_start[k]; }, a.ncat, p)
                                             : catalogue_of(a.cats, a.ncat, p));
    if (cat != tile_cat) {
      do_contract();
      tile_cat = cat;
    }
    if (cat != cur_cat) {
      const CatDesc& cd = a.cats[cat];
      cu.sh = uniform(cd.sh);
      cu.K = uniform(cd.K);
      cu.nc = uniform(cd.nc);
      cu.nx = uniform(cd.nx);
      cu.periodic = uniform(cd.periodic);
      cu.row_lo = uniform(cd.row_lo);
      cu.row_w = uniform(cd.row_w);
      cu.cell_base = uniform(cd.cell_base);
      // wave-uniform values live in scalar registers
      cu.cs = uniform_f(cd.cs);
      cu.inv_cs = uniform_f(cd.inv_cs);
      cu.inv_csx = uniform_f(cd.inv_csx);
      cu.span = uniform_f(cd.span);
      cu.inv_span = uniform_f(1.0f / cd.span);
      cu.reach = uniform_f(cd.reach);
      cu.margin = uniform_f(cd.margin);
      cu.inv_dl = uniform_f(cd.inv_delta_l);
      cu.u0 = uniform_f(cd.u0);
      cu.eps = uniform_f(cd.eps);
      cu.one_me = uniform_f(cd.one_minus_eps);
      cu.inv_w = uniform_f(1.0f / (float)cu.row_w);
      cu.hinv = uniform_f(cd.half_inv_scale);
      cu.asin_small = uniform(cd.asin_small);
      if (lane <= nb) sT[lane] = cd.T[lane];
      cur_cat = cat;
      __syncthreads();
    }
    const double T0 = sT[0], Tn = sT[nb];

    // ---- primary (a point, or a shared pivot)
    const uint4 rp = a.prim_rec ? a.prim_rec[p] : a.rec[p];
    Primary P0;
    P0.qx = uniform(rp.x);
    P0.qy = uniform(rp.y);
    P0.qz = uniform(rp.z);
    P0.sh = cu.sh;
    const real wp = F64 ? (real)(a.prim_rec ? a.prim_w64[p] : a.w64[p]) : (real)__uint_as_float(uniform(rp.w));
    const uint32_t ux = P0.qx >> cu.sh, uy = P0.qy >> cu.sh, uz = P0.qz >> cu.sh;
    const int cx = (int)(((uint64_t)ux * (uint64_t)cu.nc) >> cu.K);
    const int cy = (int)(((uint64_t)uy * (uint64_t)cu.nc) >> cu.K);
    const int cz = (int)(((uint64_t)uz * (uint64_t)cu.nc) >> cu.K);
    const float qxf = (float)ux, qyf = (float)uy, qzf = (float)uz;
    Tangent<real> tb = {};
    if constexpr (SPH) tb = tangent_basis<real>(ux, uy, uz, 2.0 * (double)cu.hinv);

    // Bin cursors: low word = next free entry of the bin's region, high word = its soft limit.
    auto reset_cursors = [&]() {
      if (lane < nb) {
        const uint32_t r0 = reg[lane], r1 = reg[lane + 1];
        cur[lane] = (unsigned long long)(r0 * kBlock) |
                    ((unsigned long long)(r1 * kBlock - kSoftReserve) << 32);
      }
      lds_order();
    };
    if (lane < 32) {
      btot[lane] = 0;
      bblk[lane] = 0;
    }
    reset_cursors();
    uint32_t written = 0;  // bins whose shell already holds a stored value
    real* slot = tile + (size_t)tile_n * nb * NC;

    // ---- stencil generator. Rows are built 64 at a time (one per lane) and their non-empty
    // runs compacted into LDS; runs are taken 64 at a time into a sub-chunk held in registers
    // (lane r: first candidate position of run r and the offset from candidate position to
    // sorted position). Rounds are 64 consecutive candidate positions of the sub-chunk.
    const int nrows = cu.row_w * cu.row_w;
    int row_base = 0;      // first row of the next row chunk
    int nrun = 0;          // runs of the current row chunk
    int run_next = 0;      // first run of the row chunk not yet taken into a sub-chunk
    uint32_t sub_T = 0;    // candidates of the sub-chunk
    uint32_t o = 0;        // next candidate position
    uint32_t delta_c = 0;  // sorted minus candidate position for the run holding position o - 1
    uint32_t pre_v = kInvalid, dl_v = 0;

    // Phase alignment: start at the row holding candidate floor(total * phase), phase = (ticket
    // within the segment mod the segment's waves) / those waves, and wrap around. Tickets are
    // handed out at a steady rate, so a wave's phase is where the waves in flight on its segment
    // are in their own stencils when it starts, and all of them keep reading about the same rows
    // (shared through L2) instead of the whole neighbourhood. Rows are counted in chunks of 64 (at
    // most 64 chunks: lane k keeps chunk k's candidates).
    int rot = 0;
    if (!DET && a.phase_rows && nrows <= 64 * 64) {
      const int nchunk = (nrows + 63) >> 6;
      uint32_t ctot = 0, total = 0;
      for (int k = 0; k < nchunk; ++k) {
        const Row rw = make_row(a.cell_start, cu, k * 64 + lane, cx, cy, cz, qxf, qyf, qzf);
        const uint32_t sk = uniform(__builtin_amdgcn_readlane(wave_incl_scan(row_len(rw), lane), 63));
        if (lane == k) ctot = sk;
        total += sk;
      }
      const uint32_t target = (uint32_t)((uint64_t)total * (j % seg_waves) / seg_waves);  // < total if total > 0
      const uint32_t incl = wave_incl_scan(ctot, lane);
      // chunk holding the target: lanes at or past nchunk have incl == total > target
      const int k = __popcll(__ballot(incl <= target));
      if (k < nchunk) {
        const uint32_t before = uniform(__builtin_amdgcn_readlane(incl - ctot, k));
        const Row rw = make_row(a.cell_start, cu, k * 64 + lane, cx, cy, cz, qxf, qyf, qzf);
        const uint32_t li = wave_incl_scan(row_len(rw), lane);
        const int r = k * 64 + __popcll(__ballot(before + li <= target));
        rot = r < nrows ? r : 0;
      }
    }

    auto build_rows = [&]() {
      int tr = row_base + lane;  // rows past nrows stay past it (empty)
      if (tr < nrows) {
        tr += rot;
        if (tr >= nrows) tr -= nrows;
      }
      const Row rw = make_row(a.cell_start, cu, tr, cx, cy, cz, qxf, qyf, qzf);
      const bool h0 = rw.e0 > rw.b0, h1 = rw.e1 > rw.b1;
      const uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
      const int below = lanes_below(m0) + lanes_below(m1);
      if (h0) runs[below] = make_uint2(rw.b0, rw.e0);
      if (h1) runs[below + (h0 ? 1 : 0)] = make_uint2(rw.b1, rw.e1);
      lds_order();
      nrun = __popcll(m0) + __popcll(m1);
      run_next = 0;
      row_base += 64;
    };
    auto load_sub = [&]() {
      const int cnt = min(64, nrun - run_next);
      uint2 rr = make_uint2(0u, 0u);
      if (lane < cnt) rr = runs[run_next + lane];
      const uint32_t len = rr.y - rr.x;
      uint32_t incl = len;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(incl, (unsigned)d);
        if (lane >= d) incl += v;
      }
      const uint32_t pre = incl - len;
      pre_v = lane < cnt ? pre : kInvalid;
      dl_v = rr.x - pre;
      sub_T = uniform(__builtin_amdgcn_readlane(incl, 63));
      my_cand += sub_T;  // the batches of the sub-chunk cover its candidates once
      run_next += cnt;
      o = 0;
      lds_order();
    };
    // Next batch: up to kBatch rounds from the current sub-chunk. Lane k of round u gets the sorted
    // position of candidate o + 64 u + k, or past the sub-chunk's end the index of the sentinel
    // record (never a candidate, so every lane loads a valid record). A batch never spans two
    // sub-chunks, so the run offsets of all its rounds come from one window of run starts (the
    // last batch of a sub-chunk may hold empty rounds). Returns false once the stencil is done.
    auto gen_batch = [&](uint32_t(&id)[kBatch]) -> bool {
      while (o >= sub_T) {
        if (run_next >= nrun) {
          if (row_base >= nrows) {
#pragma unroll
            for (int u = 0; u < kBatch; ++u) id[u] = a.sentinel;
            return false;
          }
          build_rows();
        } else {
          load_sub();
        }
      }
      constexpr uint32_t span = kBatch * kBlock;
      uint32_t g[kBatch], delta[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        g[u] = o + (uint32_t)(u * kBlock + lane);
        delta[u] = delta_c;
      }
      uint64_t starts = __ballot(pre_v >= o && pre_v < o + span);
      while (starts) {
        const int r = __ffsll((unsigned long long)starts) - 1;
        starts &= starts - 1;
        const uint32_t ps = uniform(__builtin_amdgcn_readlane(pre_v, r));
        const uint32_t ds = uniform(__builtin_amdgcn_readlane(dl_v, r));
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
          if (g[u] >= ps) delta[u] = ds;
        delta_c = ds;
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) id[u] = g[u] < sub_T ? g[u] + delta[u] : a.sentinel;
      o += span;
      return true;
    };
    auto load_batch = [&](const uint32_t(&id)[kBatch], uint4(&rc)[kBatch]) {
#pragma unroll
      for (int u = 0; u < kBatch; ++u) rc[u] = a.rec[id[u]];
    };

    // ---- shells: replay every bin's blocks (one copy of this code)
    auto process_blocks = [&]() {
      // Look-ahead across bins (the FP32 sphere replay, whose bins hold few short rounds): the
      // first four entries of the next non-empty bin are requested when a bin's replay starts,
      // and its first two records when that replay ends, so that a bin's first rounds do not wait
      // on two dependent loads. (The FP64 sphere kernel would need more VGPRs than three waves
      // per SIMD allow.)
      constexpr bool kAhead = SPH && !F64;
      using RecA = std::conditional_t<F64, uint3, uint4>;
      auto rec_at = [&](uint32_t j) -> RecA {
        if constexpr (F64) {
          const uint4* r = a.rec + j;
          return make_uint3(r->x, r->y, r->z);
        } else {
          return a.rec[j];
        }
      };
      auto next_bin = [&](int from) {
        int q = from;
        while (q < nb && uniform((int)bblk[q]) == 0) ++q;
        return q;
      };
      int b_ahead = nb, nblk_ahead = 0;
      uint32_t aJ[4] = {a.sentinel, a.sentinel, a.sentinel, a.sentinel};
      RecA aR[2] = {};
      real aW[2] = {real(0), real(0)};
      auto request_idx = [&](int bb) {
        nblk_ahead = uniform((int)bblk[bb]);
        const uint32_t* sa = scratch + (size_t)uniform((int)reg[bb]) * kBlock + lane;
#pragma unroll
        for (int k = 0; k < 4; ++k) aJ[k] = sa[k * kBlock];  // raw: range-checked at use
      };
      auto request_rec = [&]() {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t j = k < nblk_ahead ? aJ[k] : a.sentinel;
          aR[k] = rec_at(j);
          if constexpr (F64) aW[k] = a.w64[j];
        }
      };
      if constexpr (kAhead) {
        b_ahead = next_bin(0);
        if (b_ahead < nb) {
          request_idx(b_ahead);
          request_rec();
        }
      }
      for (int b = 0; b < nb; ++b) {
        const int nblk_b = uniform((int)bblk[b]);
        if (nblk_b == 0) continue;
        const int k0 = uniform((int)reg[b]);
        // this lane's entry of block i of the bin is entry(sb + i * kBlock)
        const uint32_t* sb = scratch + (size_t)k0 * kBlock;
        static_for<0, P::NG>([&](auto G) {
          constexpr int SG = P::slots(G);
          constexpr int per = SG >= 64 ? SG / 64 : 1;
          real acc[SG];
          // slots past the group's components are never written by the moments
#pragma unroll
          for (int i = P::gsize(G); i < SG; ++i) acc[i] = real(0);
          real hi[2] = {real(0), real(0)}, lo[2] = {real(0), real(0)};
          auto flush_acc = [&]() {
            transpose_reduce<SG>(acc, lane);
#pragma unroll
            for (int k = 0; k < per; ++k) {
              if constexpr (F64) {
                hi[k] += acc[k];
              } else {  // Kahan: hi holds the sum, lo the negated lost low part
                const real yk = acc[k] - lo[k];
                const real tk = hi[k] + yk;
                lo[k] = (tk - hi[k]) - yk;
                hi[k] = tk;
              }
            }
          };
          // Padding entries hold the zero-weight sentinel record, so every entry is evaluated
          // alike.
          if constexpr (F64 || SPH) {
            // FP64 replays every bin once per m-group and loads FP64 weights separately, and the
            // sphere's rounds are short (2 m_max + 1 components): both are latency-bound with one
            // round of look-ahead. A two-round software pipeline with separate registers for even
            // and odd rounds (no register copies, so each wait covers only its own load): as soon
            // as round i has taken its direction and weight, the record (and FP64 weight) of
            // round i + 2 and the index of round i + 4 are requested into that round's registers.
            // Reads past a bin's last block stay inside the wave's scratch (kScratchTail spare
            // blocks follow the regions); such entries are replaced by the sentinel before use.
            using RecT = std::conditional_t<F64, uint3, uint4>;
            // (plain per-lane addresses here: the scalar-base form of entry() measured 9% slower
            // on the FP64 sphere sweep)
            const uint32_t* sbl = sb + lane;
            auto idx_at = [&](int k) -> uint32_t { return k < nblk_b ? sbl[k * kBlock] : a.sentinel; };
            auto pos_at = [&](uint32_t j) -> RecT {
              if constexpr (F64) {
                const uint4* r = a.rec + j;
                return make_uint3(r->x, r->y, r->z);
              } else {
                return a.rec[j];
              }
            };
            auto wt_at = [&](uint32_t j) -> real {
              if constexpr (F64) return a.w64[j];
              else return real(0);  // mixed: the weight travels in the record
            };
            RecT R0, R1;
            real W0, W1;
            uint32_t J0, J1;
            if constexpr (kAhead) {
              // this bin's first entries were requested during the previous bin
              R0 = aR[0];
              R1 = aR[1];
              W0 = aW[0];
              W1 = aW[1];
              J0 = aJ[2];
              J1 = aJ[3];
              b_ahead = next_bin(b + 1);
              if (b_ahead < nb) request_idx(b_ahead);
            } else {
              R0 = pos_at(idx_at(0));
              R1 = pos_at(idx_at(1));
              W0 = wt_at(idx_at(0));
              W1 = wt_at(idx_at(1));
              J0 = idx_at(2);
              J1 = idx_at(3);
            }
            int i = 0;
            auto step = [&](RecT& R, real& W, uint32_t& J, auto WRITE) {
              // rounds stay in order, so each waits only for its own loads
              __builtin_amdgcn_sched_barrier(0);
              real vx, vy, vz;
              direction<SPH>(P0, tb, R, vx, vy, vz);
              real w;
              if constexpr (F64) w = W;
              else w = __uint_as_float(R.w);
              // The next loads go into this round's registers: the empty asm statement makes the
              // record address depend on this round's unit vector and weight, so the loads cannot
              // be hoisted above their last use.
              // J holds the raw entry of round i + 2 (read two rounds ago, possibly past the
              // bin's end): it is range-checked here, at its use. (Clamping it to the sentinel
              // index instead would also be safe, but past the bin's end it then fetches stale
              // records that may miss the caches and hold up the next waits: measured 0.6%
              // slower on the FP64 sphere sweep.)
              uint32_t jr = i + 2 < nblk_b ? J : a.sentinel;
              asm volatile("" : "+v"(jr), "+v"(w) : "v"(vx));
              R = pos_at(jr);
              if constexpr (F64) W = a.w64[jr];
              J = sbl[(i + 4) * kBlock];
              accumulate<LMAX, F64, SPH, G, decltype(WRITE)::value>(acc, vx, vy, vz, w);
              ++i;
            };
            // chunks of <= 64 rounds (they start at even rounds): the first round of a chunk
            // stores, the others add
            while (i < nblk_b) {
              const int n = min(64, nblk_b - i);
              step(R0, W0, J0, std::true_type{});
              for (int q = 0; q < (n - 1) >> 1; ++q) {
                step(R1, W1, J1, std::false_type{});
                step(R0, W0, J0, std::false_type{});
              }
              if (!(n & 1)) step(R1, W1, J1, std::false_type{});
              flush_acc();
            }
            if constexpr (kAhead) {
              if (b_ahead < nb) {
                // the record addresses depend on this bin's sums, so the loads stay here
                asm volatile("" : "+v"(aJ[0]), "+v"(aJ[1]) : "v"(hi[0]));
                request_rec();
              }
            }
          } else {
            // Mixed 3D: one round of software pipeline (the record of the next round and the
            // index of the round after it are in flight while the current round is evaluated);
            // its rounds are long enough to cover the latency. (Two alternating register sets
            // instead of the copies at the end of each round measured slower.)
            uint32_t jn = nblk_b > 1 ? entry(sb + kBlock) : a.sentinel;
            uint4 r = a.rec[entry(sb)];
            int i = 0;
            auto step = [&](auto WRITE) {
              uint4 rn = r;
              uint32_t jnn = a.sentinel;
              if (i + 1 < nblk_b) {
                rn = a.rec[jn];
                if (i + 2 < nblk_b) jnn = entry(sb + (i + 2) * kBlock);
              }
              real vx, vy, vz;
              direction<SPH>(P0, tb, r, vx, vy, vz);
              accumulate<LMAX, F64, SPH, G, decltype(WRITE)::value>(acc, vx, vy, vz, __uint_as_float(r.w));
              r = rn;
              jn = jnn;
              ++i;
            };
            // chunks of <= 64 rounds: the first round of a chunk stores, the others add
            while (i < nblk_b) {
              const int n = min(64, nblk_b - i);
              step(std::true_type{});
              for (int q = 1; q < n; ++q) step(std::false_type{});
              flush_acc();
            }
          }
#pragma unroll
          for (int k = 0; k < per; ++k) {
            const int ms = mslot[G][k];
            if (ms >= 0 && ms < NC) mom[ms] = F64 ? hi[k] : (hi[k] - lo[k]);
          }
        });
        wave_sync();  // the moments in LDS, for every lane
        if (lane == b) sdd += (double)mom[0];  // M_00 = sum of w_j over the bin
        // moments -> normalised a_lm of bin b (on the sphere the moments are the a_m)
        if constexpr (SPH) {
          for (int c = lane; c < NC; c += 64) {
            real v = mom[c];
            real* dst = slot + b * NC + c;
            if (written & (1u << b)) v += *dst;
            *dst = v;
          }
        } else {
          // this lane's terms in sequence; a component is stored after its last term
          real v = real(0);
          for (int q = 0; q < a.conv_q; ++q) {
            const int meta = smeta[q * 64 + lane];
            v += scoef[q * 64 + lane] * mom[meta & 0x7F];
            if (meta & 0x4000) {
              real* dst = slot + b * NC + ((meta >> 7) & 0x7F);
              if (written & (1u << b)) v += *dst;
              *dst = v;
              v = real(0);
            }
          }
        }
        wave_sync();  // mom is rewritten by the next bin (the tile is read after a barrier)
        written |= 1u << b;
      }
    };

    // Closes the regions (pads each bin's last block with the sentinel), replays the shells and
    // empties the regions.
    auto flush_shells = [&]() {
      uint32_t c_b = 0, n_b = 0;
      if (lane < nb) {
        c_b = (uint32_t)cur[lane];
        n_b = c_b - reg[lane] * kBlock;
        btot[lane] += n_b;
        bblk[lane] = (n_b + kBlock - 1) / kBlock;
      }
      uint64_t tails = __ballot(lane < nb && (n_b & (kBlock - 1)) != 0);
      while (tails) {
        const int b = __ffsll((unsigned long long)tails) - 1;
        tails &= tails - 1;
        const uint32_t c = uniform(__builtin_amdgcn_readlane(c_b, b));
        const uint32_t e = (c + kBlock - 1) & ~(uint32_t)(kBlock - 1);  // regions are block aligned
        if (c + (uint32_t)lane < e) scratch[c + lane] = a.sentinel;
      }
      __syncthreads();  // the region stores complete before the replay loads them
      process_blocks();
      reset_cursors();
    };

    // Evaluates one batch of rounds. Bin decision in FP32 when the fractional bin position is
    // farther than the proven error bound from an edge; every accepted lane takes the next entry
    // of its bin's region from one LDS cursor increment and stores its sorted position there
    // (rejected lanes sit out both). Lanes near a bin edge are decided exactly afterwards (FP64
    // squared lattice separation against the integer thresholds). Returns true when a region
    // passed its soft limit.
    // FP32 bin position of a candidate: 3D linear in the separation, sphere linear in
    // theta = 2 asin(chord / 2). fast: far enough from a bin edge for the FP32 decision.
    // The bin constants are copied into VGPRs once per batch: the kernel's wave-uniform values
    // outnumber the scalar registers, and a spilled one read back per candidate costs a VALU
    // issue slot (v_readlane) each time.
    struct BinK {
      float inv_dl, u0, eps, one_me, hinv;
    };
    auto bin_consts = [&]() {
      BinK k = {cu.inv_dl, cu.u0, cu.eps, cu.one_me, cu.hinv};
      // (3D only: the sphere kernel measured faster with its constants left to the compiler)
      if constexpr (!SPH) asm volatile("" : "+v"(k.inv_dl), "+v"(k.u0), "+v"(k.eps), "+v"(k.one_me));
      return k;
    };
    auto bin_pos = [&](const uint4& r, const BinK& k, int& bb, bool& fast) {
      const float fx = (float)sdiff(r.x, P0.qx), fy = (float)sdiff(r.y, P0.qy), fz = (float)sdiff(r.z, P0.qz);
      const float r2 = fx * fx + fy * fy + fz * fz;
      float uu;
      if constexpr (SPH) {
        const float x = __builtin_amdgcn_sqrtf(r2) * k.hinv;
        uu = (cu.asin_small ? asin_small(x) : asin01(x)) * k.inv_dl + k.u0;
      } else {
        uu = __builtin_amdgcn_sqrtf(r2) * k.inv_dl + k.u0;
      }
      // uu - floor(uu): exact for uu >= 0 (Sterbenz); a negative uu is outside the bins anyway.
      // v_cvt_flr_i32_f32 is floor and conversion in one instruction.
      const float fr = __builtin_amdgcn_fractf(uu);
      asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(bb) : "v"(uu));
      fast = fr >= k.eps && fr <= k.one_me;
    };
    auto process_batch = [&](const uint32_t(&id)[kBatch], const uint4(&rc)[kBatch]) -> bool {
      bool soft = false;
      bool accv[kBatch];
      unsigned long long cwv[kBatch];  // set (and read) on accepted lanes only
      bool slow = false;  // this lane has a candidate near a bin edge
      const BinK bk = bin_consts();
      // all cursor increments of the batch are issued before the first result is used, so their
      // LDS round trips overlap
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        int bb;
        bool fast;
        bin_pos(rc[u], bk, bb, fast);
        const bool ok = id[u] != a.sentinel;
        const bool acc = ok && fast && (uint32_t)bb < (uint32_t)nb;
        slow |= ok && !fast;
        accv[u] = acc;
        if (acc) cwv[u] = atomicAdd(&cur[bb], 1ull);
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        if (accv[u]) {
          const unsigned long long cw = cwv[u];
          soft |= (uint32_t)cw >= (uint32_t)(cw >> 32);
          put((uint32_t)cw, id[u]);
        }
      }
      if (__builtin_amdgcn_ballot_w64(slow)) {  // rare: the FP32 position is recomputed rather than kept
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          int bb;
          bool fast;
          bin_pos(rc[u], bk, bb, fast);
          if (id[u] != a.sentinel && !fast) {
            const double ddx = sdiff(rc[u].x, P0.qx) >> cu.sh, ddy = sdiff(rc[u].y, P0.qy) >> cu.sh,
                         ddz = sdiff(rc[u].z, P0.qz) >> cu.sh;
            const double R2 = fma(ddx, ddx, fma(ddy, ddy, ddz * ddz));
            if (R2 > 0.0 && R2 >= T0 && R2 < Tn) {
              bb = bb < 0 ? 0 : (bb >= nb ? nb - 1 : bb);
              while (R2 < sT[bb]) --bb;
              while (bb + 1 < nb && R2 >= sT[bb + 1]) ++bb;
              const unsigned long long cw = atomicAdd(&cur[bb], 1ull);
              soft |= (uint32_t)cw >= (uint32_t)(cw >> 32);
              put((uint32_t)cw, id[u]);
            }
          }
        }
      }
      return __ballot(soft) != 0;
    };

    // ---- pass over the stencil: batch B is generated and its records loaded while batch A is
    // evaluated.
    // The shells are replayed from one place (keeps a single copy of their code).
    uint32_t idA[kBatch], idB[kBatch];
    uint4 rA[kBatch], rB[kBatch];
    bool moreA = gen_batch(idA);
    load_batch(idA, rA);
    for (;;) {
      const bool last = !moreA;
      bool flush = last;
      if (!last) {
        const bool moreB = gen_batch(idB);
        load_batch(idB, rB);
        flush = process_batch(idA, rA);
        moreA = moreB;
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          idA[u] = idB[u];
          rA[u] = rB[u];
        }
      }
      if (flush) {
        // The batch in flight waits in LDS while the shells are replayed, so that the replay has
        // the register file to itself (three waves per SIMD without spilling in the replay).
        uint4* prec = reinterpret_cast<uint4*>(smem + Lds::PARK);
        uint32_t* pid = reinterpret_cast<uint32_t*>(smem + Lds::PARK + kBatch * 64 * 16);
        if (!last) {
#pragma unroll
          for (int u = 0; u < kBatch; ++u) {
            prec[u * 64 + lane] = rA[u];
            pid[u * 64 + lane] = idA[u];
          }
        }
        asm volatile("" ::: "memory");
        flush_shells();
        asm volatile("" ::: "memory");
        if (!last) {
#pragma unroll
          for (int u = 0; u < kBatch; ++u) {
            rA[u] = prec[u * 64 + lane];
            idA[u] = pid[u * 64 + lane];
          }
        }
      }
      if (last) break;
    }

    // bins without any pair: zero shells
    for (int b = 0; b < nb; ++b)
      if (!(written & (1u << b)))
        for (int c = lane; c < NC; c += 64) slot[b * NC + c] = real(0);

    uint32_t pairs_p = lane < nb ? btot[lane] : 0u;
    if (a.counts && lane < nb) a.counts[(size_t)p * nb + lane] = (int32_t)pairs_p;
    if (cat != bins_cat) {
      flush_bins();
      bins_cat = cat;
    }
    bins_np += pairs_p;
    bins_dd += (double)wp * sdd;
    sdd = 0.0;
    for (int off = 32; off > 0; off >>= 1) pairs_p += __shfl_xor(pairs_p, off);
    my_pairs += pairs_p;
    if (a.alm_debug) {
      __syncthreads();  // the tile's stores by every lane
      real* dbg = reinterpret_cast<real*>(a.alm_debug) + (size_t)p * nb * NC;
      for (int i = lane; i < nb * NC; i += 64) dbg[i] = slot[i];
    }
    if (lane == 0) swt[tile_n] = wp;
    __syncthreads();
    ++tile_n;
    if (tile_n == TP) do_contract();
  }
  if constexpr (!DET) {  // (DET closed its last tile before leaving the loop)
    do_contract();
    flush_part();
  }
  flush_bins();
  if (lane == 0) {
    atomicAdd(&a.stats[0], my_pairs);
    atomicAdd(&a.stats[1], my_cand);
  }
}

// ------------------------------------------------------------------------------------------
// Host-side launch table.
// ------------------------------------------------------------------------------------------
template <int LMAX, bool F64, bool SPH, bool DET>
static hipError_t launch_det(SweepArgs args, int waves, size_t lds, hipStream_t stream) {
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sweep_kernel<LMAX, F64, SPH, DET>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((sweep_kernel<LMAX, F64, SPH, DET>), dim3(waves), dim3(64), lds, stream, args);
  return hipSuccess;
}
template <int LMAX, bool F64, bool SPH>
static hipError_t launch_one(SweepArgs args, int waves, size_t lds, hipStream_t stream) {
  return args.det_tiles ? launch_det<LMAX, F64, SPH, true>(args, waves, lds, stream)
                        : launch_det<LMAX, F64, SPH, false>(args, waves, lds, stream);
}

// Deterministic form, second step: the tile slots are added in tile order, in two fixed levels
// (chunks of consecutive tiles, then the chunks of each catalogue).
__global__ void k_det_chunks(const double* __restrict__ det_out, uint32_t stride, const uint2* __restrict__ chunks,
                             uint32_t nchunk, double* __restrict__ part1) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (size_t)nchunk * stride) return;
  const uint32_t q = (uint32_t)(g / stride), i = (uint32_t)(g % stride);
  const uint2 c = chunks[q];
  double s = 0.0;
  for (uint32_t t = c.x; t < c.y; ++t) s += det_out[(size_t)t * stride + i];
  part1[g] = s;
}
__global__ void k_det_cats(const double* __restrict__ part1, uint32_t stride, const uint32_t* __restrict__ cat_chunk,
                           int ncat, uint32_t Z, int nb, double* __restrict__ zeta, double* __restrict__ dd) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (size_t)ncat * stride) return;
  const uint32_t k = (uint32_t)(g / stride), i = (uint32_t)(g % stride);
  double s = 0.0;
  for (uint32_t q = cat_chunk[k]; q < cat_chunk[k + 1]; ++q) s += part1[(size_t)q * stride + i];
  if (i < Z) zeta[(size_t)k * Z + i] = s;
  else dd[(size_t)k * nb + (i - Z)] = s;
}

hipError_t launch_det_reduce(const double* det_out, uint32_t stride, const uint2* chunks, uint32_t nchunk,
                             const uint32_t* cat_chunk, int ncat, uint32_t Z, int nb, double* part1, double* zeta,
                             double* dd, hipStream_t s) {
  const size_t n1 = (size_t)nchunk * stride, n2 = (size_t)ncat * stride;
  if (n1) hipLaunchKernelGGL(k_det_chunks, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, det_out, stride, chunks,
                             nchunk, part1);
  if (n2) hipLaunchKernelGGL(k_det_cats, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, part1, stride, cat_chunk,
                             ncat, Z, nb, zeta, dd);
  return hipGetLastError();
}

size_t sweep_lds_bytes(int nb, int lmax, bool f64, bool sphere) {
  (void)nb;
  return (size_t)Lds::bytes(lmax, f64, sphere);
}

// Bytes of per-wave tile area, including the FP64 zeta partial.
size_t sweep_tile_bytes_per_wave(int lmax, int nb, bool f64, bool sphere) {
  const int NC = ncomp(lmax, sphere);
  const size_t tp = tile_primaries(f64, sphere);
  const size_t elem = f64 ? 8 : 4;
  return tp * nb * NC * elem + (size_t)(lmax + 1) * nb * nb * 8;
}

template <int L>
static hipError_t launch_l(bool f64, bool sphere, const SweepArgs& args, int waves, size_t lds, hipStream_t s) {
  if (sphere) return f64 ? launch_one<L, true, true>(args, waves, lds, s) : launch_one<L, false, true>(args, waves, lds, s);
  return f64 ? launch_one<L, true, false>(args, waves, lds, s) : launch_one<L, false, false>(args, waves, lds, s);
}

hipError_t launch_sweep(int lmax, bool f64, bool sphere, const SweepArgs& args, int waves, hipStream_t stream) {
  const size_t lds = sweep_lds_bytes(args.nb, lmax, f64, sphere);
  hipError_t err = hipErrorInvalidValue;
  switch (lmax) {
    case 0: err = launch_l<0>(f64, sphere, args, waves, lds, stream); break;
    case 1: err = launch_l<1>(f64, sphere, args, waves, lds, stream); break;
    case 2: err = launch_l<2>(f64, sphere, args, waves, lds, stream); break;
    case 3: err = launch_l<3>(f64, sphere, args, waves, lds, stream); break;
    case 4: err = launch_l<4>(f64, sphere, args, waves, lds, stream); break;
    case 5: err = launch_l<5>(f64, sphere, args, waves, lds, stream); break;
    case 6: err = launch_l<6>(f64, sphere, args, waves, lds, stream); break;
    case 7: err = launch_l<7>(f64, sphere, args, waves, lds, stream); break;
    case 8: err = launch_l<8>(f64, sphere, args, waves, lds, stream); break;
    case 9: err = launch_l<9>(f64, sphere, args, waves, lds, stream); break;
    case 10: err = launch_l<10>(f64, sphere, args, waves, lds, stream); break;
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess) return err;
  return hipGetLastError();
}

// Group plan query for the host (normalisation constants are per global component).
int plan_groups(int lmax, bool f64) { return (f64 && (lmax + 1) * (lmax + 1) > 64) ? 2 : 1; }

}  // namespace tpcf
