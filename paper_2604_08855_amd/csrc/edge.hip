// edge.hip -- edge correction of the multipoles for data-minus-randoms fields.
//
// With N the multipoles of the data-minus-randoms field and R those of the weighted randoms
// (both as computed by the sweep), the corrected three-point function is zeta(mu) = N(mu)/R(mu)
// for every bin pair (Slepian & Eisenstein 2015, cited in the paper's Features section; the
// paper gives no formula). Products of Legendre polynomials expand with squared 3j symbols,
//     P_a P_b = sum_c (2c + 1) (a b c; 0 0 0)^2 P_c,
// so in Legendre coefficients N_L = R_0 sum_l'' M_{L l''} zeta_l'' with
//     M_{L l''} = (2L + 1) sum_l' (L l' l''; 0 0 0)^2 f_l',   f_l' = R_l' / R_0,
// truncated at l_max. The sweep's zeta_l are (2l + 1)/(4 pi) times the Legendre sums, the same
// factor for N and R, so they enter as they are. One thread solves one bin pair's system by
// Gaussian elimination with partial pivoting in FP64.
//
// On the sphere (masked maps) the same construction acts on the cosine moments of the position
// angle: with zeta(phi) = N(phi)/R(phi) = c_0 + 2 sum_{m>=1} c_m cos(m phi) and the raw zeta_m
// being the moments int X(phi) cos(m phi) dphi,
//     N_m = sum_{m'} eps_m' c_m' (R_{m+m'} + R_{|m-m'|}) / 2,   eps_0 = 1, eps_m' = 2,
// truncated at m_max (R_k = 0 above it), since cos a cos b = (cos(a+b) + cos(a-b)) / 2.
#include <vector>

#include "tpcf_internal.h"

namespace tpcf {

// (a b c; 0 0 0)^2 from the closed form for zero projections: zero unless a + b + c = 2g is even
// and (a, b, c) is a triangle; otherwise
//     (2g-2a)! (2g-2b)! (2g-2c)! / (2g+1)! * [g! / ((g-a)! (g-b)! (g-c)!)]^2.
std::vector<double> threej_squared_table(int lmax) {
  const int L1 = lmax + 1;
  std::vector<long double> fact(3 * L1 + 2, 1.0L);
  for (size_t k = 1; k < fact.size(); ++k) fact[k] = fact[k - 1] * (long double)k;
  std::vector<double> t((size_t)L1 * L1 * L1, 0.0);
  for (int a = 0; a < L1; ++a)
    for (int b = 0; b < L1; ++b)
      for (int c = 0; c < L1; ++c) {
        const int J = a + b + c;
        if (J & 1) continue;
        if (c > a + b || c < (a > b ? a - b : b - a)) continue;
        const int g = J / 2;
        const long double r = fact[J - 2 * a] * fact[J - 2 * b] * fact[J - 2 * c] / fact[J + 1];
        const long double q = fact[g] / (fact[g - a] * fact[g - b] * fact[g - c]);
        t[((size_t)a * L1 + b) * L1 + c] = (double)(r * q * q);
      }
  return t;
}

// Solves A x = b (b in column L1 of A) by Gaussian elimination with partial pivoting.
__device__ void solve_augmented(double (&A)[kMaxLmax + 1][kMaxLmax + 2], int L1, double (&x)[kMaxLmax + 1]) {
  for (int k = 0; k < L1; ++k) {
    int piv = k;
    for (int r = k + 1; r < L1; ++r)
      if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
    if (piv != k)
      for (int j = 0; j <= L1; ++j) {
        const double t = A[k][j];
        A[k][j] = A[piv][j];
        A[piv][j] = t;
      }
    for (int r = k + 1; r < L1; ++r) {
      const double m = A[r][k] / A[k][k];
      for (int j = k; j <= L1; ++j) A[r][j] -= m * A[k][j];
    }
  }
  for (int k = L1 - 1; k >= 0; --k) {
    double s = A[k][L1];
    for (int j = k + 1; j < L1; ++j) s -= A[k][j] * x[j];
    x[k] = s / A[k][k];
  }
}

__global__ void k_edge_correct(int count, int lmax, int nb, const double* __restrict__ N,
                               const double* __restrict__ R, const double* __restrict__ t3,
                               double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // (catalogue, b1, b2)
  if (i >= count) return;
  const int nn = nb * nb;
  const int cat = i / nn, bb = i - cat * nn;
  const int L1 = lmax + 1;
  const size_t base = (size_t)cat * L1 * nn + bb;
  const double R0 = R[base];
  if (R0 == 0.0) {
    for (int l = 0; l < L1; ++l) out[base + (size_t)l * nn] = 0.0;
    return;
  }
  double f[kMaxLmax + 1];
  for (int l = 0; l < L1; ++l) f[l] = R[base + (size_t)l * nn] / R0;
  double A[kMaxLmax + 1][kMaxLmax + 2];
  for (int L = 0; L < L1; ++L) {
    for (int l2 = 0; l2 < L1; ++l2) {
      double s = 0.0;
      for (int lp = 0; lp < L1; ++lp) s += t3[((size_t)L * L1 + lp) * L1 + l2] * f[lp];
      A[L][l2] = (2 * L + 1) * s;
    }
    A[L][L1] = N[base + (size_t)L * nn] / R0;
  }
  double x[kMaxLmax + 1];
  solve_augmented(A, L1, x);
  for (int l = 0; l < L1; ++l) out[base + (size_t)l * nn] = x[l];
}

__global__ void k_edge_correct_sphere(int count, int mmax, int nb, const double* __restrict__ N,
                                      const double* __restrict__ R, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // (catalogue, b1, b2)
  if (i >= count) return;
  const int nn = nb * nb;
  const int cat = i / nn, bb = i - cat * nn;
  const int M1 = mmax + 1;
  const size_t base = (size_t)cat * M1 * nn + bb;
  const double R0 = R[base];
  if (R0 == 0.0) {
    for (int m = 0; m < M1; ++m) out[base + (size_t)m * nn] = 0.0;
    return;
  }
  double f[kMaxLmax + 1];
  for (int m = 0; m < M1; ++m) f[m] = R[base + (size_t)m * nn] / R0;
  double A[kMaxLmax + 1][kMaxLmax + 2];
  for (int m = 0; m < M1; ++m) {
    for (int mp = 0; mp < M1; ++mp) {
      const double hi = m + mp < M1 ? f[m + mp] : 0.0;
      const double lo = f[m > mp ? m - mp : mp - m];
      A[m][mp] = (mp == 0 ? 0.5 : 1.0) * (hi + lo);
    }
    A[m][M1] = N[base + (size_t)m * nn] / R0;
  }
  double x[kMaxLmax + 1];
  solve_augmented(A, M1, x);
  for (int m = 0; m < M1; ++m) out[base + (size_t)m * nn] = x[m];
}

hipError_t launch_edge_correct(int ncat, int lmax, int nb, const double* N, const double* R,
                               const double* t3, double* out, hipStream_t s) {
  const int count = ncat * nb * nb;
  if (count > 0)
    hipLaunchKernelGGL(k_edge_correct, dim3((count + 63) / 64), dim3(64), 0, s, count, lmax, nb, N, R, t3, out);
  return hipGetLastError();
}

hipError_t launch_edge_correct_sphere(int ncat, int mmax, int nb, const double* N, const double* R, double* out,
                                      hipStream_t s) {
  const int count = ncat * nb * nb;
  if (count > 0)
    hipLaunchKernelGGL(k_edge_correct_sphere, dim3((count + 63) / 64), dim3(64), 0, s, count, mmax, nb, N, R, out);
  return hipGetLastError();
}

}  // namespace tpcf
