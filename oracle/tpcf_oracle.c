/*
 * tpcf_oracle.c -- plain, slow FP64 CPU oracle for the 3PCF multipoles.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library. The product path never calls it, and this file shares no
 * code, header, table or constant with the GPU library: everything below is written out
 * from the definition of the estimator.
 *
 * What is computed (Implementation section of the paper: a harmonic decomposition of the
 * triangle angle; per pivot, all neighbours in range fill multipole bins; the spherical
 * harmonic form is the 3D version of the expansion the paper builds on, Szapudi 2004 and
 * Slepian & Eisenstein 2015, both cited in the Statement of need and Features sections):
 *
 *   for every primary p and secondary j != p with r_min <= |x_j - x_p| < r_max,
 *     b(p,j)     = radial bin of the separation,
 *     a_lm(p,b)  = sum_{j in b} w_j conj(Y_lm(unit(x_j - x_p))),    -l <= m <= l,
 *   zeta_l(b1,b2) = sum_p w_p sum_{m=-l}^{l} Re[ a_lm(p,b1) conj(a_lm(p,b2)) ].
 *
 * Y_lm is the orthonormal spherical harmonic with the Condon-Shortley phase, evaluated here
 * the textbook way: theta = acos(u_z), phi = atan2(u_y, u_x),
 *   Y_lm = N_lm P_l^m(cos theta) e^{i m phi},  N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),
 *   Y_{l,-m} = (-1)^m conj(Y_lm).
 * P_l^m comes from the standard upward recurrence in l at fixed m, seeded by
 *   P_m^m = (-1)^m (2m-1)!! (1-x^2)^{m/2},  P_{m+1}^m = (2m+1) x P_m^m.
 *
 * Readings where the paper is silent (the paper prints no estimator formula):
 *   - Positions are snapped to a cubic lattice of spacing s = L / 2^K with
 *     K = 25 + floor(log2(L / r_max)), capped at 32 (periodic) or 31 (non-periodic), so that
 *     r_max / s <= 2^25 and every in-range squared separation is an exact integer below 2^53.
 *     q = floor(x * (2^K / L)) taken mod 2^K (periodic) or clamped to [0, 2^K) (non-periodic).
 *   - Periodic boxes use the minimum image of the lattice displacement.
 *   - Bins are half-open and linear: e_k = r_min + k (r_max - r_min)/n_b, e_{n_b} = r_max;
 *     integer thresholds T_k = ceil(fl64(fl64(e_k * 2^K/L)^2)); the pair is in bin k iff
 *     T_k <= R^2 < T_{k+1} with R^2 the exact integer squared lattice separation.
 *   - Pairs with R^2 = 0 have no direction and are skipped.
 *   - The primary weight w_p multiplies each primary's contribution.
 *   - The j = k term (one secondary on both triangle legs) is included, as it is in
 *     a a^* itself.
 *
 * Summation: each primary's a_lm is a plain sequential FP64 sum over j in input order. The
 * primaries are cut into at most ORACLE_CHUNKS fixed chunks; each chunk is summed
 * sequentially and the chunk partials are added in chunk order, so the result does not depend
 * on the number of threads.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_LMAX_CAP 16
#define ORACLE_CHUNKS 1024

/* ---------------------------------------------------------------- lattice and bins */

int oracle_lattice_bits(double box, double rmax, int periodic)
{
    int e = 0;
    frexp(box / rmax, &e); /* box/rmax = f * 2^e with f in [0.5, 1): floor(log2) = e - 1 */
    int K = 25 + (e - 1);
    int kcap = periodic ? 32 : 31;
    if (K > kcap) K = kcap;
    if (K < 1) K = 1;
    return K;
}

static double lattice_scale(double box, int K) { return ldexp(1.0, K) / box; }

void oracle_thresholds(int nbins, double rmin, double rmax, double box, int K, uint64_t *T)
{
    double sc = lattice_scale(box, K);
    double delta = (rmax - rmin) / nbins;
    for (int k = 0; k <= nbins; k++) {
        double e = (k == nbins) ? rmax : rmin + k * delta;
        double v = e * sc;
        T[k] = (uint64_t)ceil(v * v);
    }
}

/* Lattice coordinate of one position. */
static int64_t snap(double x, double sc, int K, int periodic)
{
    int64_t M = (int64_t)1 << K;
    int64_t t = (int64_t)floor(x * sc);
    if (periodic) {
        t %= M;
        if (t < 0) t += M;
    } else {
        if (t < 0) t = 0;
        if (t > M - 1) t = M - 1;
    }
    return t;
}

/* Snap a whole catalogue (exported so tests can check the lattice itself). */
void oracle_snap(int64_t n, const double *x, double box, int K, int periodic, int64_t *q)
{
    double sc = lattice_scale(box, K);
    for (int64_t i = 0; i < n; i++) q[i] = snap(x[i], sc, K, periodic);
}

/* ---------------------------------------------------------------- spherical harmonics */

static int lm_index(int l, int m) { return l * l + l + m; } /* m in [-l, l] */

/* Y_lm(u) for 0 <= l <= lmax, -l <= m <= l, into Y[lm_index(l,m)]. u must be a unit vector. */
static void ylm_unit(int lmax, double ux, double uy, double uz, double complex *Y)
{
    double P[ORACLE_LMAX_CAP + 1][ORACLE_LMAX_CAP + 1];
    double ct = uz;
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    double theta = acos(ct);
    double phi = atan2(uy, ux);
    double x = cos(theta);
    double sx = sin(theta); /* (1 - x^2)^{1/2} >= 0 */

    for (int m = 0; m <= lmax; m++) {
        /* P_m^m = (-1)^m (2m-1)!! (1-x^2)^{m/2} */
        double pmm = 1.0;
        for (int i = 1; i <= m; i++) pmm *= -(2.0 * i - 1.0) * sx;
        P[m][m] = pmm;
        if (m + 1 <= lmax) P[m + 1][m] = (2.0 * m + 1.0) * x * pmm;
        for (int l = m + 2; l <= lmax; l++)
            P[l][m] = ((2.0 * l - 1.0) * x * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (double)(l - m);
    }
    for (int l = 0; l <= lmax; l++) {
        for (int m = 0; m <= l; m++) {
            long double ratio = 1.0L; /* (l-m)!/(l+m)! */
            for (int i = l - m + 1; i <= l + m; i++) ratio /= (long double)i;
            double N = sqrt((double)((2.0L * l + 1.0L) / (4.0L * 3.14159265358979323846264338327950288L) * ratio));
            double complex e = cos(m * phi) + I * sin(m * phi);
            double complex y = N * P[l][m] * e;
            Y[lm_index(l, m)] = y;
            if (m > 0) Y[lm_index(l, -m)] = ((m & 1) ? -1.0 : 1.0) * conj(y);
        }
    }
}

/* Exported for the tests: Y_lm of n unit vectors, out arrays [n][(lmax+1)^2]. */
int oracle_ylm(int lmax, int64_t n, const double *ux, const double *uy, const double *uz,
               double *out_re, double *out_im)
{
    if (lmax < 0 || lmax > ORACLE_LMAX_CAP) return 1;
    int nc = (lmax + 1) * (lmax + 1);
    double complex Y[(ORACLE_LMAX_CAP + 1) * (ORACLE_LMAX_CAP + 1)];
    for (int64_t i = 0; i < n; i++) {
        ylm_unit(lmax, ux[i], uy[i], uz[i], Y);
        for (int c = 0; c < nc; c++) {
            out_re[i * nc + c] = creal(Y[c]);
            out_im[i * nc + c] = cimag(Y[c]);
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- the estimator */

typedef struct {
    int64_t n;
    const int64_t *qx, *qy, *qz;
    const double *w;
    int K, periodic, nbins, lmax;
    const uint64_t *T;
} problem;

/* Minimum-image (periodic) or plain lattice displacement along one axis. */
static int64_t displacement(int64_t qj, int64_t qp, int K, int periodic)
{
    int64_t d = qj - qp;
    if (periodic) {
        int64_t M = (int64_t)1 << K;
        if (d >= M / 2) d -= M;
        if (d < -M / 2) d += M;
    }
    return d;
}

/* Bin of the pair (pivot at lattice point qp, secondary j): -1 when out of range. Also returns
 * the displacement. */
static int pair_bin_at(const problem *P, const int64_t qp[3], int64_t j, int64_t d[3])
{
    d[0] = displacement(P->qx[j], qp[0], P->K, P->periodic);
    d[1] = displacement(P->qy[j], qp[1], P->K, P->periodic);
    d[2] = displacement(P->qz[j], qp[2], P->K, P->periodic);
    const int64_t lim = (int64_t)1 << 26; /* beyond this on one axis, R^2 > 2^52 > T_nb */
    for (int a = 0; a < 3; a++)
        if (d[a] > lim || d[a] < -lim) return -1;
    uint64_t R2 = (uint64_t)(d[0] * d[0]) + (uint64_t)(d[1] * d[1]) + (uint64_t)(d[2] * d[2]);
    if (R2 == 0) return -1;
    if (R2 < P->T[0] || R2 >= P->T[P->nbins]) return -1;
    int b = 0;
    while (b + 1 < P->nbins && R2 >= P->T[b + 1]) b++;
    return b;
}

static int pair_bin(const problem *P, int64_t p, int64_t j, int64_t d[3])
{
    const int64_t qp[3] = {P->qx[p], P->qy[p], P->qz[p]};
    return pair_bin_at(P, qp, j, d);
}

/* One pivot at lattice point qp with weight wp: a_lm over all secondaries other than `skip`, then
 * its contribution to zeta (added into zacc). */
static void one_pivot(const problem *P, const int64_t qp[3], double wp, int64_t skip, double complex *alm,
                      double complex *Y, double *zacc, int64_t *counts, int64_t *npairs)
{
    const int nb = P->nbins, lmax = P->lmax, nc = (lmax + 1) * (lmax + 1);
    memset(alm, 0, sizeof(double complex) * (size_t)nb * nc);
    for (int b = 0; b < nb; b++) counts[b] = 0;
    for (int64_t j = 0; j < P->n; j++) {
        if (j == skip) continue;
        int64_t d[3];
        int b = pair_bin_at(P, qp, j, d);
        if (b < 0) continue;
        double r = sqrt((double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2]);
        ylm_unit(lmax, d[0] / r, d[1] / r, d[2] / r, Y);
        double complex *a = alm + (size_t)b * nc;
        for (int c = 0; c < nc; c++) a[c] += P->w[j] * conj(Y[c]);
        counts[b]++;
        (*npairs)++;
    }
    for (int l = 0; l <= lmax; l++)
        for (int b1 = 0; b1 < nb; b1++)
            for (int b2 = 0; b2 < nb; b2++) {
                double s = 0.0;
                for (int m = -l; m <= l; m++) {
                    int c = lm_index(l, m);
                    s += creal(alm[(size_t)b1 * nc + c] * conj(alm[(size_t)b2 * nc + c]));
                }
                zacc[((size_t)l * nb + b1) * nb + b2] += wp * s;
            }
}

/* One primary of the catalogue (input index p). */
static void one_primary(const problem *P, int64_t p, double complex *alm, double complex *Y,
                        double *zacc, int64_t *counts, int64_t *npairs)
{
    const int64_t qp[3] = {P->qx[p], P->qy[p], P->qz[p]};
    one_pivot(P, qp, P->w[p], p, alm, Y, zacc, counts, npairs);
}

/*
 * zeta[(lmax+1)][nbins][nbins]: primaries are input indices [p_begin, p_end), secondaries are
 * all n points. counts (optional) receives [p_end-p_begin][nbins] unit-weight pair counts;
 * alm_out (optional) receives a_lm as [p_end-p_begin][nbins][(lmax+1)^2][2] (re, im).
 * Returns 0, or 1 on invalid arguments.
 */
int oracle_zeta(int64_t n, const double *x, const double *y, const double *z, const double *w,
                double box, int periodic, int nbins, double rmin, double rmax, int lmax,
                int64_t p_begin, int64_t p_end, double *zeta, int64_t *counts, double *alm_out,
                int64_t *npairs_out, int nthreads)
{
    if (n < 0 || nbins < 1 || lmax < 0 || lmax > ORACLE_LMAX_CAP || !(rmin >= 0.0) ||
        !(rmax > rmin) || !(box > 0.0) || p_begin < 0 || p_end > n || p_begin > p_end)
        return 1;
    const int nb = nbins, nc = (lmax + 1) * (lmax + 1);
    const size_t zsize = (size_t)(lmax + 1) * nb * nb;
    memset(zeta, 0, sizeof(double) * zsize);
    if (npairs_out) *npairs_out = 0;
    if (n == 0 || p_begin == p_end) return 0;

    int K = oracle_lattice_bits(box, rmax, periodic);
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
    oracle_snap(n, x, box, K, periodic, q);
    oracle_snap(n, y, box, K, periodic, q + n);
    oracle_snap(n, z, box, K, periodic, q + 2 * n);
    oracle_thresholds(nb, rmin, rmax, box, K, T);
    problem P = {n, q, q + n, q + 2 * n, w, K, periodic, nb, lmax, T};

    const int64_t np = p_end - p_begin;
    const int64_t nchunk = np < ORACLE_CHUNKS ? np : ORACLE_CHUNKS;
    double *part = (double *)calloc((size_t)nchunk * zsize, sizeof(double));
    int64_t *pairs = (int64_t *)calloc((size_t)nchunk, sizeof(int64_t));

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double complex *alm = (double complex *)malloc(sizeof(double complex) * (size_t)nb * nc);
        double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)nc);
        int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < nchunk; c++) {
            int64_t lo = p_begin + np * c / nchunk, hi = p_begin + np * (c + 1) / nchunk;
            for (int64_t p = lo; p < hi; p++) {
                one_primary(&P, p, alm, Y, part + (size_t)c * zsize, cnt, &pairs[c]);
                if (counts)
                    for (int b = 0; b < nb; b++) counts[(p - p_begin) * nb + b] = cnt[b];
                if (alm_out)
                    for (size_t k = 0; k < (size_t)nb * nc; k++) {
                        alm_out[((size_t)(p - p_begin) * nb * nc + k) * 2] = creal(alm[k]);
                        alm_out[((size_t)(p - p_begin) * nb * nc + k) * 2 + 1] = cimag(alm[k]);
                    }
            }
        }
        free(alm);
        free(Y);
        free(cnt);
    }
    int64_t total = 0;
    for (int64_t c = 0; c < nchunk; c++) {
        for (size_t k = 0; k < zsize; k++) zeta[k] += part[(size_t)c * zsize + k];
        total += pairs[c];
    }
    if (npairs_out) *npairs_out = total;
    free(part);
    free(pairs);
    free(q);
    free(T);
    return 0;
}

/*
 * Pair sums per radial bin, the two-point by-product of the same sweep (the paper's second
 * statistic; Introduction and Features sections): for primaries [p_begin, p_end) and all
 * secondaries j != p,
 *     npairs[b] = number of (p, j) with (p, j) in bin b           (exact integer)
 *     dd[b]     = sum over those pairs of w_p w_j                 (FP64)
 * with the same lattice binning as oracle_zeta. Returns 0, or 1 on invalid arguments.
 */
int oracle_pair_sums(int64_t n, const double *x, const double *y, const double *z, const double *w,
                     double box, int periodic, int nbins, double rmin, double rmax, int64_t p_begin,
                     int64_t p_end, int64_t *npairs, double *dd, int nthreads)
{
    if (n < 0 || nbins < 1 || !(rmin >= 0.0) || !(rmax > rmin) || !(box > 0.0) || p_begin < 0 ||
        p_end > n || p_begin > p_end)
        return 1;
    const int nb = nbins;
    for (int b = 0; b < nb; b++) {
        npairs[b] = 0;
        dd[b] = 0.0;
    }
    if (n == 0 || p_begin == p_end) return 0;
    int K = oracle_lattice_bits(box, rmax, periodic);
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
    oracle_snap(n, x, box, K, periodic, q);
    oracle_snap(n, y, box, K, periodic, q + n);
    oracle_snap(n, z, box, K, periodic, q + 2 * n);
    oracle_thresholds(nb, rmin, rmax, box, K, T);
    problem P = {n, q, q + n, q + 2 * n, w, K, periodic, nb, 0, T};

    /* fixed chunks of primaries, merged in order: the result does not depend on threads */
    const int64_t np = p_end - p_begin;
    const int64_t nchunk = np < ORACLE_CHUNKS ? np : ORACLE_CHUNKS;
    int64_t *cpart = (int64_t *)calloc((size_t)nchunk * nb, sizeof(int64_t));
    double *dpart = (double *)calloc((size_t)nchunk * nb, sizeof(double));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nchunk; c++) {
        int64_t lo = p_begin + np * c / nchunk, hi = p_begin + np * (c + 1) / nchunk;
        for (int64_t p = lo; p < hi; p++)
            for (int64_t j = 0; j < n; j++) {
                if (j == p) continue;
                int64_t d[3];
                int b = pair_bin(&P, p, j, d);
                if (b < 0) continue;
                cpart[c * nb + b] += 1;
                dpart[c * nb + b] += w[p] * w[j];
            }
    }
    for (int64_t c = 0; c < nchunk; c++)
        for (int b = 0; b < nb; b++) {
            npairs[b] += cpart[c * nb + b];
            dd[b] += dpart[c * nb + b];
        }
    free(cpart);
    free(dpart);
    free(q);
    free(T);
    return 0;
}

/*
 * The degenerate (j = k) part of the estimator: triangles whose two legs end on the same
 * secondary. In zeta_l(b, b) = sum_p w_p sum_m |a_lm(p, b)|^2 every secondary j of bin b meets
 * itself once, and by the addition theorem sum_m |Y_lm(u)|^2 = (2l + 1) / (4 pi) for any unit u,
 * so that part is
 *     D_l(b) = (2l + 1) / (4 pi) * sum_p w_p sum_{j in b(p)} w_j^2,
 * to be subtracted from the diagonal by callers who want triangles of distinct points only.
 * Same lattice binning as oracle_zeta. Output D[(lmax+1)][nbins]. Returns 0, or 1 on invalid
 * arguments.
 */
static void degenerate_sums(const problem *P, int64_t p_begin, int64_t p_end, double *S, int nthreads)
{
    const int nb = P->nbins;
    const int64_t np = p_end - p_begin;
    for (int b = 0; b < nb; b++) S[b] = 0.0;
    if (np <= 0) return;
    const int64_t nchunk = np < ORACLE_CHUNKS ? np : ORACLE_CHUNKS;
    double *part = (double *)calloc((size_t)nchunk * nb, sizeof(double));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nchunk; c++) {
        int64_t lo = p_begin + np * c / nchunk, hi = p_begin + np * (c + 1) / nchunk;
        for (int64_t p = lo; p < hi; p++)
            for (int64_t j = 0; j < P->n; j++) {
                if (j == p) continue;
                int64_t d[3];
                int b = pair_bin(P, p, j, d);
                if (b < 0) continue;
                part[c * nb + b] += P->w[p] * P->w[j] * P->w[j];
            }
    }
    for (int64_t c = 0; c < nchunk; c++)
        for (int b = 0; b < nb; b++) S[b] += part[c * nb + b];
    free(part);
}

int oracle_degenerate(int64_t n, const double *x, const double *y, const double *z, const double *w, double box,
                      int periodic, int nbins, double rmin, double rmax, int lmax, int64_t p_begin, int64_t p_end,
                      double *D, int nthreads)
{
    if (n < 0 || nbins < 1 || lmax < 0 || !(rmin >= 0.0) || !(rmax > rmin) || !(box > 0.0) || p_begin < 0 ||
        p_end > n || p_begin > p_end || !w)
        return 1;
    const int nb = nbins;
    for (int i = 0; i < (lmax + 1) * nb; i++) D[i] = 0.0;
    if (n == 0 || p_begin == p_end) return 0;
    int K = oracle_lattice_bits(box, rmax, periodic);
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
    double *S = (double *)malloc(sizeof(double) * (size_t)nb);
    oracle_snap(n, x, box, K, periodic, q);
    oracle_snap(n, y, box, K, periodic, q + n);
    oracle_snap(n, z, box, K, periodic, q + 2 * n);
    oracle_thresholds(nb, rmin, rmax, box, K, T);
    problem P = {n, q, q + n, q + 2 * n, w, K, periodic, nb, lmax, T};
    degenerate_sums(&P, p_begin, p_end, S, nthreads);
    for (int l = 0; l <= lmax; l++)
        for (int b = 0; b < nb; b++) D[l * nb + b] = (2.0 * l + 1.0) / (4.0 * 3.14159265358979323846) * S[b];
    free(S);
    free(q);
    free(T);
    return 0;
}

/* Legendre polynomials P_0..P_lmax at x (Bonnet recurrence). */
static void legendre_all(int lmax, double x, double *P)
{
    P[0] = 1.0;
    if (lmax >= 1) P[1] = x;
    for (int l = 2; l <= lmax; l++) P[l] = ((2.0 * l - 1.0) * x * P[l - 1] - (l - 1.0) * P[l - 2]) / l;
}

/* Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n). */
static void gauss_legendre(int n, double *x, double *wt)
{
    for (int i = 0; i < n; i++) {
        double t = cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; k++) {
                double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        x[i] = t;
        wt[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

/*
 * Edge correction of the Legendre multipoles (Slepian & Eisenstein 2015, cited in the paper's
 * Features section; the paper gives no formula): with N the multipoles of the data-minus-randoms
 * field and R those of the (weighted) randoms, the corrected 3PCF is zeta(mu) = N(mu) / R(mu)
 * for every bin pair. In Legendre coefficients, N_L = sum_l'' M_{L l''} zeta_l'' R_0 with
 *     M_{L l''} = (2L + 1)/2 * integral_{-1}^{1} P_L(mu) P_l''(mu) sum_l' f_l' P_l'(mu) dmu,
 *     f_l' = R_l' / R_0,
 * truncated at lmax, and zeta solves M zeta = N / R_0. The integral is taken here by 32-point
 * Gauss-Legendre quadrature, exact for the integrand's degree (at most 3 lmax <= 48), and the
 * system is solved by Gaussian elimination with partial pivoting. The zeta_l of the library are
 * (2l + 1)/(4 pi) times the Legendre sums, the same factor for N and R, so they enter as they are.
 * Arrays are [ncat][(lmax+1)][nbins][nbins]; bin pairs with R_0 = 0 give 0.
 * Returns 0, or 1 on invalid arguments.
 */
int oracle_edge_correct(int ncat, int lmax, int nbins, const double *N, const double *R, double *zeta)
{
    if (ncat < 1 || lmax < 0 || lmax > ORACLE_LMAX_CAP || nbins < 1) return 1;
    enum { NQ = 32 }; /* exact for polynomial integrands of degree <= 63 */
    double xq[NQ], wq[NQ], Pq[NQ][ORACLE_LMAX_CAP + 1];
    gauss_legendre(NQ, xq, wq);
    for (int i = 0; i < NQ; i++) legendre_all(lmax, xq[i], Pq[i]);
    const int L1 = lmax + 1, nb = nbins;
    double M[ORACLE_LMAX_CAP + 1][ORACLE_LMAX_CAP + 2];
    for (int c = 0; c < ncat; c++)
        for (int b1 = 0; b1 < nb; b1++)
            for (int b2 = 0; b2 < nb; b2++) {
                const size_t base = (size_t)c * L1 * nb * nb + (size_t)b1 * nb + b2;
#define AT(arr, l) arr[base + (size_t)(l) * nb * nb]
                const double R0 = AT(R, 0);
                if (R0 == 0.0) {
                    for (int l = 0; l < L1; l++) AT(zeta, l) = 0.0;
                    continue;
                }
                /* R(mu) / R_0 at the nodes */
                double g[NQ];
                for (int i = 0; i < NQ; i++) {
                    double s = 0.0;
                    for (int l = 0; l < L1; l++) s += AT(R, l) / R0 * Pq[i][l];
                    g[i] = s;
                }
                for (int L = 0; L < L1; L++) {
                    for (int l2 = 0; l2 < L1; l2++) {
                        double s = 0.0;
                        for (int i = 0; i < NQ; i++) s += wq[i] * Pq[i][L] * Pq[i][l2] * g[i];
                        M[L][l2] = 0.5 * (2.0 * L + 1.0) * s;
                    }
                    M[L][L1] = AT(N, L) / R0;
                }
                /* Gaussian elimination with partial pivoting on the augmented matrix */
                for (int k = 0; k < L1; k++) {
                    int piv = k;
                    for (int r = k + 1; r < L1; r++)
                        if (fabs(M[r][k]) > fabs(M[piv][k])) piv = r;
                    for (int j = 0; j <= L1; j++) {
                        double t = M[k][j];
                        M[k][j] = M[piv][j];
                        M[piv][j] = t;
                    }
                    for (int r = k + 1; r < L1; r++) {
                        double f = M[r][k] / M[k][k];
                        for (int j = k; j <= L1; j++) M[r][j] -= f * M[k][j];
                    }
                }
                for (int k = L1 - 1; k >= 0; k--) {
                    double s = M[k][L1];
                    for (int j = k + 1; j < L1; j++) s -= M[k][j] * AT(zeta, j);
                    AT(zeta, k) = s / M[k][k];
                }
#undef AT
            }
    return 0;
}

/*
 * Edge correction on the sphere (masked maps). The paper lists edge corrections for regions that
 * are not the full sky (Features section, citing Slepian & Eisenstein 2015 for the construction);
 * its 2D counterpart for the multipoles of the position angle, a reading since the paper gives no
 * formula: per bin pair the triangle-angle densities of the masked field, N(phi), and of the mask,
 * R(phi), have cosine moments N_m = int N(phi) cos(m phi) dphi (the raw zeta_m) and R_m; writing
 * zeta(phi) = N(phi) / R(phi) = c_0 + 2 sum_{m>=1} c_m cos(m phi),
 *     N_m = sum_{m'} eps_m' c_m' int cos(m phi) cos(m' phi) R(phi) dphi,   eps_0 = 1, eps_m' = 2,
 * truncated at m_max (R_k = 0 above it), solved for c per bin pair; c = N / R_0 when R is
 * isotropic. The coupling integrals are taken here by the trapezoid rule on 64 equispaced angles
 * over R(phi) / R_0 = (1 + 2 sum_k R_k / R_0 cos(k phi)) / (2 pi), exact for these trigonometric
 * polynomials. Arrays [ncat][(mmax+1)][nbins][nbins]; R_0 = 0 gives 0. Returns 0, or 1.
 */
int oracle_edge_correct_sphere(int ncat, int mmax, int nbins, const double *N, const double *R, double *zeta)
{
    if (ncat < 1 || mmax < 0 || mmax > ORACLE_LMAX_CAP || nbins < 1) return 1;
    enum { NQ = 64 };
    const double twopi = 6.283185307179586476925286766559;
    const int M1 = mmax + 1, nb = nbins;
    double A[ORACLE_LMAX_CAP + 1][ORACLE_LMAX_CAP + 2], cq[NQ][ORACLE_LMAX_CAP + 1];
    for (int i = 0; i < NQ; i++)
        for (int m = 0; m < M1; m++) cq[i][m] = cos(m * (twopi * i / NQ));
    for (int c = 0; c < ncat; c++)
        for (int b1 = 0; b1 < nb; b1++)
            for (int b2 = 0; b2 < nb; b2++) {
                const size_t base = (size_t)c * M1 * nb * nb + (size_t)b1 * nb + b2;
#define AT(arr, m) arr[base + (size_t)(m) * nb * nb]
                const double R0 = AT(R, 0);
                if (R0 == 0.0) {
                    for (int m = 0; m < M1; m++) AT(zeta, m) = 0.0;
                    continue;
                }
                double g[NQ];
                for (int i = 0; i < NQ; i++) {
                    double t = 1.0;
                    for (int k = 1; k < M1; k++) t += 2.0 * AT(R, k) / R0 * cq[i][k];
                    g[i] = t / twopi;
                }
                for (int m = 0; m < M1; m++) {
                    for (int mp = 0; mp < M1; mp++) {
                        double t = 0.0;
                        for (int i = 0; i < NQ; i++) t += cq[i][m] * cq[i][mp] * g[i];
                        A[m][mp] = (mp == 0 ? 1.0 : 2.0) * t * (twopi / NQ);
                    }
                    A[m][M1] = AT(N, m) / R0;
                }
                for (int k = 0; k < M1; k++) {
                    int piv = k;
                    for (int r = k + 1; r < M1; r++)
                        if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
                    for (int j = 0; j <= M1; j++) {
                        double t = A[k][j];
                        A[k][j] = A[piv][j];
                        A[piv][j] = t;
                    }
                    for (int r = k + 1; r < M1; r++) {
                        double f = A[r][k] / A[k][k];
                        for (int j = k; j <= M1; j++) A[r][j] -= f * A[k][j];
                    }
                }
                for (int k = M1 - 1; k >= 0; k--) {
                    double t = A[k][M1];
                    for (int j = k + 1; j < M1; j++) t -= A[k][j] * AT(zeta, j);
                    AT(zeta, k) = t / A[k][k];
                }
#undef AT
            }
    return 0;
}

/* ---------------------------------------------------------------- projected fields on the sphere */

/*
 * Projected scalar fields on the unit sphere, the geometry of the paper's main application
 * (convergence maps; Statement of need and Features sections) with the triangle's position angle
 * decomposed in multipoles (Implementation section). Readings where the paper is silent:
 *   - Positions are unit vectors n (FP64), shifted by +2 and snapped to the lattice of the
 *     non-periodic cube [0, 4)^3, K = 25 + floor(log2(4 / c_max)) capped at 31, c = 2 sin(theta / 2)
 *     the chord.
 *   - Angular bins are linear in theta: theta_k = theta_min + k dtheta, theta_nb = theta_max,
 *     with chord thresholds T_k = ceil(fl64(fl64(c_k 2^K / 4)^2)), c_k = 2 sin(theta_k / 2);
 *     a pair is in bin k iff T_k <= R^2 < T_{k+1}, R^2 the exact squared lattice separation.
 *   - Position angle of j around p: phi = atan2(d.e2, d.e1) with d = q_j - q_p (lattice) and the
 *     tangent basis at n_p = unit(q_p s - 2): e1 = unit(z x n_p) (unit(x x n_p) within 1e-6 rad
 *     of the poles), e2 = n_p x e1. zeta_m does not depend on this basis (a rotation of the
 *     basis multiplies both a_m of a product by the same phase).
 *   - a_m(p, b) = sum_{j in b} w_j exp(-i m phi_j),
 *     zeta_m(b1, b2) = sum_p w_p Re[a_m(p, b1) conj(a_m(p, b2))],  0 <= m <= mmax.
 * Output zeta[(mmax+1)][nbins][nbins]; counts (optional) [p_end-p_begin][nbins].
 * Returns 0, or 1 on invalid arguments.
 */
/* Snaps unit vectors (shifted by +2) and sets the chord thresholds; returns K. */
static int sphere_setup(int64_t n, const double *x, const double *y, const double *z, int nb, double theta_min,
                        double theta_max, int64_t *q, uint64_t *T)
{
    const double box = 4.0;
    const int K = oracle_lattice_bits(box, 2.0 * sin(0.5 * theta_max), 0);
    const double sc = lattice_scale(box, K);
    for (int64_t i = 0; i < n; i++) {
        const double v[3] = {x[i], y[i], z[i]};
        for (int a = 0; a < 3; a++) q[a * n + i] = snap(v[a] + 2.0, sc, K, 0);
    }
    const double dth = (theta_max - theta_min) / nb;
    for (int k = 0; k <= nb; k++) {
        const double th = (k == nb) ? theta_max : theta_min + k * dth;
        const double v = 2.0 * sin(0.5 * th) * sc;
        T[k] = (uint64_t)ceil(v * v);
    }
    return K;
}

/* One pivot on the sphere at lattice point qp (weight wp) against every point but `skip`: its
 * a_m over all bins and its contribution to zeta (added into z); counts and pairs as in 3D.
 * s = 1 / scale. */
static void sphere_pivot(int64_t n, const int64_t *q, const double *w, const uint64_t *T, int nb, int mmax,
                         double s, const int64_t qp[3], double wp, int64_t skip, double complex *am,
                         int64_t *cnt, double *z, int64_t *pairs)
{
    const int M1 = mmax + 1;
    memset(am, 0, sizeof(double complex) * (size_t)nb * M1);
    for (int b = 0; b < nb; b++) cnt[b] = 0;
    /* tangent basis at the pivot's lattice position */
    double np_[3] = {qp[0] * s - 2.0, qp[1] * s - 2.0, qp[2] * s - 2.0};
    const double nn = sqrt(np_[0] * np_[0] + np_[1] * np_[1] + np_[2] * np_[2]);
    for (int a = 0; a < 3; a++) np_[a] /= nn;
    double e1[3] = {-np_[1], np_[0], 0.0}; /* z x n */
    double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1]);
    if (l1 < 1e-6) { /* x x n */
        e1[0] = 0.0;
        e1[1] = -np_[2];
        e1[2] = np_[1];
        l1 = sqrt(e1[1] * e1[1] + e1[2] * e1[2]);
    }
    for (int a = 0; a < 3; a++) e1[a] /= l1;
    const double e2[3] = {np_[1] * e1[2] - np_[2] * e1[1], np_[2] * e1[0] - np_[0] * e1[2],
                          np_[0] * e1[1] - np_[1] * e1[0]};
    for (int64_t j = 0; j < n; j++) {
        if (j == skip) continue;
        int64_t d[3];
        for (int a = 0; a < 3; a++) d[a] = q[a * n + j] - qp[a];
        const uint64_t R2 = (uint64_t)(d[0] * d[0]) + (uint64_t)(d[1] * d[1]) + (uint64_t)(d[2] * d[2]);
        if (R2 == 0 || R2 < T[0] || R2 >= T[nb]) continue;
        int b = 0;
        while (b + 1 < nb && R2 >= T[b + 1]) b++;
        const double t1 = d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2];
        const double t2 = d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2];
        const double phi = atan2(t2, t1);
        for (int m = 0; m <= mmax; m++) am[b * M1 + m] += w[j] * cexp(-I * (m * phi));
        cnt[b]++;
        (*pairs)++;
    }
    for (int m = 0; m <= mmax; m++)
        for (int b1 = 0; b1 < nb; b1++)
            for (int b2 = 0; b2 < nb; b2++)
                z[((size_t)m * nb + b1) * nb + b2] += wp * creal(am[b1 * M1 + m] * conj(am[b2 * M1 + m]));
}

int oracle_zeta_sphere(int64_t n, const double *x, const double *y, const double *z, const double *w, int nbins,
                       double theta_min, double theta_max, int mmax, int64_t p_begin, int64_t p_end,
                       double *zeta, int64_t *counts, int64_t *npairs_out, int nthreads)
{
    if (n < 0 || nbins < 1 || mmax < 0 || !(theta_min >= 0.0) || !(theta_max > theta_min) ||
        !(theta_max <= 3.14159265358979323846) || p_begin < 0 || p_end > n || p_begin > p_end)
        return 1;
    const int nb = nbins, M1 = mmax + 1;
    const size_t zsize = (size_t)M1 * nb * nb;
    memset(zeta, 0, sizeof(double) * zsize);
    if (npairs_out) *npairs_out = 0;
    if (n == 0 || p_begin == p_end) return 0;
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
    const int K = sphere_setup(n, x, y, z, nb, theta_min, theta_max, q, T);
    const double s = 1.0 / lattice_scale(4.0, K);
    const int64_t np = p_end - p_begin;
    const int64_t nchunk = np < ORACLE_CHUNKS ? np : ORACLE_CHUNKS;
    double *part = (double *)calloc((size_t)nchunk * zsize, sizeof(double));
    int64_t *pairs = (int64_t *)calloc((size_t)nchunk, sizeof(int64_t));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double complex *am = (double complex *)malloc(sizeof(double complex) * (size_t)nb * M1);
        int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < nchunk; c++) {
            int64_t lo = p_begin + np * c / nchunk, hi = p_begin + np * (c + 1) / nchunk;
            for (int64_t p = lo; p < hi; p++) {
                const int64_t qp[3] = {q[p], q[n + p], q[2 * n + p]};
                sphere_pivot(n, q, w, T, nb, mmax, s, qp, w[p], p, am, cnt, part + (size_t)c * zsize, &pairs[c]);
                if (counts)
                    for (int b = 0; b < nb; b++) counts[(p - p_begin) * nb + b] = cnt[b];
            }
        }
        free(am);
        free(cnt);
    }
    int64_t total = 0;
    for (int64_t c = 0; c < nchunk; c++) {
        for (size_t k = 0; k < zsize; k++) zeta[k] += part[(size_t)c * zsize + k];
        total += pairs[c];
    }
    if (npairs_out) *npairs_out = total;
    free(part);
    free(pairs);
    free(q);
    free(T);
    return 0;
}


/* ---------------------------------------------------------------- shared pivots (approximate) */

/*
 * Approximate pivot sharing (Implementation section: spatially close pivots share one neighbour
 * list, closeness set by a pivot length scale that defaults to the mean separation). Reading,
 * since the paper gives no formula:
 *   - pivots are grouped by a cubic pivot cell of Hq = max(1, floor(h * 2^K / L)) lattice units:
 *     the group of lattice point q is (floor(qx/Hq), floor(qy/Hq), floor(qz/Hq));
 *   - every non-empty group g becomes one pivot at X_g = round-half-up of the mean lattice position
 *     of its members, per axis (2 sum q + n_g) div (2 n_g), with weight W_g = sum of its members'
 *     weights (input order);
 *   - the pivot's multipoles use every point as a secondary (pairs at zero separation skipped):
 *         zeta~_l(b1, b2) = sum_g W_g sum_m a_lm(X_g, b1) conj(a_lm(X_g, b2)).
 * Groups are visited in (gz, gy, gx) order. Outputs: zeta as oracle_zeta; ngroups; optionally the
 * group pivots (gq[3][n], gw[n], first ngroups entries). Returns 0, or 1 on invalid arguments.
 */
typedef struct {
    int64_t gx, gy, gz, idx;
} group_key;

static int cmp_group_key(const void *a, const void *b)
{
    const group_key *u = (const group_key *)a, *v = (const group_key *)b;
    if (u->gz != v->gz) return u->gz < v->gz ? -1 : 1;
    if (u->gy != v->gy) return u->gy < v->gy ? -1 : 1;
    if (u->gx != v->gx) return u->gx < v->gx ? -1 : 1;
    return u->idx < v->idx ? -1 : (u->idx > v->idx);
}

/* Groups the lattice points q[3][n] by pivot cells of Hq lattice units, in (gz, gy, gx) order;
 * writes each group's pivot (round-half-up mean lattice position, pq[3][n]) and summed weight
 * (members in input order, pw[n]); returns the number of groups. */
static int64_t build_groups(int64_t n, const int64_t *q, const double *w, int64_t Hq, int64_t *pq, double *pw)
{
    group_key *keys = (group_key *)malloc(sizeof(group_key) * (size_t)n);
    for (int64_t i = 0; i < n; i++) {
        keys[i].gx = q[i] / Hq;
        keys[i].gy = q[n + i] / Hq;
        keys[i].gz = q[2 * n + i] / Hq;
        keys[i].idx = i;
    }
    qsort(keys, (size_t)n, sizeof(group_key), cmp_group_key);
    int64_t G = 0;
    for (int64_t a = 0; a < n;) {
        int64_t b = a;
        int64_t sum[3] = {0, 0, 0};
        double W = 0.0;
        while (b < n && keys[b].gx == keys[a].gx && keys[b].gy == keys[a].gy && keys[b].gz == keys[a].gz) {
            const int64_t i = keys[b].idx;
            sum[0] += q[i];
            sum[1] += q[n + i];
            sum[2] += q[2 * n + i];
            b++;
        }
        /* weights in input order: members were sorted by index within the group */
        for (int64_t k = a; k < b; k++) W += w[keys[k].idx];
        const int64_t cnt = b - a;
        for (int ax = 0; ax < 3; ax++) pq[ax * n + G] = (2 * sum[ax] + cnt) / (2 * cnt);
        pw[G] = W;
        G++;
        a = b;
    }
    free(keys);
    return G;
}

int oracle_zeta_pivots(int64_t n, const double *x, const double *y, const double *z, const double *w,
                       double box, int periodic, int nbins, double rmin, double rmax, int lmax, double h,
                       double *zeta, int64_t *ngroups_out, int64_t *npairs_out, int64_t *gq, double *gw,
                       int nthreads)
{
    if (n < 0 || nbins < 1 || lmax < 0 || lmax > ORACLE_LMAX_CAP || !(rmin >= 0.0) || !(rmax > rmin) ||
        !(box > 0.0) || !(h > 0.0))
        return 1;
    const int nb = nbins, nc = (lmax + 1) * (lmax + 1);
    const size_t zsize = (size_t)(lmax + 1) * nb * nb;
    memset(zeta, 0, sizeof(double) * zsize);
    *ngroups_out = 0;
    if (npairs_out) *npairs_out = 0;
    if (n == 0) return 0;
    const int K = oracle_lattice_bits(box, rmax, periodic);
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
    oracle_snap(n, x, box, K, periodic, q);
    oracle_snap(n, y, box, K, periodic, q + n);
    oracle_snap(n, z, box, K, periodic, q + 2 * n);
    oracle_thresholds(nb, rmin, rmax, box, K, T);
    problem P = {n, q, q + n, q + 2 * n, w, K, periodic, nb, lmax, T};

    int64_t Hq = (int64_t)floor(h * lattice_scale(box, K));
    if (Hq < 1) Hq = 1;
    int64_t *pq = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    double *pw = (double *)malloc(sizeof(double) * (size_t)n);
    const int64_t G = build_groups(n, q, w, Hq, pq, pw);
    *ngroups_out = G;
    if (gq)
        for (int64_t g = 0; g < G; g++)
            for (int ax = 0; ax < 3; ax++) gq[ax * n + g] = pq[ax * n + g];
    if (gw)
        for (int64_t g = 0; g < G; g++) gw[g] = pw[g];

    const int64_t nchunk = G < ORACLE_CHUNKS ? G : ORACLE_CHUNKS;
    double *part = (double *)calloc((size_t)nchunk * zsize, sizeof(double));
    int64_t *pairs = (int64_t *)calloc((size_t)nchunk, sizeof(int64_t));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double complex *alm = (double complex *)malloc(sizeof(double complex) * (size_t)nb * nc);
        double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)nc);
        int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < nchunk; c++) {
            const int64_t lo = G * c / nchunk, hi = G * (c + 1) / nchunk;
            for (int64_t g = lo; g < hi; g++) {
                const int64_t qp[3] = {pq[g], pq[n + g], pq[2 * n + g]};
                one_pivot(&P, qp, pw[g], -1, alm, Y, part + (size_t)c * zsize, cnt, &pairs[c]);
            }
        }
        free(alm);
        free(Y);
        free(cnt);
    }
    int64_t total = 0;
    for (int64_t c = 0; c < nchunk; c++) {
        for (size_t k = 0; k < zsize; k++) zeta[k] += part[(size_t)c * zsize + k];
        total += pairs[c];
    }
    if (npairs_out) *npairs_out = total;
    free(part);
    free(pairs);
    free(pq);
    free(pw);
    free(q);
    free(T);
    return 0;
}

/*
 * Shared pivots on the sphere: the grouping of oracle_zeta_pivots applied to the sphere's lattice
 * (unit vectors shifted by +2, cube of side 4, K from the largest chord), pivot cell h in the
 * cube's units (the mean pixel separation sqrt(4 pi / n) for a full-sky map); each group's pivot
 * sits at the rounded mean lattice position of its members (just inside the sphere), its tangent
 * basis is taken at unit(X s - 2) and its angles and chord bins from the lattice displacements,
 * exactly as for a point; zeta~_m = sum_g W_g Re[a_m(X_g, b1) conj(a_m(X_g, b2))].
 */
int oracle_zeta_sphere_pivots(int64_t n, const double *x, const double *y, const double *z, const double *w,
                              int nbins, double theta_min, double theta_max, int mmax, double h, double *zeta,
                              int64_t *ngroups_out, int64_t *npairs_out, int nthreads)
{
    if (n < 0 || nbins < 1 || mmax < 0 || !(theta_min >= 0.0) || !(theta_max > theta_min) ||
        !(theta_max <= 3.14159265358979323846) || !(h > 0.0))
        return 1;
    const int nb = nbins, M1 = mmax + 1;
    const size_t zsize = (size_t)M1 * nb * nb;
    memset(zeta, 0, sizeof(double) * zsize);
    *ngroups_out = 0;
    if (npairs_out) *npairs_out = 0;
    if (n == 0) return 0;
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
    const int K = sphere_setup(n, x, y, z, nb, theta_min, theta_max, q, T);
    const double sc = lattice_scale(4.0, K), s = 1.0 / sc;
    int64_t Hq = (int64_t)floor(h * sc);
    if (Hq < 1) Hq = 1;
    int64_t *pq = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    double *pw = (double *)malloc(sizeof(double) * (size_t)n);
    const int64_t G = build_groups(n, q, w, Hq, pq, pw);
    *ngroups_out = G;
    const int64_t nchunk = G < ORACLE_CHUNKS ? G : ORACLE_CHUNKS;
    double *part = (double *)calloc((size_t)nchunk * zsize, sizeof(double));
    int64_t *pairs = (int64_t *)calloc((size_t)nchunk, sizeof(int64_t));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double complex *am = (double complex *)malloc(sizeof(double complex) * (size_t)nb * M1);
        int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < nchunk; c++) {
            const int64_t lo = G * c / nchunk, hi = G * (c + 1) / nchunk;
            for (int64_t g = lo; g < hi; g++) {
                const int64_t qp[3] = {pq[g], pq[n + g], pq[2 * n + g]};
                sphere_pivot(n, q, w, T, nb, mmax, s, qp, pw[g], -1, am, cnt, part + (size_t)c * zsize, &pairs[c]);
            }
        }
        free(am);
        free(cnt);
    }
    int64_t total = 0;
    for (int64_t c = 0; c < nchunk; c++) {
        for (size_t k = 0; k < zsize; k++) zeta[k] += part[(size_t)c * zsize + k];
        total += pairs[c];
    }
    if (npairs_out) *npairs_out = total;
    free(part);
    free(pairs);
    free(pq);
    free(pw);
    free(q);
    free(T);
    return 0;
}

/*
 * The degenerate (j = k) part of zeta_m on the sphere: |exp(-i m phi)|^2 = 1, so for every m
 *     D_m(b) = sum_p w_p sum_{j in b(p)} w_j^2,
 * the part of zeta_m(b, b) from one secondary on both legs. Same lattice and chord thresholds
 * as oracle_zeta_sphere. Output D[(mmax+1)][nbins]. Returns 0, or 1 on invalid arguments.
 */
int oracle_degenerate_sphere(int64_t n, const double *x, const double *y, const double *z, const double *w,
                             int nbins, double theta_min, double theta_max, int mmax, int64_t p_begin,
                             int64_t p_end, double *D, int nthreads)
{
    if (n < 0 || nbins < 1 || mmax < 0 || !(theta_min >= 0.0) || !(theta_max > theta_min) ||
        !(theta_max <= 3.14159265358979323846) || p_begin < 0 || p_end > n || p_begin > p_end || !w)
        return 1;
    const int nb = nbins;
    for (int i = 0; i < (mmax + 1) * nb; i++) D[i] = 0.0;
    if (n == 0 || p_begin == p_end) return 0;
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)n);
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
    double *S = (double *)malloc(sizeof(double) * (size_t)nb);
    const int K = sphere_setup(n, x, y, z, nb, theta_min, theta_max, q, T);
    problem P = {n, q, q + n, q + 2 * n, w, K, 0, nb, mmax, T};
    degenerate_sums(&P, p_begin, p_end, S, nthreads);
    for (int m = 0; m <= mmax; m++)
        for (int b = 0; b < nb; b++) D[m * nb + b] = S[b];
    free(S);
    free(q);
    free(T);
    return 0;
}
