/*
 * The library driven from plain C through include/tpcf.h, with no Python in the process: the C
 * engine on its own, as the paper's C engine is (Implementation section).
 *
 *   c_api_demo validate              argument and state errors that need no device
 *   c_api_demo compute IN OUT        IN: int64 n, then n FP64 x, n y, n z (native byte order);
 *                                    computes zeta_l for 8 bins [4, 30), l_max = 4, periodic
 *                                    box 100, FP64, host memory; writes the (l_max+1) x 8 x 8
 *                                    FP64 values to OUT and prints the pair count
 *
 * Exit status 0 on success; otherwise the number of the failed step.
 */
#include <stdio.h>
#include <stdlib.h>

#include "tpcf.h"

static int expect(int rc, int want, int step, tpcf_ctx* c)
{
    if (rc != want) {
        fprintf(stderr, "step %d: status %d, expected %d (%s)\n", step, rc, want, c ? tpcf_last_error(c) : "");
        return step;
    }
    return 0;
}

static int validate(void)
{
    tpcf_ctx* c = NULL;
    int e;
    if ((e = expect(tpcf_create(NULL, 0, NULL), TPCF_E_INVALID_ARG, 1, NULL))) return e;
    if ((e = expect(tpcf_create(&c, 0, NULL), TPCF_OK, 2, NULL))) return e;
    if ((e = expect(tpcf_set_bins(c, 0, 1.0, 2.0, 3), TPCF_E_INVALID_ARG, 3, c))) return e;
    if ((e = expect(tpcf_set_bins(c, 4, 2.0, 1.0, 3), TPCF_E_INVALID_ARG, 4, c))) return e;
    if ((e = expect(tpcf_set_bins(c, 4, 1.0, 2.0, TPCF_MAX_LMAX + 1), TPCF_E_INVALID_ARG, 5, c))) return e;
    if ((e = expect(tpcf_set_precision(c, 9), TPCF_E_INVALID_ARG, 6, c))) return e;
    if ((e = expect(tpcf_set_tuning(c, -1.0, 0, 0), TPCF_E_INVALID_ARG, 7, c))) return e;
    double zeta[1];
    if ((e = expect(tpcf_compute_zeta(c, zeta, TPCF_MEM_HOST), TPCF_E_STATE, 8, c))) return e;
    if ((e = expect(tpcf_set_bins(c, 4, 1.0, 2.0, 3), TPCF_OK, 9, c))) return e;
    if ((e = expect(tpcf_compute_zeta(c, zeta, TPCF_MEM_HOST), TPCF_E_STATE, 10, c))) return e;
    if ((e = expect(tpcf_set_phase_aligned(c, 3), TPCF_E_INVALID_ARG, 11, c))) return e;
    if ((e = expect(tpcf_set_deterministic(c, 2), TPCF_E_INVALID_ARG, 12, c))) return e;
    if ((e = expect(tpcf_set_deterministic(c, 1), TPCF_OK, 13, c))) return e;
    tpcf_destroy(c);
    tpcf_destroy(NULL);
    printf("validate: ok (%s)\n", tpcf_version());
    return 0;
}

static int compute(const char* in, const char* out)
{
    FILE* f = fopen(in, "rb");
    if (!f) return 20;
    int64_t n = 0;
    if (fread(&n, sizeof n, 1, f) != 1 || n < 0) return 21;
    double* xyz = (double*)malloc(sizeof(double) * (size_t)(3 * n + 1));
    if (!xyz || fread(xyz, sizeof(double), (size_t)(3 * n), f) != (size_t)(3 * n)) return 22;
    fclose(f);
    const int nb = 8, L = 4;
    double zeta[(4 + 1) * 8 * 8];
    tpcf_ctx* c = NULL;
    int e;
    if ((e = expect(tpcf_create(&c, 0, NULL), TPCF_OK, 23, NULL))) return e;
    if ((e = expect(tpcf_set_bins(c, nb, 4.0, 30.0, L), TPCF_OK, 24, c))) return e;
    if ((e = expect(tpcf_set_precision(c, TPCF_PREC_FP64), TPCF_OK, 25, c))) return e;
    if ((e = expect(tpcf_set_catalog(c, n, xyz, xyz + n, xyz + 2 * n, NULL, 100.0, 1, TPCF_MEM_HOST), TPCF_OK, 26,
                    c)))
        return e;
    if ((e = expect(tpcf_compute_zeta(c, zeta, TPCF_MEM_HOST), TPCF_OK, 27, c))) return e;
    tpcf_stats st;
    if ((e = expect(tpcf_get_stats(c, &st), TPCF_OK, 28, c))) return e;
    tpcf_destroy(c);
    free(xyz);
    f = fopen(out, "wb");
    if (!f || fwrite(zeta, sizeof(double), (size_t)((L + 1) * nb * nb), f) != (size_t)((L + 1) * nb * nb)) return 29;
    fclose(f);
    printf("compute: ok, %lld pairs\n", (long long)st.n_pairs);
    return 0;
}

int main(int argc, char** argv)
{
    if (argc == 2 && argv[1][0] == 'v') return validate();
    if (argc == 4 && argv[1][0] == 'c') return compute(argv[2], argv[3]);
    fprintf(stderr, "usage: %s validate | compute IN OUT\n", argv[0]);
    return 64;
}
