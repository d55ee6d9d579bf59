/*
 * tpcf.h -- C ABI of the MI355X (gfx950) three-point correlation function multipole library.
 *
 * The library computes, for one or many point catalogues, the multipoles of the three-point
 * correlation function in the spherical-harmonic form: for every primary p and every secondary
 * j within [r_min, r_max) of it (found through a cubic cell grid),
 *
 *     a_lm(p, b)     = sum_{j in bin b} w_j conj(Y_lm(unit(x_j - x_p))),       0 <= m <= l <= l_max
 *     zeta_l(b1, b2) = sum_p w_p sum_{m=-l}^{l} a_lm(p, b1) conj(a_lm(p, b2)).
 *
 * This is the harmonic decomposition of the triangle angle that the paper's Implementation
 * section builds its fast estimator on (per pivot: find all neighbours in range, fill the
 * multipole bins), written for 3D positions with spherical harmonics as in the works the paper
 * cites (Szapudi 2004; Slepian & Eisenstein 2015). Fields on the unit sphere, the paper's own
 * workload, use the 2D multipoles of the position angle instead (tpcf_set_sphere_catalog).
 * Beside zeta: the two-point by-product (tpcf_pair_sums), the degenerate j = k term
 * (tpcf_degenerate), edge corrections (tpcf_edge_correct, tpcf_edge_correct_sphere), batches of
 * catalogues in one launch, and an opt-in shared-pivot approximation (tpcf_set_pivot_cell).
 *
 * Conventions fixed by the library (the paper gives no formula):
 *   - Positions are snapped to a lattice of spacing L / 2^K, K = 25 + floor(log2(L / r_max)),
 *     capped at 32 (periodic) / 31 (non-periodic). Separations are exact lattice integers and
 *     bin membership is decided exactly against integer thresholds, so pair counts are exact.
 *   - Bins are linear and half-open: [r_min + k D, r_min + (k+1) D), D = (r_max - r_min)/nbins.
 *   - Periodic boxes use the minimum image and need r_max < L/2.
 *   - Y_lm is orthonormal with the Condon-Shortley phase; the j = k (same secondary on both
 *     legs) term is included (tpcf_degenerate returns it); pairs at zero separation are skipped.
 *   - zeta is written as double [(lmax+1)][nbins][nbins], row-major.
 *
 * Every function returns a status code (TPCF_OK = 0). No C++ exception crosses this boundary.
 * On an error the outputs are left untouched and tpcf_last_error() describes the failure.
 * A context is not thread-safe; use one context per host thread and HIP stream.
 *
 * Memory spaces: TPCF_MEM_HOST pointers are ordinary host memory; the call returns after the
 * data has been consumed (inputs) or written (outputs). TPCF_MEM_DEVICE pointers are device
 * memory on the context's device; they are read/written in order on the context's stream.
 */
#ifndef TPCF_H
#define TPCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpcf_ctx tpcf_ctx;

enum {
    TPCF_OK = 0,
    TPCF_E_INVALID_ARG = 1, /* a value out of its documented range */
    TPCF_E_STATE = 2,       /* a call made before the calls it needs (e.g. compute before set_*) */
    TPCF_E_OUT_OF_MEMORY = 3,
    TPCF_E_DEVICE = 4,      /* a HIP runtime error (message in tpcf_last_error) */
    TPCF_E_UNSUPPORTED = 5
};

enum { TPCF_PREC_FP64 = 0, TPCF_PREC_MIXED = 1 };
enum { TPCF_MEM_HOST = 0, TPCF_MEM_DEVICE = 1 };

#define TPCF_MAX_NBINS 32
#define TPCF_MAX_LMAX 10

/* Run statistics of the last compute call. */
typedef struct tpcf_stats {
    int64_t n_pairs;        /* in-range ordered (primary, secondary) pairs */
    int64_t n_candidates;   /* secondaries tested (cell-grid stencil) */
    int64_t n_primaries;
    double ms_grid;         /* lattice snap + cell-list build (set_catalog / batch) */
    double ms_sweep;        /* pair sweep + contraction kernel */
    double ms_total;        /* whole compute call, device time */
    int cells_per_axis;     /* grid of the first catalogue */
    int waves;              /* persistent waves launched */
    int precision;
    int lmax;
    int nbins;
} tpcf_stats;

/* Tuning picked by tpcf_autotune. */
typedef struct tpcf_tuning {
    double points_per_cell; /* grid density */
    int waves_per_cu;       /* persistent waves per compute unit */
    int scratch_blocks;     /* scratch blocks of 64 secondaries per wave (pair-list length) */
    int candidates;         /* configurations timed */
    double ms_best;         /* sweep time of the sample with the chosen configuration */
    double ms_default;      /* sweep time of the sample with the configuration in force before */
} tpcf_tuning;

/* Library version string, e.g. "tpcf 1.0.0 gfx950". Never NULL. */
const char* tpcf_version(void);

/*
 * Creates a context on HIP device `device` using stream `hip_stream` (a hipStream_t; NULL means
 * the null stream). Every device operation of the context is ordered on that stream. The device
 * is first touched by the first call that needs it, so a context can be created and configured
 * on a machine without a GPU. If the environment variable TPCF_MAX_DEVICE_BYTES holds a byte
 * count, a context never holds more device memory than that: a call that would need more fails
 * with TPCF_E_OUT_OF_MEMORY.
 * Errors: TPCF_E_INVALID_ARG if out is NULL or device < 0; TPCF_E_OUT_OF_MEMORY.
 */
int tpcf_create(tpcf_ctx** out, int device, void* hip_stream);

/* Frees the context and every device buffer it owns. NULL is accepted. */
void tpcf_destroy(tpcf_ctx* ctx);

/*
 * Radial bins and multipole order: the multipole bins a pivot's neighbours fill (paper,
 * Implementation section). nbins in [1, TPCF_MAX_NBINS], 0 <= rmin < rmax (finite),
 * lmax in [0, TPCF_MAX_LMAX]. With a catalogue on the sphere (tpcf_set_sphere_catalog) rmin and
 * rmax are angles in radians (rmax <= pi) and lmax is m_max. Errors: TPCF_E_INVALID_ARG.
 */
int tpcf_set_bins(tpcf_ctx* ctx, int nbins, double rmin, double rmax, int lmax);

/*
 * TPCF_PREC_FP64: FP64 pair sweep, FP64 shells and FP64 MFMA contraction.
 * TPCF_PREC_MIXED: FP32 pair sweep with register partials and Kahan-compensated shell sums,
 * contraction in split-BF16 MFMA with FP32 accumulation per tile, FP64 global reduction.
 * Errors: TPCF_E_INVALID_ARG.
 */
int tpcf_set_precision(tpcf_ctx* ctx, int precision);

/*
 * Optional tuning: target mean points per grid cell (default 8; the grid side in y and z follows
 * from it and the catalogue density, and each such cell is split into up to 4 thinner cells along
 * x), persistent waves per compute unit (default 12, or 8 for the FP64 sweep of a 3D catalogue;
 * capped by what the compute unit's LDS holds), and scratch blocks
 * of 64 secondaries per wave (default 1024 in 3D and 512 on the sphere). A value of 0 keeps the
 * current setting.
 * Errors: TPCF_E_INVALID_ARG for negative or non-finite values, waves_per_cu above 64, or
 * scratch_blocks not a multiple of 64 or above 8192; a compute call with scratch_blocks below
 * 5 x nbins fails with TPCF_E_INVALID_ARG.
 */
int tpcf_set_tuning(tpcf_ctx* ctx, double points_per_cell, int waves_per_cu, int scratch_blocks);

/*
 * Optional device allocator (for example torch's caching allocator). From this call on, every
 * device buffer the context allocates (catalogue staging, grid, sweep scratch, outputs, debug
 * staging) comes from alloc(bytes, user) and goes back through free_(ptr, user); buffers that
 * exist already keep the allocator that made them and are freed by it. alloc must return device
 * memory of the context's device, aligned to at least 256 bytes, or NULL on failure (the call that
 * needed it then fails with TPCF_E_OUT_OF_MEMORY). The library frees a buffer while work that used
 * it may still be queued on the context's stream, so the allocator must follow that stream's order
 * (as a caching allocator bound to the stream does); with plain hipMalloc semantics nothing is
 * needed. The TPCF_MAX_DEVICE_BYTES cap applies as well. alloc = free_ = NULL restores hipMalloc /
 * hipFree for later buffers.
 * Errors: TPCF_E_INVALID_ARG if exactly one of alloc and free_ is NULL.
 */
typedef void* (*tpcf_alloc_fn)(size_t bytes, void* user);
typedef void (*tpcf_free_fn)(void* ptr, void* user);
int tpcf_set_allocator(tpcf_ctx* ctx, tpcf_alloc_fn alloc, tpcf_free_fn free_, void* user);

/*
 * Optional: phase-aligned stencil sweeps (a performance setting; results agree up to the rounding
 * of a different summation order, pair counts are identical). Each wave takes the stencil rows of
 * its primary in a rotated order that starts where the waves in flight currently are, so that they
 * read the same records at about the same time and share them through L2. mode -1 (default):
 * on when the expected neighbourhood of one primary exceeds 2 MiB of records; 0: off; 1: on.
 * Stencils of more than 4096 rows (grids far finer than the search radius) keep their natural
 * order either way.
 * Takes effect at the next compute call. Errors: TPCF_E_INVALID_ARG for another mode.
 */
int tpcf_set_phase_aligned(tpcf_ctx* ctx, int mode);

/*
 * Optional: deterministic mode, for bit-for-bit reproducible results (the same inputs, settings
 * and library give the same bits on every run). Every primary's shells are already fixed by its
 * stencil order; what scheduling changes is how primaries are grouped into contraction tiles and
 * the order in which partial sums meet (the reduction over primaries of the paper's
 * Implementation section is a plain sum, so any order is correct up to rounding). With enable = 1
 * the sweep hands out fixed tiles of consecutive primaries (32 mixed, 16 FP64; a tile never spans
 * two catalogues), writes each tile's zeta contribution and 2PCF weight sums to a slot of its own
 * (device memory: (lmax+1) nbins^2 + nbins doubles per tile, about 1.1 GB for 10^6 points at
 * 20 bins and lmax 10 in mixed precision) and adds the slots in tile order in a second kernel
 * (chunks of 64 tiles, then the chunks of each catalogue), in place of atomic additions;
 * phase-aligned sweeps are off. Applies to tpcf_compute_zeta, tpcf_compute_zeta_range,
 * tpcf_compute_batch, tpcf_compute_sphere_batch and tpcf_degenerate. enable = 0 (default)
 * restores the faster atomic reduction.
 * Takes effect at the next compute call. Errors: TPCF_E_INVALID_ARG for another value; a compute
 * call whose slots do not fit fails with TPCF_E_OUT_OF_MEMORY.
 */
int tpcf_set_deterministic(tpcf_ctx* ctx, int enable);

/*
 * Autotuner for the persistent sweep. On the catalogue(s) staged by the last tpcf_set_catalog,
 * tpcf_set_sphere_catalog or tpcf_compute_batch call, with the current bins and precision, it times
 * the sweep over a sample of primaries (a fraction sample_fraction of all, taken as up to 16 evenly
 * spaced runs of consecutive cell-sorted points, so the sample follows the catalogue's density and
 * keeps the full sweep's neighbour sharing; each configuration timed twice after a warm-up, the
 * faster run kept)
 * for grid densities of 3-48 points per cell (9 values) and 12 and 8 waves per compute unit (the
 * default and the other one), then, at the fastest of those, for half and twice the
 * scratch blocks per wave in use, and keeps the fastest of the 20 configurations as if set by
 * tpcf_set_tuning. sample_fraction in (0, 1]; 0 means
 * 0.05. Results of later compute calls do not depend on the tuning. The call synchronises the
 * context's stream. Stats of the last compute call are kept; its debug output is dropped
 * (tpcf_debug_pair_counts / tpcf_debug_alm return TPCF_E_STATE until the next compute call with
 * debug output enabled). out may be NULL.
 * Errors: TPCF_E_STATE (bins or catalogue missing), TPCF_E_INVALID_ARG (sample_fraction out of
 * range), TPCF_E_OUT_OF_MEMORY, TPCF_E_DEVICE.
 */
int tpcf_autotune(tpcf_ctx* ctx, double sample_fraction, tpcf_tuning* out);

/*
 * One catalogue of n points, the pivots and neighbours of the estimator (paper, Implementation
 * section: every point is a pivot whose neighbours in range fill the bins): positions x, y, z and
 * weights w (w = NULL means unit weights), all
 * FP64 arrays of length n in memory space `memspace`. box is the cube side; periodic != 0 wraps
 * positions into [0, box) and uses minimum images; otherwise every coordinate must lie in
 * [0, box). The positions are copied into library-owned, cell-sorted device buffers (lattice
 * snap + counting-sort cell grid); the caller may free or reuse its arrays when the call
 * returns. The call synchronises the context's stream.
 * Errors: TPCF_E_INVALID_ARG (n < 0, n >= 2^31, box not finite and > 0, a non-finite position
 * or weight, a non-periodic point outside [0, box), NULL arrays with n > 0, periodic with
 * rmax >= box/2 when bins are already set), TPCF_E_OUT_OF_MEMORY, TPCF_E_DEVICE.
 */
int tpcf_set_catalog(tpcf_ctx* ctx, int64_t n, const double* x, const double* y, const double* z,
                     const double* w, double box, int periodic, int memspace);

/*
 * tpcf_set_catalog with FP32 arrays (same meaning, layout, ownership and errors). Each value is
 * widened to FP64 exactly before anything else happens, so the result is that of
 * tpcf_set_catalog on the widened values. Host arrays are widened on the host, device arrays by a
 * kernel on the context's stream.
 */
int tpcf_set_catalog_f32(tpcf_ctx* ctx, int64_t n, const float* x, const float* y, const float* z,
                         const float* w, double box, int periodic, int memspace);

/*
 * One projected scalar field on the unit sphere (the paper's own geometry: pixels or galaxies of
 * a map; Statement of need, Features and Performance sections): n unit vectors x, y, z (FP64,
 * |v|^2 within 1e-6 of 1) with field values w (NULL = unit weights), in `memspace`. Replaces the
 * catalogue of the context; the compute calls then return the 2D multipoles of the position
 * angle phi of each secondary around its primary,
 *
 *     a_m(p, b)      = sum_{j in bin b} w_j exp(-i m phi_pj),                 0 <= m <= m_max,
 *     zeta_m(b1, b2) = sum_p w_p Re[a_m(p, b1) conj(a_m(p, b2))],
 *
 * as double [(m_max+1)][nbins][nbins], with the bins of tpcf_set_bins read as angles: linear,
 * half-open [theta_min + k D, theta_min + (k+1) D) in radians. Conventions: the unit vectors are
 * shifted by +2 and snapped to the lattice of the non-periodic cube [0, 4)^3 with
 * K = 25 + floor(log2(4 / c_max)) (capped at 31) bits, c = 2 sin(theta / 2) the chord; a pair is
 * in bin k iff T_k <= R^2 < T_{k+1}, R^2 the exact squared lattice separation and
 * T_k = ceil(fl(fl(2 sin(theta_k / 2) 2^K / 4)^2)), so pair counts are exact; phi is measured
 * from a tangent basis at the primary's lattice position, which zeta_m does not depend on.
 * Debug a_m (tpcf_debug_alm) has 2 m_max + 1 components per bin: Re a_0, then Re a_m, Im a_m
 * (index 2m - 1, 2m). tpcf_pair_sums reports the angular bins; masked maps are corrected with
 * tpcf_edge_correct_sphere (tpcf_edge_correct, the 3D coupling, is refused). The call
 * synchronises the context's stream.
 * Errors: TPCF_E_INVALID_ARG (n < 0, n >= 2^31, NULL arrays with n > 0, a non-finite value, a
 * vector that is not a unit vector, rmax > pi when bins are already set), TPCF_E_OUT_OF_MEMORY,
 * TPCF_E_DEVICE.
 */
int tpcf_set_sphere_catalog(tpcf_ctx* ctx, int64_t n, const double* x, const double* y,
                            const double* z, const double* w, int memspace);

/*
 * tpcf_set_sphere_catalog with FP32 arrays (same meaning, layout, ownership and errors), widened
 * to FP64 exactly first. FP32 unit vectors are unit to about 1e-7 in |v|^2, well within the 1e-6
 * the check allows.
 */
int tpcf_set_sphere_catalog_f32(tpcf_ctx* ctx, int64_t n, const float* x, const float* y, const float* z,
                                const float* w, int memspace);

/*
 * ncat independent maps on the sphere in one persistent launch (the batch form of
 * tpcf_set_sphere_catalog + tpcf_compute_zeta, for many simulated maps): map c holds the unit
 * vectors [offsets[c], offsets[c+1]) of the concatenated FP64 arrays x, y, z and values w (w may
 * be NULL); offsets is a host array; zeta receives [ncat][(m_max+1)][nbins][nbins] doubles in
 * `memspace`. Maps never interact. The batch replaces the context's catalogue; graph capture and
 * replay as for tpcf_compute_batch.
 * Errors: TPCF_E_INVALID_ARG (ncat < 1, offsets not non-decreasing from 0, total points >= 2^31,
 * NULL arrays, a vector that is not a unit vector, rmax > pi), TPCF_E_STATE (bins not set),
 * TPCF_E_UNSUPPORTED (shared pivots set), TPCF_E_OUT_OF_MEMORY, TPCF_E_DEVICE.
 */
int tpcf_compute_sphere_batch(tpcf_ctx* ctx, int ncat, const int64_t* offsets, const double* x,
                              const double* y, const double* z, const double* w, double* zeta,
                              int memspace);

/*
 * zeta for the catalogue set by tpcf_set_catalog: every point is a primary and a secondary; the
 * multipoles of each pivot's neighbours, contracted over m and summed over pivots (paper,
 * Implementation section).
 * zeta has (lmax+1)*nbins*nbins doubles in memory space `memspace`.
 * Errors: TPCF_E_STATE (bins or catalogue missing), TPCF_E_INVALID_ARG (periodic with
 * rmax >= box/2, NULL zeta), TPCF_E_OUT_OF_MEMORY, TPCF_E_DEVICE.
 */
int tpcf_compute_zeta(tpcf_ctx* ctx, double* zeta, int memspace);

/*
 * As tpcf_compute_zeta, but only the points with input index in [p_begin, p_end) are primaries
 * (every point stays a secondary). zeta over disjoint ranges adds up to the full zeta.
 * Errors: as tpcf_compute_zeta, plus TPCF_E_INVALID_ARG for a range outside [0, n].
 */
int tpcf_compute_zeta_range(tpcf_ctx* ctx, int64_t p_begin, int64_t p_end, double* zeta,
                            int memspace);

/*
 * ncat independent catalogues in one persistent launch, each measured as tpcf_compute_zeta does
 * (paper, Implementation section; the paper's engine runs its pivots in parallel over threads,
 * Features section). Catalogue c holds the points
 * [offsets[c], offsets[c+1]) of the concatenated FP64 arrays x, y, z, w (w may be NULL); its box
 * side is box_side[c] and periodic flag periodic[c]. offsets, box_side and periodic are host
 * arrays; x, y, z, w live in `memspace`; zeta receives [ncat][(lmax+1)][nbins][nbins] doubles in
 * `memspace`. Catalogues never interact. The batch replaces the catalogue set by
 * tpcf_set_catalog. On a non-null stream the device sequence (grid build, clears, persistent
 * sweep) is captured in a HIP graph on first use for a given batch shape and replayed by later
 * calls of the same shape (environment TPCF_GRAPH=0 disables this); stats then report the
 * whole graph as ms_sweep.
 * Errors: TPCF_E_INVALID_ARG (ncat < 1, offsets not non-decreasing from 0, total points >= 2^31,
 * any per-catalogue error of tpcf_set_catalog), TPCF_E_STATE, TPCF_E_OUT_OF_MEMORY,
 * TPCF_E_DEVICE.
 */
int tpcf_compute_batch(tpcf_ctx* ctx, int ncat, const int64_t* offsets, const double* x,
                       const double* y, const double* z, const double* w,
                       const double* box_side, const int* periodic, double* zeta, int memspace);

/*
 * tpcf_compute_batch for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): same arguments, meaning, layout,
 * ownership and results, but the call allocates nothing. Every device buffer it needs (staged
 * positions, cell grid, per-wave pair lists and tiles, zeta and pair-sum partials, deterministic
 * tiles) is a slice of one static device array of TPCF_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on each GPU it runs on, from its first kernel launch there until the process ends; the
 * caller's allocator and TPCF_MAX_DEVICE_BYTES do not apply. The sweep runs as many waves as that
 * array holds beside the batch's other buffers (with 256 scratch blocks per wave unless
 * tpcf_set_tuning sets them), so large batches run with fewer waves than tpcf_compute_batch. No HIP
 * graph is captured. The call returns after the context's stream has drained. The context's own
 * buffers, catalogue and grid are left as they were; afterwards tpcf_get_stats describes this call,
 * while tpcf_pair_sums and the debug calls fail with TPCF_E_STATE until the next compute call.
 * Every call on one GPU shares that GPU's array and overwrites it: calls that overlap in time on
 * one GPU (several host threads, or contexts on different streams) race and must be serialised
 * by the caller.
 * Errors: as tpcf_compute_batch; TPCF_E_OUT_OF_MEMORY when the batch does not fit in the array
 * (the message gives the bytes needed).
 */
#define TPCF_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int tpcf_compute_batch_noalloc(tpcf_ctx* ctx, int ncat, const int64_t* offsets, const double* x,
                               const double* y, const double* z, const double* w,
                               const double* box_side, const int* periodic, double* zeta, int memspace);

/*
 * Exact unit-weight pair counts of the last compute call: counts[i][b] (host, int64,
 * n x nbins, input order) is the number of secondaries of primary i in bin b (0 for points that
 * were not primaries). Enable with tpcf_set_debug(ctx, 1) before the compute call.
 * Errors: TPCF_E_STATE if no compute call ran with debug output enabled.
 */
int tpcf_debug_pair_counts(tpcf_ctx* ctx, int64_t* counts);

/*
 * Debug output of the normalised a_lm of the last compute call, host FP64,
 * [n][nbins][(lmax+1)^2] in input order, real components per l: Re a_l0, then Re a_lm, Im a_lm
 * for m = 1..l (index l*l, then l*l + 2m - 1 and l*l + 2m). Enabled by tpcf_set_debug.
 * Errors: TPCF_E_STATE.
 */
int tpcf_debug_alm(tpcf_ctx* ctx, double* alm);

/*
 * The degenerate (j = k) part of the estimator, for the catalogue(s) staged by the last
 * tpcf_set_catalog, tpcf_set_sphere_catalog or batch call, with the current bins: the triangles
 * whose two legs end on the same secondary, which zeta includes on its diagonal b1 = b2 (the
 * paper's estimator leaves their treatment open; they are part of sum_m |a_lm|^2). In 3D
 *     D_l(b) = (2l + 1) / (4 pi) * sum_p w_p sum_{j in b(p)} w_j^2
 * (the addition theorem: sum_m |Y_lm(u)|^2 = (2l + 1) / (4 pi)); on the sphere
 *     D_m(b) = sum_p w_p sum_{j in b(p)} w_j^2 for every m.
 * zeta_l(b, b) - D_l(b) is then the sum over triangles of three distinct points. Always the exact
 * estimator (every point a primary, also when shared pivots are set), in FP64: one extra sweep at
 * l_max = 0 with squared secondary weights. The outputs of the last compute call (zeta, pair
 * sums, debug rows, statistics) are left as they are.
 * D: [ncat][(lmax+1)][nbins] row-major, FP64, caller-owned, in `memspace`.
 * Errors: TPCF_E_STATE before tpcf_set_bins or without a catalogue; TPCF_E_INVALID_ARG for a NULL
 * D or an unknown memspace or the periodic range check of tpcf_compute_zeta; TPCF_E_OUT_OF_MEMORY.
 */
int tpcf_degenerate(tpcf_ctx* ctx, double* D, int memspace);

/*
 * Two-point by-product of the last compute call (tpcf_compute_zeta, _range or _batch), per
 * catalogue c and radial bin b, over that call's primaries and all secondaries:
 *     npairs[c][b] = ordered (primary, secondary) pairs in bin b, exact;
 *     dd[c][b]     = sum over those pairs of w_p w_j (FP64 sum of per-primary bin sums, which
 *                    are the M_00 moments of the shells: FP32 with compensation in the mixed
 *                    path, FP64 in the FP64 path).
 * This is the weighted pair count DD(r) of the two-point function the paper computes alongside
 * the 3PCF (Introduction and Features sections). npairs and dd are host arrays of `capacity`
 * elements each (either may be NULL); ncat x nbins of the last compute call are written, row-major.
 * The call synchronises the context's stream.
 * Errors: TPCF_E_STATE before the first compute call; TPCF_E_INVALID_ARG if capacity is below
 * ncat x nbins.
 */
int tpcf_pair_sums(tpcf_ctx* ctx, int64_t capacity, int64_t* npairs, double* dd);

/*
 * Edge correction for data-minus-randoms fields (Slepian & Eisenstein 2015, the estimator the
 * paper's Features section cites): N holds the multipoles of the data-minus-randoms field and R
 * those of the randoms alone (weighted as in N, with the opposite sign), both as returned by the
 * compute calls with the current bins and l_max, [ncat][(lmax+1)][nbins][nbins]. For every
 * catalogue and bin pair, zeta receives the Legendre coefficients of N(mu) / R(mu) truncated at
 * l_max: the solution of M zeta = N / R_0 with M_{L l''} = (2L+1) sum_l' (L l' l''; 0 0 0)^2
 * R_l' / R_0. Bin pairs with R_0 = 0 give 0. All three arrays are in `memspace`; zeta may alias N
 * or R. Device arrays are processed in order on the context's stream; host arrays are copied
 * through the device and the call returns when zeta is written.
 * Errors: TPCF_E_INVALID_ARG (ncat < 1, NULL arrays, unknown memory space), TPCF_E_STATE (bins
 * not set), TPCF_E_UNSUPPORTED (the context holds a catalogue on the sphere: see
 * tpcf_edge_correct_sphere), TPCF_E_OUT_OF_MEMORY, TPCF_E_DEVICE.
 */
int tpcf_edge_correct(tpcf_ctx* ctx, int ncat, const double* N, const double* R, double* zeta,
                      int memspace);

/*
 * Edge correction on the sphere, for maps that do not cover the full sky (the paper's Features
 * section lists edge corrections for such regions). The same construction as tpcf_edge_correct
 * applied to the 2D multipoles of the position angle: N holds zeta_m of the masked map values and
 * R those of the mask (unit weights on the observed pixels), both [ncat][(m_max+1)][nbins][nbins]
 * with the current bins and m_max. Per bin pair, zeta receives the cosine coefficients c_m of
 * N(phi) / R(phi) = c_0 + 2 sum_{m>=1} c_m cos(m phi), truncated at m_max: the solution of
 *     N_m / R_0 = sum_{m'} eps_m' (R_{m+m'} + R_{|m-m'|}) / (2 R_0) c_m',  eps_0 = 1, eps_m' = 2,
 * with R_k = 0 above m_max; for a full-sky (isotropic) mask c = N / R_0. Bin pairs with R_0 = 0
 * give 0. Memory spaces, aliasing and synchronisation as for tpcf_edge_correct.
 * Errors: TPCF_E_INVALID_ARG (ncat < 1, NULL arrays, unknown memory space), TPCF_E_STATE (bins
 * not set), TPCF_E_OUT_OF_MEMORY, TPCF_E_DEVICE.
 */
int tpcf_edge_correct_sphere(tpcf_ctx* ctx, int ncat, const double* N, const double* R, double* zeta,
                             int memspace);

/*
 * Shared pivots, an approximation with a speed knob (the paper's Implementation section: spatially
 * close pivots share one neighbour list, closeness set by a pivot length scale that defaults to the
 * mean separation). side > 0: pivots are grouped by cubic pivot cells of Hq = max(1, floor(side *
 * 2^K / L)) lattice units (K and the lattice as for the exact estimator); every occupied cell
 * becomes one pivot at the round-half-up mean lattice position of its members, (2 sum q + n)
 * div (2 n) per axis, with weight W = sum of their weights, and every point stays a secondary:
 *     zeta~_l(b1, b2) = sum_cells W sum_m a_lm(X, b1) conj(a_lm(X, b2)),
 * pairs at zero separation skipped. side < 0 uses the mean separation, L / n^(1/3) in a box and
 * sqrt(4 pi / n) on the sphere; side = 0 (default) is the exact estimator. On the sphere the
 * cells are those of the unit-vector cube (side in its units, about radians at small angles), a
 * pivot sits at its members' rounded mean lattice position (just inside the sphere) and its
 * position angles are measured in the tangent plane at that point's direction. The error falls
 * with the cell side (the tests and the benchmark measure it against the exact estimator); stats
 * report the pivot count as n_primaries. Applies to tpcf_compute_zeta and to the batch calls
 * (tpcf_compute_batch, tpcf_compute_sphere_batch), where every catalogue gets its own pivots, with
 * side in its own units (side < 0: its own mean separation); batches with pivots launch eagerly,
 * not from a graph.
 * The compute call synchronises the context's stream once (to learn the pivot count). The
 * autotuner times the exact sweep, not the shared pivots.
 * Errors: TPCF_E_INVALID_ARG (side not finite). A compute call fails with TPCF_E_UNSUPPORTED for
 * primary ranges, and with TPCF_E_INVALID_ARG when the pivot cells number more than 2^B per axis
 * (B = 21 for one catalogue, floor((63 - ceil(log2 ncat)) / 3) for a batch of ncat) or, on the
 * sphere, are larger than 0.25.
 * Debug output (per-point counts, a_lm) is not kept.
 */
int tpcf_set_pivot_cell(tpcf_ctx* ctx, double side);

/* 0 (default) or 1: keep per-primary pair counts and a_lm of the next compute calls. */
int tpcf_set_debug(tpcf_ctx* ctx, int enable);

/* Statistics of the last compute call. Errors: TPCF_E_INVALID_ARG for NULL pointers. */
int tpcf_get_stats(const tpcf_ctx* ctx, tpcf_stats* out);

/* Text of the last error on ctx ("" if none). Valid until the next call on ctx. */
const char* tpcf_last_error(const tpcf_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* TPCF_H */
