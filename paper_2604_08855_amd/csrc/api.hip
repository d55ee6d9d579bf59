// api.hip -- host side of the library: context, argument validation, lattice and cell-grid set
// up, stencil rows, spherical-harmonic normalisation, launches, HIP-graph replay of batches and
// the extern "C" entry points declared in include/tpcf.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "tpcf.h"
#include "tpcf_internal.h"

namespace tpcf {
hipError_t build_grid(const double* x, const double* y, const double* z, const double* w, uint32_t n,
                      const CatDesc* cats, int ncat, uint32_t ncell, uint4* qtmp, uint32_t* cell, uint32_t* hist,
                      uint32_t* idx_a, uint32_t* idx_b, uint32_t* block_sum, int* err, uint32_t* cell_start,
                      uint4* rec, double* w64, uint32_t* perm, hipStream_t s);
void validate_inputs(const double* x, const double* y, const double* z, const double* w, uint32_t n,
                     const CatDesc* cats, int ncat, int* err, hipStream_t s);
size_t scan_block_count(uint32_t ncell);
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void fill_f64(double* p, double v, size_t n, hipStream_t s);
void widen_f32(const float* in, double* out, size_t n, hipStream_t s);
hipError_t range_tasks(const uint32_t* perm, uint32_t n, uint32_t lo, uint32_t hi, uint32_t* flag, uint32_t* pos,
                       uint32_t* block_sum, uint32_t* list, hipStream_t s);
hipError_t square_weights(const uint4* rec, const double* w64, uint32_t n, uint4* out, double* w2, hipStream_t s);
void unsort_counts(const int32_t* in, const uint32_t* perm, int64_t* out, uint32_t n, int nb, hipStream_t s);
void unsort_alm(const void* in, bool f64, const uint32_t* perm, double* out, uint32_t n, int row, hipStream_t s);
hipError_t launch_sweep(int lmax, bool f64, bool sphere, const SweepArgs& args, int waves, hipStream_t stream);
hipError_t launch_det_reduce(const double* det_out, uint32_t stride, const uint2* chunks, uint32_t nchunk,
                             const uint32_t* cat_chunk, int ncat, uint32_t Z, int nb, double* part1, double* zeta,
                             double* dd, hipStream_t s);
size_t sweep_lds_bytes(int nb, int lmax, bool f64, bool sphere);
size_t sweep_tile_bytes_per_wave(int lmax, int nb, bool f64, bool sphere);
std::vector<double> threej_squared_table(int lmax);
hipError_t launch_edge_correct(int ncat, int lmax, int nb, const double* N, const double* R, const double* t3,
                               double* out, hipStream_t s);
hipError_t launch_edge_correct_sphere(int ncat, int mmax, int nb, const double* N, const double* R, double* out,
                                      hipStream_t s);
size_t pivot_sort_bytes(uint32_t n);
int pivot_axis_bits(int ncat);
hipError_t build_pivots(const uint4* rec, const double* w64, uint32_t n, const CatDesc* cats, int ncat,
                        const unsigned long long* hq, unsigned long long* key_a, unsigned long long* key_b,
                        uint32_t* idx_a, uint32_t* idx_b, uint32_t* head, uint32_t* slot, uint32_t* block_sum,
                        void* sort_tmp, size_t sort_bytes, uint4* prim_rec, double* prim_w, uint32_t* start,
                        hipStream_t s);
}  // namespace tpcf

using namespace tpcf;

namespace {

constexpr int64_t kMaxPoints = (int64_t)1 << 31;
constexpr uint32_t kDetChunk = 64;   // deterministic form: tiles per first-level reduction chunk
constexpr int kStaticScratchBlocks = 256;  // default scratch blocks per wave from the static scratch

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  tpcf_free_fn free_fn = nullptr;  // the caller's free function if the caller's allocator made it
  void* user = nullptr;
  bool fixed = false;  // a slice of the static scratch: never freed
};

// Bump allocation from the static scratch during tpcf_compute_batch_noalloc.
struct Arena {
  bool on = false;
  char* base = nullptr;
  size_t cap = 0, used = 0;
};

// Per-catalogue host description.
struct HostCat {
  int64_t first, n;
  double box;
  int periodic;
  int sphere;  // unit vectors on the sphere (box 4, not periodic, shifted by +2 on the device)
};

constexpr double kPi = 3.14159265358979323846;

}  // namespace

struct tpcf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool dev_ready = false;
  int ncu = 0;
  size_t lds_per_block = 0;

  bool bins_set = false;
  int nbins = 0;
  double rmin = 0, rmax = 0;
  int lmax = 0;
  int precision = TPCF_PREC_FP64;
  double ppc = 8.0;
  int waves_per_cu = 0;    // 0: the default for the kernel (waves_per_cu_for)
  int scratch_blocks = 0;  // 0: the default for the geometry (scratch_blocks_for)
  int phase_mode = -1;  // phase-aligned stencil sweeps: -1 by neighbourhood size, 0 off, 1 on
  // optional caller-supplied device allocator (both set or both NULL)
  tpcf_alloc_fn alloc_fn = nullptr;
  tpcf_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  bool debug = false;
  bool deterministic = false;  // fixed tiles and a fixed-order reduction (tpcf_set_deterministic)

  // staged input (device FP64 copies, concatenated catalogues)
  bool cat_set = false;
  std::vector<HostCat> cats;
  int64_t ntot = 0;
  bool have_w = false;
  DevBuf sx, sy, sz, sw;

  // cell grid, valid for (grid_rmax, grid_ppc, grid_nb)
  bool grid_valid = false;
  double grid_rmax = -1, grid_ppc = -1, grid_rmin = -1;
  int grid_nb = -1;
  std::vector<CatDesc> cd;
  uint32_t ncell = 0;
  DevBuf cats_d, qtmp, cellid, hist, idx_a, idx_b, bsum, errflag, cell_start, rec, w64, perm;

  // sweep buffers
  DevBuf scratch, tile, zeta_d, queue, stats_d, tasks, counts32, alm_dbg, conv_idx, conv32, conv64, regions;
  DevBuf bin_pairs, bin_dd;  // two-point by-product of the last compute call, [ncat][nbins]
  DevBuf edge_tab, edge_io;  // squared 3j table (for edge_lmax) and host-call staging
  // degenerate-term sweep: records with squared weights, and its own outputs
  DevBuf dg_rec, dg_w64, dg_zeta, dg_stats, dg_pairs, dg_dd;
  DevBuf rg_flag, rg_pos, rg_bsum;  // primary-range task lists
  DevBuf det_tiles, det_out, det_chunks, det_catchunk, det_part1;  // deterministic form
  uint32_t det_nchunk = 0;
  // shared pivots: pivot cell side (0 = exact, < 0 = the mean separation), cell tables, pivots
  double pivot_h = 0.0;
  DevBuf pv_keys, pv_idx, pv_head, pv_slot, pv_bsum, pv_tmp, pv_rec, pv_w64, pv_hq, pv_start;
  int edge_lmax = -1;
  bool sums_valid = false;
  int sums_ncat = 0, sums_nb = 0;
  int conv_lmax = -1;
  int conv_q = 0;  // terms per lane of the conversion table in use
  int regions_key = -1;

  // results of the last compute
  bool dbg_valid = false;
  bool dbg_f64 = false;
  int dbg_nb = 0, dbg_nc = 0;
  tpcf_stats stats{};
  std::string err;

  // batch graph cache
  hipGraphExec_t gexec = nullptr;
  std::string gkey;

  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

  Arena arena;  // on only inside tpcf_compute_batch_noalloc
};

namespace {

// Log messages: TPCF_LOG_LEVEL = 0 (default) silent, 1 errors, 2 also one line per catalogue and
// compute call (stage times, pairs, device memory held), 3 also every device allocation and every
// autotuner configuration. They go to stderr, or appended to the file TPCF_LOG_FILE names.
int log_level() {
  const char* s = getenv("TPCF_LOG_LEVEL");
  return (s && *s) ? atoi(s) : 0;
}

std::mutex g_log_mu;

__attribute__((format(printf, 2, 3))) void log_msg(int level, const char* fmt, ...) {
  if (log_level() < level) return;
  static const char* const names[] = {"", "error", "info", "debug"};
  std::lock_guard<std::mutex> lock(g_log_mu);
  const char* path = getenv("TPCF_LOG_FILE");
  FILE* f = (path && *path) ? fopen(path, "a") : nullptr;
  FILE* out = f ? f : stderr;
  fprintf(out, "tpcf[%s] ", names[level < 0 ? 0 : level > 3 ? 3 : level]);
  va_list ap;
  va_start(ap, fmt);
  vfprintf(out, fmt, ap);
  va_end(ap);
  fputc('\n', out);
  if (f) fclose(f);
  else fflush(out);
}

int fail(tpcf_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  log_msg(1, "status %d: %s", code, msg.c_str());
  return code;
}

int hip_fail(tpcf_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return fail(c, e == hipErrorOutOfMemory ? TPCF_E_OUT_OF_MEMORY : TPCF_E_DEVICE, m);
}

#define HIP_TRY(ctx, call)                           \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

size_t device_cap() {
  const char* s = getenv("TPCF_MAX_DEVICE_BYTES");
  if (!s || !*s) return (size_t)-1;
  return (size_t)strtoull(s, nullptr, 10);
}

// Every device buffer the context owns.
std::vector<DevBuf*> all_bufs(tpcf_ctx* c) {
  return {&c->sx, &c->sy, &c->sz, &c->sw, &c->cats_d, &c->qtmp, &c->cellid, &c->hist,
          &c->idx_a, &c->idx_b, &c->bsum, &c->errflag, &c->cell_start, &c->rec, &c->w64, &c->perm,
          &c->scratch, &c->tile, &c->zeta_d, &c->queue, &c->stats_d, &c->tasks, &c->counts32,
          &c->alm_dbg, &c->conv_idx, &c->conv32, &c->conv64, &c->regions, &c->bin_pairs, &c->bin_dd,
          &c->edge_tab, &c->edge_io, &c->pv_keys, &c->pv_idx, &c->pv_head, &c->pv_slot,
          &c->pv_bsum, &c->pv_tmp, &c->pv_rec, &c->pv_w64, &c->pv_hq, &c->pv_start, &c->dg_rec, &c->dg_w64,
          &c->dg_zeta, &c->dg_stats, &c->dg_pairs, &c->dg_dd, &c->rg_flag, &c->rg_pos, &c->rg_bsum,
          &c->det_tiles, &c->det_out, &c->det_chunks, &c->det_catchunk, &c->det_part1};
}

size_t total_bytes(tpcf_ctx* c) {
  size_t t = 0;
  for (DevBuf* b : all_bufs(c)) t += b->bytes;
  return t;
}

// Frees a buffer with whatever allocated it (the caller's free function or hipFree).
void release(DevBuf& b) {
  if (b.p && !b.fixed) {
    if (b.free_fn) b.free_fn(b.p, b.user);
    else (void)hipFree(b.p);
  }
  b.p = nullptr;
  b.bytes = 0;
  b.free_fn = nullptr;
  b.user = nullptr;
  b.fixed = false;
}

constexpr size_t kArenaAlign = 256;

size_t arena_left(const tpcf_ctx* c) {
  const size_t at = (c->arena.used + kArenaAlign - 1) & ~(kArenaAlign - 1);
  return at >= c->arena.cap ? 0 : c->arena.cap - at;
}

int ensure(tpcf_ctx* c, DevBuf& b, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return TPCF_OK;
  if (c->arena.on) {
    // a new slice; a smaller earlier slice of this buffer is simply left behind
    if (bytes > arena_left(c))
      return fail(c, TPCF_E_OUT_OF_MEMORY,
                  std::string("the static scratch of tpcf_compute_batch_noalloc (") + std::to_string(c->arena.cap) +
                      " bytes) cannot hold " + what + " (" + std::to_string(bytes) + " bytes with " +
                      std::to_string(c->arena.cap - arena_left(c)) + " in use)");
    const size_t at = c->arena.cap - arena_left(c);
    b.p = c->arena.base + at;
    b.bytes = bytes;
    b.free_fn = nullptr;
    b.user = nullptr;
    b.fixed = true;
    c->arena.used = at + bytes;
    log_msg(3, "static scratch: %s %zu bytes at offset %zu", what, bytes, at);
    return TPCF_OK;
  }
  const size_t cap = device_cap();
  if (total_bytes(c) - b.bytes + bytes > cap)
    return fail(c, TPCF_E_OUT_OF_MEMORY, std::string("device byte cap (TPCF_MAX_DEVICE_BYTES) exceeded by ") + what);
  release(b);
  if (c->alloc_fn) {
    b.p = c->alloc_fn(bytes, c->alloc_user);
    if (!b.p) return fail(c, TPCF_E_OUT_OF_MEMORY, std::string("the caller's allocator failed for ") + what);
    b.free_fn = c->free_fn;
    b.user = c->alloc_user;
  } else {
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return fail(c, TPCF_E_OUT_OF_MEMORY, std::string("hipMalloc failed for ") + what);
    }
  }
  b.bytes = bytes;
  log_msg(3, "device buffer: %s %zu bytes (%zu held)", what, bytes, total_bytes(c));
  return TPCF_OK;
}

int ensure_device(tpcf_ctx* c) {
  HIP_TRY(c, hipSetDevice(c->device));
  if (c->dev_ready) return TPCF_OK;
  hipDeviceProp_t prop;
  HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
  c->ncu = prop.multiProcessorCount;
  c->lds_per_block = prop.sharedMemPerBlock;
  for (auto& e : c->ev) HIP_TRY(c, hipEventCreate(&e));
  c->dev_ready = true;
  return TPCF_OK;
}

bool is_finite(double v) { return isfinite(v) != 0; }

// The context holds a catalogue on the sphere: bins are angles and lmax is m_max.
bool is_sphere(const tpcf_ctx* c) { return c->cat_set && !c->cats.empty() && c->cats[0].sphere; }

// Lattice bits K: the largest K <= 25 + log2(L / r_max), capped at 32 (periodic) / 31.
int lattice_bits(double box, double rmax, int periodic) {
  int e = 0;
  frexp(box / rmax, &e);
  int K = 25 + (e - 1);
  const int cap = periodic ? 32 : 31;
  if (K > cap) K = cap;
  if (K < 1) K = 1;
  return K;
}

// Conversion of the Chebyshev moments M_{m,k} = sum_j w_j T_k(z_j) (x_j - i y_j)^m into a_lm:
//   a_lm = N_lm (-1)^m sum_k g_lmk M_{m,k},   d^m P_l / dz^m = sum_k g_lmk T_k(z),
//   N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),
// so that a_lm = sum_j w_j conj(Y_lm) with the Condon-Shortley phase. Real component c of a_lm
// (index l*l, or l*l + 2m - 1 / l*l + 2m for Re / Im) is a sum of at most kConvTerms moments;
// moment (m, k) has the index of component (m + k, m). Entries with idx = -1 are unused.
void conversion(int lmax, std::vector<int16_t>& idx, std::vector<double>& coef) {
  const int nc = (lmax + 1) * (lmax + 1);
  idx.assign((size_t)nc * kConvTerms, (int16_t)-1);
  coef.assign((size_t)nc * kConvTerms, 0.0);
  const int D = lmax + 1;
  // A[n][t]: z^n = sum_t A[n][t] T_t(z)
  std::vector<long double> A((size_t)D * D, 0.0L);
  A[0] = 1.0L;
  for (int n = 0; n + 1 < D; ++n)
    for (int t = 0; t < D; ++t) {
      const long double v = A[(size_t)n * D + t];
      if (v == 0.0L) continue;
      if (t == 0) {
        A[(size_t)(n + 1) * D + 1] += v;
      } else {
        if (t + 1 < D) A[(size_t)(n + 1) * D + t + 1] += 0.5L * v;
        A[(size_t)(n + 1) * D + t - 1] += 0.5L * v;
      }
    }
  auto choose = [](int n, int k) {
    long double r = 1.0L;
    for (int i = 1; i <= k; ++i) r = r * (long double)(n - k + i) / (long double)i;
    return r;
  };
  for (int l = 0; l <= lmax; ++l) {
    // monomial coefficients of P_l
    std::vector<long double> pl(D, 0.0L);
    for (int k = 0; 2 * k <= l; ++k)
      pl[l - 2 * k] = ((k & 1) ? -1.0L : 1.0L) * choose(l, k) * choose(2 * l - 2 * k, l) / powl(2.0L, (long double)l);
    for (int m = 0; m <= l; ++m) {
      // d^m P_l / dz^m in monomials, then in Chebyshev polynomials
      std::vector<long double> g(D, 0.0L), gc(D, 0.0L);
      for (int n = 0; n + m <= l; ++n) {
        long double f = 1.0L;
        for (int i = n + 1; i <= n + m; ++i) f *= (long double)i;
        g[n] = pl[n + m] * f;
      }
      for (int n = 0; n < D; ++n)
        if (g[n] != 0.0L)
          for (int t = 0; t < D; ++t) gc[t] += g[n] * A[(size_t)n * D + t];
      long double ratio = 1.0L;
      for (int i = l - m + 1; i <= l + m; ++i) ratio /= (long double)i;
      const long double N =
          sqrtl((2.0L * l + 1.0L) / (4.0L * 3.14159265358979323846264338327950288L) * ratio) * ((m & 1) ? -1.0L : 1.0L);
      for (int part = 0; part < (m == 0 ? 1 : 2); ++part) {
        const int c = m == 0 ? l * l : l * l + 2 * m - 1 + part;
        int q = 0;
        for (int k = 0; k <= l - m; ++k) {
          if ((l - m - k) & 1) continue;  // parity of d^m P_l
          const int mi = m == 0 ? (m + k) * (m + k) : (m + k) * (m + k) + 2 * m - 1 + part;
          idx[(size_t)c * kConvTerms + q] = (int16_t)mi;
          coef[(size_t)c * kConvTerms + q] = (double)(N * gc[k]);
          ++q;
        }
      }
    }
  }
}

// The conversion's non-zero terms spread over the 64 lanes of a wave, so that each lane runs a few
// terms instead of every term slot of its components (at l_max = 10, 286 terms in 726 slots):
// components are taken longest first, each to the lane with the fewest terms so far, and a lane
// runs its components' terms in sequence. Entry (q, lane) is coef[q * 64 + lane] and
// meta[q * 64 + lane] = moment | component << 7 | (last term of the component) << 14; padding
// entries are zero. Q is the longest lane (at most kConvTerms).
void conversion_lanes(int lmax, const std::vector<int16_t>& idx, const std::vector<double>& coef, int& Q,
                      std::vector<int16_t>& meta, std::vector<double>& lcoef) {
  const int nc = (lmax + 1) * (lmax + 1);
  std::vector<int> count(nc, 0), order(nc);
  for (int c = 0; c < nc; ++c) {
    order[c] = c;
    while (count[c] < kConvTerms && idx[(size_t)c * kConvTerms + count[c]] >= 0) ++count[c];
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return count[x] > count[y]; });
  std::vector<std::vector<int>> lanes(64);
  std::vector<int> load(64, 0);
  for (int c : order) {
    const int ln = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lanes[ln].push_back(c);
    load[ln] += count[c];
  }
  Q = *std::max_element(load.begin(), load.end());
  meta.assign((size_t)kConvTerms * 64, 0);
  lcoef.assign((size_t)kConvTerms * 64, 0.0);
  for (int ln = 0; ln < 64; ++ln) {
    int q = 0;
    for (int c : lanes[ln])
      for (int t = 0; t < count[c]; ++t, ++q) {
        const int mi = idx[(size_t)c * kConvTerms + t];
        meta[(size_t)q * 64 + ln] = (int16_t)(mi | (c << 7) | (t + 1 == count[c] ? 1 << 14 : 0));
        lcoef[(size_t)q * 64 + ln] = coef[(size_t)c * kConvTerms + t];
      }
  }
}

typedef unsigned __int128 u128;

// Catalogue on the unit sphere (bins in the angle theta, radians). Points are unit vectors
// shifted by +2 into the non-periodic cube [0, 4)^3; a pair at angle theta has chord
// 2 sin(theta / 2). Lattice and thresholds as in 3D with chord edges: K from the largest chord,
// T_k = ceil(fl(fl(2 sin(theta_k / 2) 2^K / 4)^2)). The grid side follows the surface density
// (a plane through a cubic grid cuts 1.5 / cs^2 cells per unit area on average, so cells on the
// sphere hold about n cs^2 / (6 pi) points).
// Cells along x per cell along y and z. A stencil row (fixed y, z) is one contiguous run of
// cell-sorted records however many x cells it spans, so thinner x cells clip each row closer to
// the chord of the r_max sphere at no cost in the sweep: 4 thinner cells take the candidates per
// in-range pair from about 1.31 to 1.23 at 16 points per cell. Capped so that a grid keeps at most
// `budget` cells.
int x_split(int nc, double budget) {
  const double cube = (double)nc * nc * nc;
  int f = 4;
  while (f > 1 && cube * f > budget) f >>= 1;
  return f;
}

void configure_sphere(const tpcf_ctx* c, const HostCat& h, CatDesc& d, int max_nc, double cell_budget) {
  const int nb = c->nbins;
  const double dth = (c->rmax - c->rmin) / nb;
  const double cmax = 2.0 * sin(0.5 * c->rmax);
  d.sphere = 1;
  d.periodic = 0;
  d.box = 4.0;
  d.K = lattice_bits(4.0, cmax, 0);
  d.sh = 0;
  d.scale = ldexp(1.0, d.K) / 4.0;
  for (int b = 0; b <= nb; ++b) {
    const double th = (b == nb) ? c->rmax : c->rmin + b * dth;
    const double v = 2.0 * sin(0.5 * th) * d.scale;
    d.T[b] = ceil(v * v);
  }
  int ncx = 1;
  if (h.n > 0) ncx = (int)floor(4.0 / sqrt(6.0 * kPi * c->ppc / (double)h.n));
  ncx = std::max(1, std::min(ncx, max_nc));
  d.nc = ncx;
  d.nx = ncx * x_split(ncx, cell_budget);
  const double span = ldexp(1.0, d.K);
  const double margin = ldexp(1.0, d.K - 14);
  const double reach = cmax * d.scale + margin;
  const double cs_min = floor(span / ncx);
  const int R = std::min((int)ceil(reach / cs_min) + 1, ncx - 1);
  d.row_lo = -R;
  d.row_w = 2 * R + 1;
  d.cs = (float)(span / ncx);
  d.inv_cs = (float)(ncx / span);
  d.inv_csx = (float)(d.nx / span);
  d.span = (float)span;
  d.reach = (float)reach;
  d.margin = (float)margin;
  // fast decision: u = 2 asin(sqrt(R^2) / (2 scale)) / dtheta - theta_min / dtheta
  d.inv_delta_l = (float)(2.0 / dth);
  d.u0 = (float)(-c->rmin / dth);
  d.half_inv_scale = (float)(0.5 / d.scale);
  d.asin_small = 0.5 * cmax <= 0.06 ? 1 : 0;
  // |u_fp32 - u_exact| <= (theta_max / dtheta + 1) (4.5 kappa + 20) 2^-24, kappa the condition
  // number of asin at the largest argument (the chord's relative error is at most 4.5 2^-24, the
  // arcsine's own 16 2^-24, the scaling and offset 4 2^-24); integer thresholds move an edge by
  // at most 1 / (2 c scale^2 cos(theta / 2) dtheta) bins. Decisions are taken in FP32 only 4x that
  // far from an edge.
  const double xmax = 0.5 * cmax;
  double kappa = 1.0;
  if (xmax >= 0.999) kappa = 1e30;
  else if (xmax > 1e-4) kappa = xmax / (sqrt(1.0 - xmax * xmax) * asin(xmax));
  const double c1 = 2.0 * sin(0.5 * (c->rmin > 0.0 ? c->rmin : dth));
  const double edge = 1.0 / (2.0 * c1 * d.scale * d.scale * sqrt(1.0 - std::min(xmax * xmax, 0.998)) * dth);
  double eps = 4.0 * ((c->rmax / dth + 1.0) * (4.5 * kappa + 24.0) * ldexp(1.0, -24) + edge);
  if (!(eps <= 0.2)) eps = 2.0;  // every candidate takes the exact path
  d.eps = (float)eps;
  d.one_minus_eps = 1.0f - d.eps;
}

// Grid side, lattice, thresholds, stencil geometry and FP32 bin-decision bound of every
// catalogue.
int configure_grid(tpcf_ctx* c) {
  const int nb = c->nbins;
  const double delta = (c->rmax - c->rmin) / nb;
  c->cd.clear();
  uint64_t cells = 0;
  for (size_t k = 0; k < c->cats.size(); ++k) {
    const HostCat& h = c->cats[k];
    CatDesc d;
    memset(&d, 0, sizeof(d));
    d.point_base = (uint32_t)h.first;
    d.npoints = (uint32_t)h.n;
    d.periodic = h.periodic;
    d.box = h.box;
    if (h.sphere) {
      // the dense cell table of a sphere's cube grows as nc^3: at most 512 per axis, and at most
      // 2^30 cells over all the maps of a batch
      const int max_nc = std::max(16, std::min(512, (int)floor(cbrt(1073741824.0 / (double)c->cats.size()))));
      configure_sphere(c, h, d, max_nc, std::min(67108864.0, 1073741824.0 / (double)c->cats.size()));
      d.cell_base = (uint32_t)cells;
      cells += (uint64_t)d.nx * d.nc * d.nc;
      if (cells >= ((uint64_t)1 << 31)) return fail(c, TPCF_E_UNSUPPORTED, "too many grid cells");
      c->cd.push_back(d);
      continue;
    }
    d.K = lattice_bits(h.box, c->rmax, h.periodic);
    d.sh = h.periodic ? 32 - d.K : 0;
    d.scale = ldexp(1.0, d.K) / h.box;
    for (int b = 0; b <= nb; ++b) {
      const double e = (b == nb) ? c->rmax : c->rmin + b * delta;
      const double v = e * d.scale;
      d.T[b] = ceil(v * v);
    }
    // grid side from the target points per cell
    int ncx = 1;
    if (h.n > 0) {
      const double dens = (double)h.n / (h.box * h.box * h.box);
      const double side = cbrt(c->ppc / dens);
      ncx = (int)floor(h.box / side);
    }
    ncx = std::max(1, std::min(ncx, 512));
    d.nc = ncx;
    d.nx = ncx * x_split(ncx, 67108864.0);
    d.cell_base = (uint32_t)cells;
    cells += (uint64_t)d.nx * ncx * ncx;
    if (cells >= ((uint64_t)1 << 31)) return fail(c, TPCF_E_UNSUPPORTED, "too many grid cells");
    // per-primary stencil: rows within reach = r_max + margin (lattice units) of the primary
    const double span = ldexp(1.0, d.K);
    const double margin = ldexp(1.0, d.K - 14);
    const double reach = c->rmax * d.scale + margin;
    const double cs_min = floor(span / ncx);
    int R = (int)ceil(reach / cs_min) + 1;
    if (h.periodic) {
      if (2 * R + 1 > ncx) {
        d.row_lo = -((ncx - 1) / 2);
        d.row_w = ncx;
      } else {
        d.row_lo = -R;
        d.row_w = 2 * R + 1;
      }
    } else {
      R = std::min(R, ncx - 1);
      d.row_lo = -R;
      d.row_w = 2 * R + 1;
    }
    d.cs = (float)(span / ncx);
    d.inv_cs = (float)(ncx / span);
    d.inv_csx = (float)(d.nx / span);
    d.span = (float)span;
    d.reach = (float)reach;
    d.margin = (float)margin;
    // bin scale per unit of the stored (shifted) coordinate difference: 2^-sh exactly
    d.inv_delta_l = (float)(ldexp(1.0 / (delta * d.scale), -d.sh));
    d.u0 = (float)(-c->rmin / delta);
    // |u_fp32 - u_exact| <= 13 * 2^-24 * r_max / delta bins (see the kernel); a decision is
    // taken in FP32 only when the fractional bin position is 4x that far from an edge.
    double eps = 52.0 * ldexp(1.0, -24) * (c->rmax / delta + 1.0);
    if (eps > 0.2) eps = 2.0;  // no FP32 decisions at all: every candidate takes the exact path
    d.eps = (float)eps;
  d.one_minus_eps = 1.0f - d.eps;
    c->cd.push_back(d);
  }
  c->ncell = (uint32_t)cells;
  return TPCF_OK;
}

// Scratch regions per bin: kMinRegionBlocks blocks each plus a share of the rest proportional
// to the bin's shell volume.
// On the sphere the share follows the area of the bin's annulus, cos theta_0 - cos theta_1.
std::vector<uint32_t> scratch_regions(int nb, double rmin, double rmax, int S, bool sphere) {
  std::vector<double> vol(nb);
  double tot = 0.0;
  const double delta = (rmax - rmin) / nb;
  for (int b = 0; b < nb; ++b) {
    const double e0 = rmin + b * delta, e1 = (b + 1 == nb) ? rmax : rmin + (b + 1) * delta;
    vol[b] = sphere ? cos(e0) - cos(e1) : e1 * e1 * e1 - e0 * e0 * e0;
    tot += vol[b];
  }
  std::vector<uint32_t> r(nb + 1, 0);
  const int spare = S - kMinRegionBlocks * nb;
  for (int b = 0; b < nb; ++b) {
    const uint32_t share = (uint32_t)floor(spare * vol[b] / tot);
    r[b + 1] = r[b] + kMinRegionBlocks + share;
  }
  return r;
}

int check_periodic_range(tpcf_ctx* c) {
  for (const HostCat& h : c->cats) {
    if (h.periodic && !(c->rmax < 0.5 * h.box))
      return fail(c, TPCF_E_INVALID_ARG, "periodic catalogue needs rmax < box/2");
    if (h.sphere && !(c->rmax <= kPi))
      return fail(c, TPCF_E_INVALID_ARG, "angular bins on the sphere need theta_max <= pi");
  }
  return TPCF_OK;
}

// Host-side validation of one catalogue's host arrays.
int validate_host(tpcf_ctx* c, const double* x, const double* y, const double* z, const double* w, int64_t n,
                  double box, int periodic, int sphere) {
  const double lim = box * 1048576.0;
  for (int64_t i = 0; i < n; ++i) {
    const double p[3] = {x[i], y[i], z[i]};
    if (sphere) {
      if (!is_finite(p[0]) || !is_finite(p[1]) || !is_finite(p[2]))
        return fail(c, TPCF_E_INVALID_ARG, "non-finite position at index " + std::to_string(i));
      const double r2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      if (!(r2 >= 1.0 - 1e-6 && r2 <= 1.0 + 1e-6))
        return fail(c, TPCF_E_INVALID_ARG, "point on the sphere is not a unit vector at index " + std::to_string(i));
      if (w && !is_finite(w[i])) return fail(c, TPCF_E_INVALID_ARG, "non-finite weight at index " + std::to_string(i));
      continue;
    }
    for (double v : p) {
      if (!is_finite(v)) return fail(c, TPCF_E_INVALID_ARG, "non-finite position at index " + std::to_string(i));
      if (periodic) {
        if (fabs(v) > lim) return fail(c, TPCF_E_INVALID_ARG, "periodic position beyond 2^20 box sides");
      } else if (v < 0.0 || v >= box) {
        return fail(c, TPCF_E_INVALID_ARG, "non-periodic position outside [0, box) at index " + std::to_string(i));
      }
    }
    if (w && !is_finite(w[i])) return fail(c, TPCF_E_INVALID_ARG, "non-finite weight at index " + std::to_string(i));
  }
  return TPCF_OK;
}

// Copies (and validates) the concatenated catalogues into the staging buffers.
int stage(tpcf_ctx* c, const std::vector<HostCat>& cats, int64_t ntot, const void* xv, const void* yv,
          const void* zv, const void* wv, int memspace, bool f32 = false) {
  // FP32 host inputs are widened on the host (exact) and then staged as FP64 host inputs; FP32
  // device inputs are widened on the device into the FP64 staging arrays.
  std::vector<double> hx, hy, hz, hw;
  if (f32 && memspace == TPCF_MEM_HOST) {
    auto widen = [&](const void* p, std::vector<double>& v) -> const void* {
      if (!p) return nullptr;
      const float* f = static_cast<const float*>(p);
      v.assign(f, f + ntot);
      return v.data();
    };
    xv = widen(xv, hx);
    yv = widen(yv, hy);
    zv = widen(zv, hz);
    wv = widen(wv, hw);
    f32 = false;
  }
  const double* x = static_cast<const double*>(xv);
  const double* y = static_cast<const double*>(yv);
  const double* z = static_cast<const double*>(zv);
  const double* w = static_cast<const double*>(wv);
  if (memspace == TPCF_MEM_HOST) {
    for (const HostCat& h : cats) {
      int rc = validate_host(c, x + h.first, y + h.first, z + h.first, w ? w + h.first : nullptr, h.n, h.box,
                             h.periodic, h.sphere);
      if (rc) return rc;
    }
  }
  int rc;
  if ((rc = ensure_device(c))) return rc;
  const size_t bytes = (size_t)ntot * sizeof(double);
  if ((rc = ensure(c, c->sx, bytes, "positions")) || (rc = ensure(c, c->sy, bytes, "positions")) ||
      (rc = ensure(c, c->sz, bytes, "positions")))
    return rc;
  if (w && (rc = ensure(c, c->sw, bytes, "weights"))) return rc;
  const hipMemcpyKind kind = memspace == TPCF_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  if (ntot && f32) {
    widen_f32(static_cast<const float*>(xv), (double*)c->sx.p, (size_t)ntot, c->stream);
    widen_f32(static_cast<const float*>(yv), (double*)c->sy.p, (size_t)ntot, c->stream);
    widen_f32(static_cast<const float*>(zv), (double*)c->sz.p, (size_t)ntot, c->stream);
    if (w) widen_f32(static_cast<const float*>(wv), (double*)c->sw.p, (size_t)ntot, c->stream);
    HIP_TRY(c, hipGetLastError());
  } else if (ntot) {
    HIP_TRY(c, hipMemcpyAsync(c->sx.p, x, bytes, kind, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->sy.p, y, bytes, kind, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->sz.p, z, bytes, kind, c->stream));
    if (w) HIP_TRY(c, hipMemcpyAsync(c->sw.p, w, bytes, kind, c->stream));
  }
  if (memspace == TPCF_MEM_DEVICE && ntot) {
    // validate on the device
    std::vector<CatDesc> tmp(cats.size());
    for (size_t k = 0; k < cats.size(); ++k) {
      memset(&tmp[k], 0, sizeof(CatDesc));
      tmp[k].point_base = (uint32_t)cats[k].first;
      tmp[k].box = cats[k].box;
      tmp[k].periodic = cats[k].periodic;
      tmp[k].sphere = cats[k].sphere;
    }
    if ((rc = ensure(c, c->cats_d, tmp.size() * sizeof(CatDesc), "catalogue table")) ||
        (rc = ensure(c, c->errflag, sizeof(int), "flags")))
      return rc;
    HIP_TRY(c, hipMemcpyAsync(c->cats_d.p, tmp.data(), tmp.size() * sizeof(CatDesc), hipMemcpyHostToDevice,
                              c->stream));
    fill_u32((uint32_t*)c->errflag.p, 0u, 1, c->stream);
    validate_inputs((const double*)c->sx.p, (const double*)c->sy.p, (const double*)c->sz.p,
                    w ? (const double*)c->sw.p : nullptr, (uint32_t)ntot, (const CatDesc*)c->cats_d.p,
                    (int)cats.size(), (int*)c->errflag.p, c->stream);
    int flag = 0;
    HIP_TRY(c, hipMemcpyAsync(&flag, c->errflag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (flag & 1) return fail(c, TPCF_E_INVALID_ARG, "non-finite position or weight");
    if (flag & 2) return fail(c, TPCF_E_INVALID_ARG, "non-periodic position outside [0, box)");
    if (flag & 4) return fail(c, TPCF_E_INVALID_ARG, "periodic position beyond 2^20 box sides");
    if (flag & 8) return fail(c, TPCF_E_INVALID_ARG, "point on the sphere is not a unit vector");
  } else {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  log_msg(2, "catalogue: %lld points in %zu catalogue(s)%s, inputs in %s memory", (long long)ntot, cats.size(),
       (!cats.empty() && cats[0].sphere) ? " on the sphere" : "", memspace == TPCF_MEM_HOST ? "host" : "device");
  c->cats = cats;
  c->ntot = ntot;
  c->have_w = w != nullptr;
  c->cat_set = true;
  c->grid_valid = false;
  c->dbg_valid = false;
  return TPCF_OK;
}

bool grid_current(const tpcf_ctx* c) {
  return c->grid_valid && c->grid_rmax == c->rmax && c->grid_rmin == c->rmin && c->grid_ppc == c->ppc &&
         c->grid_nb == c->nbins;
}

// Host part of the grid build: grid geometry, stencil rows, buffers, tables on the device.
int prepare_grid(tpcf_ctx* c) {
  int rc;
  c->grid_valid = false;  // geometry and tables change: the built grid no longer matches them
  if ((rc = configure_grid(c))) return rc;
  const size_t n = (size_t)c->ntot;
  if ((rc = ensure(c, c->cats_d, c->cd.size() * sizeof(CatDesc), "catalogue table")) ||
      (rc = ensure(c, c->qtmp, n * sizeof(uint4), "grid")) || (rc = ensure(c, c->cellid, n * 4, "grid")) ||
      (rc = ensure(c, c->hist, (size_t)c->ncell * 4, "grid")) || (rc = ensure(c, c->idx_a, n * 4, "grid")) ||
      (rc = ensure(c, c->idx_b, n * 4, "grid")) ||
      (rc = ensure(c, c->bsum, scan_block_count(c->ncell) * 4 + 4, "grid")) ||
      (rc = ensure(c, c->errflag, sizeof(int), "flags")) ||
      (rc = ensure(c, c->cell_start, ((size_t)c->ncell + 1) * 4, "grid")) ||
      (rc = ensure(c, c->rec, (n + 1) * sizeof(uint4), "records")) ||
      (rc = ensure(c, c->w64, (n + 1) * 8, "weights")) ||
      (rc = ensure(c, c->perm, n * 4, "permutation")))
    return rc;
  HIP_TRY(c, hipMemcpyAsync(c->cats_d.p, c->cd.data(), c->cd.size() * sizeof(CatDesc), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TPCF_OK;
}

// Device part of the grid build (stream-ordered kernels only).
int record_grid(tpcf_ctx* c) {
  HIP_TRY(c, build_grid((const double*)c->sx.p, (const double*)c->sy.p, (const double*)c->sz.p,
                        c->have_w ? (const double*)c->sw.p : nullptr, (uint32_t)c->ntot,
                        (const CatDesc*)c->cats_d.p, (int)c->cd.size(), c->ncell, (uint4*)c->qtmp.p,
                        (uint32_t*)c->cellid.p, (uint32_t*)c->hist.p, (uint32_t*)c->idx_a.p,
                        (uint32_t*)c->idx_b.p, (uint32_t*)c->bsum.p, (int*)c->errflag.p,
                        (uint32_t*)c->cell_start.p, (uint4*)c->rec.p, (double*)c->w64.p, (uint32_t*)c->perm.p,
                        c->stream));
  return TPCF_OK;
}

void mark_grid(tpcf_ctx* c) {
  c->grid_valid = true;
  c->grid_rmax = c->rmax;
  c->grid_rmin = c->rmin;
  c->grid_ppc = c->ppc;
  c->grid_nb = c->nbins;
}

// Phase-aligned stencil sweeps. A wave reads every record within reach of its primary; the waves
// in flight hold nearby primaries (tasks are taken in cell order) and so read nearly the same
// records, but each from its own starting point, so together they touch the whole neighbourhood
// at once. Once that exceeds an XCD's 4 MiB L2 the records come from the Infinity Cache or HBM.
// Aligned, each wave starts at the point of its stencil that matches its ticket's phase among the
// waves in flight, which keeps them all at about the same rows at the same time. The counting
// that picks the starting row costs about 1-3% where the L2 already holds a neighbourhood, so it
// is on by default only when the expected neighbourhood of one primary (records of 16 bytes)
// exceeds 2 MiB, half an XCD's L2.
int phase_aligned(const tpcf_ctx* c) {
  if (c->phase_mode >= 0) return c->phase_mode;
  double most = 0.0;
  for (const HostCat& h : c->cats) {
    double nbr;
    if (h.sphere) {
      nbr = (double)h.n * 0.5 * (1.0 - cos(std::min(c->rmax, kPi)));
    } else {
      const double r = c->rmax;
      nbr = (double)h.n * (4.0 / 3.0) * kPi * r * r * r / (h.box * h.box * h.box);
    }
    most = std::max(most, std::min(nbr, (double)h.n));
  }
  return most * 16.0 > 2097152.0 ? 1 : 0;
}

// Scratch blocks per wave, unless set by tpcf_set_tuning: 1024 in 3D, 512 on the sphere. The pair
// lists of all waves in flight stream through the caches; on the sphere (fewer components per
// pair, so more pairs per unit of work) the smaller lists gain 1.6% at nside 1024 and 9% at nside
// 4096, while in 3D the extra region flushes cost 10%.
int scratch_blocks_for(const tpcf_ctx* c) {
  if (c->scratch_blocks > 0) return c->scratch_blocks;
  return is_sphere(c) ? 512 : 1024;
}

// Persistent waves per compute unit, unless set by tpcf_set_tuning: 12 (three per SIMD, as the
// register allocation of the FP32 sweeps and of the FP64 sphere sweep allows), 8 for the FP64 3D
// sweep (two per SIMD).
int waves_per_cu_for(const tpcf_ctx* c) {
  if (c->waves_per_cu > 0) return c->waves_per_cu;
  return (c->precision == TPCF_PREC_FP64 && !is_sphere(c)) ? 8 : 12;
}

// Device bytes that prepare_sweep and setup_det request after the per-wave scratch and tiles
// (upper bounds, each rounded up to the arena alignment), for a sweep over ntask tasks.
size_t later_sweep_bytes(const tpcf_ctx* c, uint32_t ntask) {
  const bool f64 = c->precision == TPCF_PREC_FP64;
  const bool sph = is_sphere(c);
  const size_t nb = (size_t)c->nbins, L = (size_t)c->lmax, NC = (size_t)ncomp(c->lmax, sph);
  const size_t ncat = c->cd.size(), n = (size_t)c->ntot;
  auto up = [](size_t b) { return (std::max<size_t>(b, 16) + kArenaAlign - 1) & ~(kArenaAlign - 1); };
  size_t t = up(ncat * (L + 1) * nb * nb * 8) + up(kQueueSegments * 4) + up(16) + 2 * up(ncat * nb * 8);
  const size_t nconv = (size_t)kConvTerms * 64;  // the conversion spread over the lanes
  t += up(nconv * 2) + up(nconv * 8) + up(nconv * 4) + up((nb + 1) * 4);
  if (c->debug) t += up(n * nb * 4) + up(n * nb * NC * (f64 ? 8 : 4));
  if (c->deterministic) {
    const size_t TP = tile_primaries(f64, sph);
    const size_t tiles = ntask / TP + ncat + 1, chunks = tiles / kDetChunk + ncat + 1;
    const size_t stride = (L + 1) * nb * nb + nb;
    t += up(tiles * 8) + up(tiles * stride * 8) + up(chunks * 8) + up((ncat + 1) * 4) + up(chunks * stride * 8);
  }
  return t;
}

// Host part of the sweep: buffers, normalisation constants and the kernel arguments.
int prepare_sweep(tpcf_ctx* c, const uint32_t* tasks_d, uint32_t ntask, SweepArgs& a, int& waves) {
  const bool f64 = c->precision == TPCF_PREC_FP64;
  const bool sph = is_sphere(c);
  const int nb = c->nbins, L = c->lmax, NC = ncomp(L, sph);
  const int ncat = (int)c->cd.size();
  int S = scratch_blocks_for(c);
  // From the static scratch, shorter pair lists by default (more waves fit in it).
  if (c->arena.on && c->scratch_blocks <= 0) S = std::min(S, std::max(kMinRegionBlocks * nb, kStaticScratchBlocks));
  int rc;
  const size_t lds = sweep_lds_bytes(nb, L, f64, sph);
  if (lds > 160 * 1024) return fail(c, TPCF_E_UNSUPPORTED, "LDS layout too large");
  // no more waves per CU than its 160 KiB of LDS holds (allocated in 512-byte granules)
  const int lds_waves = (int)((160 * 1024) / ((lds + 511) & ~(size_t)511));
  waves = std::max(1, c->ncu * std::min(waves_per_cu_for(c), lds_waves));
  if ((uint32_t)waves > ntask) waves = (int)std::max<uint32_t>(1, ntask);
  if (S < kMinRegionBlocks * nb)
    return fail(c, TPCF_E_INVALID_ARG, "scratch_blocks must be at least 5 x nbins");
  if (c->arena.on) {
    // As many waves as the static scratch holds beside the buffers still to come.
    const size_t per_wave = (size_t)(S + kScratchTail) * kBlock * 4 + sweep_tile_bytes_per_wave(L, nb, f64, sph);
    const size_t rest = later_sweep_bytes(c, ntask) + 2 * kArenaAlign;
    const size_t left = arena_left(c);
    if (left < rest + per_wave)
      return fail(c, TPCF_E_OUT_OF_MEMORY,
                  "the static scratch of tpcf_compute_batch_noalloc (" + std::to_string(c->arena.cap) +
                      " bytes) cannot hold one sweep wave beside this batch's grid (" +
                      std::to_string(c->arena.cap - left) + " bytes in use, " + std::to_string(rest + per_wave) +
                      " more needed)");
    waves = (int)std::min<size_t>((size_t)waves, (left - rest) / per_wave);
  }
  if ((rc = ensure(c, c->scratch, (size_t)waves * (S + kScratchTail) * kBlock * 4, "scratch")) ||
      (rc = ensure(c, c->tile, (size_t)waves * sweep_tile_bytes_per_wave(L, nb, f64, sph), "tiles")) ||
      (rc = ensure(c, c->zeta_d, (size_t)ncat * (L + 1) * nb * nb * 8, "zeta")) ||
      (rc = ensure(c, c->queue, kQueueSegments * 4, "queue")) || (rc = ensure(c, c->stats_d, 16, "stats")) ||
      (rc = ensure(c, c->bin_pairs, (size_t)ncat * nb * 8, "pair sums")) ||
      (rc = ensure(c, c->bin_dd, (size_t)ncat * nb * 8, "pair sums")))
    return rc;
  if (c->conv_lmax != L) {
    std::vector<int16_t> idx0, idx;
    std::vector<double> coef0, coef;
    conversion(L, idx0, coef0);
    conversion_lanes(L, idx0, coef0, c->conv_q, idx, coef);
    if (c->conv_q > kConvTerms) return fail(c, TPCF_E_UNSUPPORTED, "conversion table does not fit the lanes");
    std::vector<float> coef32(coef.begin(), coef.end());
    if ((rc = ensure(c, c->conv_idx, idx.size() * 2, "constants")) ||
        (rc = ensure(c, c->conv64, coef.size() * 8, "constants")) ||
        (rc = ensure(c, c->conv32, coef.size() * 4, "constants")))
      return rc;
    HIP_TRY(c, hipMemcpyAsync(c->conv_idx.p, idx.data(), idx.size() * 2, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->conv64.p, coef.data(), coef.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->conv32.p, coef32.data(), coef32.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->conv_lmax = L;
  }
  {
    std::vector<uint32_t> regs = scratch_regions(nb, c->rmin, c->rmax, S, sph);
    if ((rc = ensure(c, c->regions, regs.size() * 4, "regions"))) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->regions.p, regs.data(), regs.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  if (c->debug) {
    if ((rc = ensure(c, c->counts32, (size_t)c->ntot * nb * 4, "debug counts")) ||
        (rc = ensure(c, c->alm_dbg, (size_t)c->ntot * nb * NC * (f64 ? 8 : 4), "debug a_lm")))
      return rc;
  }
  memset(&a, 0, sizeof(a));
  a.rec = (const uint4*)c->rec.p;
  a.sentinel = (uint32_t)c->ntot;
  a.w64 = (const double*)c->w64.p;
  a.cell_start = (const uint32_t*)c->cell_start.p;
  a.cats = (const CatDesc*)c->cats_d.p;
  a.ncat = ncat;
  a.nb = nb;
  a.task_list = tasks_d;
  a.ntask = ntask;
  a.queue = (uint32_t*)c->queue.p;
  a.scratch = (uint32_t*)c->scratch.p;
  a.scratch_blocks = S;
  a.regions = (const uint32_t*)c->regions.p;
  a.tile = c->tile.p;
  a.zeta = (double*)c->zeta_d.p;
  a.counts = c->debug ? (int32_t*)c->counts32.p : nullptr;
  a.alm_debug = c->debug ? c->alm_dbg.p : nullptr;
  a.stats = (unsigned long long*)c->stats_d.p;
  a.bin_pairs = (unsigned long long*)c->bin_pairs.p;
  a.bin_dd = (double*)c->bin_dd.p;
  a.conv_idx = (const int16_t*)c->conv_idx.p;
  a.conv_q = c->conv_q;
  a.conv_coef32 = (const float*)c->conv32.p;
  a.conv_coef64 = (const double*)c->conv64.p;
  a.phase_rows = phase_aligned(c);
  return TPCF_OK;
}

// Deterministic form: tiles of the contraction size over each catalogue's tasks (starts[k] = first
// task of catalogue k, ncat + 1 entries), one result slot per tile, and the tables of the
// fixed-order reduction (chunks of kDetChunk consecutive tiles, then the chunks of a catalogue).
int setup_det(tpcf_ctx* c, const std::vector<uint32_t>& starts, SweepArgs& a) {
  const int ncat = (int)starts.size() - 1;
  const uint32_t TP = tile_primaries(c->precision == TPCF_PREC_FP64, is_sphere(c));
  std::vector<uint2> tiles, chunks;
  std::vector<uint32_t> cat_chunk(ncat + 1, 0);
  for (int k = 0; k < ncat; ++k) {
    const size_t tile0 = tiles.size();
    for (uint32_t t = starts[k]; t < starts[k + 1]; t += TP)
      tiles.push_back(make_uint2(t, std::min(t + TP, starts[k + 1])));
    cat_chunk[k] = (uint32_t)chunks.size();
    for (size_t q = tile0; q < tiles.size(); q += kDetChunk)
      chunks.push_back(make_uint2((uint32_t)q, (uint32_t)std::min(q + kDetChunk, tiles.size())));
  }
  cat_chunk[ncat] = (uint32_t)chunks.size();
  const size_t stride = (size_t)(c->lmax + 1) * c->nbins * c->nbins + c->nbins;
  int rc;
  if ((rc = ensure(c, c->det_tiles, std::max<size_t>(1, tiles.size()) * sizeof(uint2), "deterministic tiles")) ||
      (rc = ensure(c, c->det_out, std::max<size_t>(1, tiles.size()) * stride * 8, "deterministic tiles")) ||
      (rc = ensure(c, c->det_chunks, std::max<size_t>(1, chunks.size()) * sizeof(uint2), "deterministic tiles")) ||
      (rc = ensure(c, c->det_catchunk, cat_chunk.size() * 4, "deterministic tiles")) ||
      (rc = ensure(c, c->det_part1, std::max<size_t>(1, chunks.size()) * stride * 8, "deterministic tiles")))
    return rc;
  if (!tiles.empty()) {
    HIP_TRY(c, hipMemcpyAsync(c->det_tiles.p, tiles.data(), tiles.size() * sizeof(uint2), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->det_chunks.p, chunks.data(), chunks.size() * sizeof(uint2), hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(c, hipMemcpyAsync(c->det_catchunk.p, cat_chunk.data(), cat_chunk.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // the host tables go out of scope
  a.det_tiles = (const uint2*)c->det_tiles.p;
  a.ndet = (uint32_t)tiles.size();
  a.det_out = (double*)c->det_out.p;
  a.phase_rows = 0;
  c->det_nchunk = (uint32_t)chunks.size();
  return TPCF_OK;
}

// First task of every catalogue when every point is a primary.
std::vector<uint32_t> point_starts(const tpcf_ctx* c) {
  std::vector<uint32_t> st;
  for (const CatDesc& d : c->cd) st.push_back(d.point_base);
  st.push_back((uint32_t)c->ntot);
  return st;
}

// Device part of the sweep: clears (fill kernels, never memset nodes) and the persistent launch.
int record_sweep(tpcf_ctx* c, const SweepArgs& a, int waves) {
  const bool f64 = c->precision == TPCF_PREC_FP64;
  const bool sph = is_sphere(c);
  const int nb = c->nbins, L = c->lmax, NC = ncomp(L, sph);
  if (c->debug) {
    fill_u32((uint32_t*)c->counts32.p, 0u, (size_t)c->ntot * nb, c->stream);
    fill_u32((uint32_t*)c->alm_dbg.p, 0u, (size_t)c->ntot * nb * NC * (f64 ? 2 : 1), c->stream);
  }
  fill_f64(a.zeta, 0.0, (size_t)a.ncat * (L + 1) * nb * nb, c->stream);
  fill_u32(a.queue, 0u, kQueueSegments, c->stream);
  fill_u32(reinterpret_cast<uint32_t*>(a.stats), 0u, 4, c->stream);
  fill_u32(reinterpret_cast<uint32_t*>(a.bin_pairs), 0u, (size_t)a.ncat * nb * 2, c->stream);
  fill_f64(a.bin_dd, 0.0, (size_t)a.ncat * nb, c->stream);
  if (a.ntask > 0) HIP_TRY(c, launch_sweep(L, f64, sph, a, waves, c->stream));
  if (a.det_tiles && a.ntask > 0) {
    const uint32_t Z = (uint32_t)((L + 1) * nb * nb);
    HIP_TRY(c, launch_det_reduce(a.det_out, Z + (uint32_t)nb, (const uint2*)c->det_chunks.p, c->det_nchunk,
                                 (const uint32_t*)c->det_catchunk.p, a.ncat, Z, nb, (double*)c->det_part1.p,
                                 a.zeta, a.bin_dd, c->stream));
  }
  return TPCF_OK;
}

int finish_stats(tpcf_ctx* c, bool grid_built, uint32_t ntask) {
  unsigned long long st[2] = {0, 0};
  HIP_TRY(c, hipMemcpyAsync(st, c->stats_d.p, 16, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->stats.n_pairs = (int64_t)st[0];
  c->stats.n_candidates = (int64_t)st[1];
  c->stats.n_primaries = ntask;
  float ms = 0.f;
  c->stats.ms_grid = 0.0;
  if (grid_built && hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) c->stats.ms_grid = ms;
  c->stats.ms_sweep = hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess ? ms : 0.0;
  c->stats.ms_total = c->stats.ms_grid + c->stats.ms_sweep;
  c->stats.cells_per_axis = c->cd.empty() ? 0 : c->cd[0].nc;
  c->stats.precision = c->precision;
  c->stats.lmax = c->lmax;
  c->stats.nbins = c->nbins;
  c->dbg_valid = c->debug;
  c->sums_valid = true;
  c->sums_ncat = (int)c->cd.size();
  c->sums_nb = c->nbins;
  c->dbg_f64 = c->precision == TPCF_PREC_FP64;
  c->dbg_nb = c->nbins;
  c->dbg_nc = ncomp(c->lmax, is_sphere(c));
  log_msg(2, "compute: %zu catalogue(s), %u primaries, %lld pairs, %lld candidates, %s%s, grid %.3f ms, sweep %.3f ms, "
       "%d waves, device memory %zu bytes%s",
       c->cd.size(), ntask, (long long)st[0], (long long)st[1], c->precision == TPCF_PREC_FP64 ? "fp64" : "mixed",
       c->deterministic ? " deterministic" : "", c->stats.ms_grid, c->stats.ms_sweep, c->stats.waves,
       c->arena.on ? c->arena.used : total_bytes(c), c->arena.on ? " of the static scratch" : " held");
  return TPCF_OK;
}

int copy_out(tpcf_ctx* c, double* zeta, size_t count, int memspace) {
  const hipMemcpyKind kind = memspace == TPCF_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  HIP_TRY(c, hipMemcpyAsync(zeta, c->zeta_d.p, count * 8, kind, c->stream));
  return TPCF_OK;
}

// Key of everything a captured batch graph depends on.
std::string graph_key(const tpcf_ctx* c, const SweepArgs& a, int waves) {
  std::string k;
  auto add = [&](const void* p, size_t n) { k.append((const char*)p, n); };
  add(&c->ntot, sizeof(c->ntot));
  for (const HostCat& h : c->cats) add(&h, sizeof(h));
  add(&c->nbins, sizeof(int));
  add(&c->rmin, sizeof(double));
  add(&c->rmax, sizeof(double));
  add(&c->lmax, sizeof(int));
  add(&c->precision, sizeof(int));
  add(&c->ppc, sizeof(double));
  add(&c->have_w, sizeof(bool));
  add(&c->debug, sizeof(bool));
  add(&a, sizeof(a));
  add(&waves, sizeof(int));
  return k;
}

bool graphs_enabled() {
  const char* s = getenv("TPCF_GRAPH");
  return !(s && s[0] == '0');
}

// Shared pivots of the (single) catalogue: pivot cells of Hq = max(1, floor(h * scale)) lattice
// units, h the pivot cell side; when pivot_h < 0 the mean separation, L / n^(1/3) in a box and
// sqrt(4 pi / n) on the sphere. Builds the pivots on the stream and returns their number G
// (synchronises).
int prepare_pivots(tpcf_ctx* c, uint32_t& G) {
  const int ncat = (int)c->cats.size();
  const int B = pivot_axis_bits(ncat);
  std::vector<unsigned long long> hq(ncat);
  for (int k = 0; k < ncat; ++k) {
    const CatDesc& d = c->cd[k];
    const HostCat& h = c->cats[k];
    double side = c->pivot_h;
    if (side < 0.0) {
      if (h.n == 0) side = h.box;
      else side = h.sphere ? sqrt(4.0 * kPi / (double)h.n) : h.box / cbrt((double)h.n);
    }
    // On the sphere a cell must stay well below the radius: a pivot is its members' mean position,
    // which must keep a direction.
    if (h.sphere && side > 0.25) return fail(c, TPCF_E_INVALID_ARG, "pivot cell on the sphere must be at most 0.25");
    const uint64_t span = (uint64_t)1 << d.K;
    double q = floor(side * d.scale);
    if (!(q >= 1.0)) q = 1.0;
    if (q > (double)span) q = (double)span;
    hq[k] = (unsigned long long)q;
    if ((span + hq[k] - 1) / hq[k] > ((uint64_t)1 << B))
      return fail(c, TPCF_E_INVALID_ARG,
                  "pivot cell too small: more than 2^" + std::to_string(B) + " pivot cells per axis" +
                      (ncat > 1 ? " in a batch of " + std::to_string(ncat) + " catalogues" : std::string()));
  }
  const size_t n = (size_t)c->ntot;
  const size_t sort_bytes = pivot_sort_bytes((uint32_t)n);
  int rc;
  if ((rc = ensure(c, c->pv_keys, (n + 1) * 16, "pivot keys")) || (rc = ensure(c, c->pv_idx, (n + 1) * 8, "pivot keys")) ||
      (rc = ensure(c, c->pv_head, (n + 1) * 4, "pivot keys")) || (rc = ensure(c, c->pv_slot, (n + 1) * 4, "pivot keys")) ||
      (rc = ensure(c, c->pv_bsum, scan_block_count((uint32_t)n) * 4 + 4, "pivot keys")) ||
      (rc = ensure(c, c->pv_tmp, sort_bytes, "pivot sort")) ||
      (rc = ensure(c, c->pv_rec, (n + 1) * 16, "pivots")) || (rc = ensure(c, c->pv_w64, (n + 1) * 8, "pivots")) ||
      (rc = ensure(c, c->pv_hq, (size_t)ncat * 8, "pivot cells")) ||
      (rc = ensure(c, c->pv_start, ((size_t)ncat + 1) * 4, "pivot ranges")))
    return rc;
  HIP_TRY(c, hipMemcpyAsync(c->pv_hq.p, hq.data(), hq.size() * 8, hipMemcpyHostToDevice, c->stream));
  unsigned long long* keys = (unsigned long long*)c->pv_keys.p;
  uint32_t* idx = (uint32_t*)c->pv_idx.p;
  HIP_TRY(c, build_pivots((const uint4*)c->rec.p, (const double*)c->w64.p, (uint32_t)n, (const CatDesc*)c->cats_d.p,
                          ncat, (const unsigned long long*)c->pv_hq.p, keys, keys + (n + 1), idx, idx + (n + 1),
                          (uint32_t*)c->pv_head.p, (uint32_t*)c->pv_slot.p, (uint32_t*)c->pv_bsum.p, c->pv_tmp.p,
                          sort_bytes, (uint4*)c->pv_rec.p, (double*)c->pv_w64.p, (uint32_t*)c->pv_start.p,
                          c->stream));
  HIP_TRY(c, hipMemcpyAsync(&G, (uint32_t*)c->pv_slot.p + n, 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return TPCF_OK;
}

int compute(tpcf_ctx* c, int64_t p_begin, int64_t p_end, double* zeta, int memspace, bool use_graph) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (!c->bins_set) return fail(c, TPCF_E_STATE, "set_bins has not been called");
  if (!c->cat_set) return fail(c, TPCF_E_STATE, "no catalogue set");
  if (!zeta) return fail(c, TPCF_E_INVALID_ARG, "zeta is NULL");
  if (memspace != TPCF_MEM_HOST && memspace != TPCF_MEM_DEVICE)
    return fail(c, TPCF_E_INVALID_ARG, "unknown memory space");
  int rc;
  if ((rc = check_periodic_range(c))) return rc;
  if ((rc = ensure_device(c))) return rc;
  const bool rebuild = !grid_current(c);
  const bool pivots = c->pivot_h != 0.0;
  if (pivots && (p_begin != 0 || p_end != c->ntot))
    return fail(c, TPCF_E_UNSUPPORTED, "shared pivots cover the whole catalogue: no primary ranges");
  if (rebuild && (rc = prepare_grid(c))) return rc;
  const uint32_t* tasks = nullptr;
  uint32_t ntask = (uint32_t)c->ntot;
  if (pivots) {
    if (rebuild) {
      if ((rc = record_grid(c))) return rc;
      mark_grid(c);
    }
    if ((rc = prepare_pivots(c, ntask))) return rc;
  } else if (p_begin != 0 || p_end != c->ntot) {
    // primaries by input index -> sorted positions (needs the grid: build it eagerly first)
    if (rebuild) {
      if ((rc = record_grid(c))) return rc;
      mark_grid(c);
    }
    // sorted positions of the range's primaries, in sorted order, built on the device
    const size_t n = (size_t)c->ntot;
    if ((rc = ensure(c, c->rg_flag, std::max<size_t>(1, n) * 4, "range tasks")) ||
        (rc = ensure(c, c->rg_pos, (n + 1) * 4, "range tasks")) ||
        (rc = ensure(c, c->rg_bsum, scan_block_count((uint32_t)n) * 4 + 4, "range tasks")) ||
        (rc = ensure(c, c->tasks, std::max<size_t>(1, n) * 4, "task list")))
      return rc;
    HIP_TRY(c, range_tasks((const uint32_t*)c->perm.p, (uint32_t)n, (uint32_t)p_begin, (uint32_t)p_end,
                           (uint32_t*)c->rg_flag.p, (uint32_t*)c->rg_pos.p, (uint32_t*)c->rg_bsum.p,
                           (uint32_t*)c->tasks.p, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&ntask, (uint32_t*)c->rg_pos.p + n, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    tasks = (const uint32_t*)c->tasks.p;
  }
  const bool grid_in_run = rebuild && !c->grid_valid;
  SweepArgs a;
  int waves = 0;
  if ((rc = prepare_sweep(c, tasks, ntask, a, waves))) return rc;
  if (pivots) {
    a.prim_rec = (const uint4*)c->pv_rec.p;
    a.prim_w64 = (const double*)c->pv_w64.p;
    a.prim_cat_start = (const uint32_t*)c->pv_start.p;
    a.counts = nullptr;  // per-point debug rows do not apply to pivots
    a.alm_debug = nullptr;
  }
  if (c->deterministic) {
    std::vector<uint32_t> starts;
    if (pivots) {
      starts.resize(c->cd.size() + 1);
      HIP_TRY(c, hipMemcpyAsync(starts.data(), c->pv_start.p, starts.size() * 4, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
    } else if (tasks) {  // a primary range: its tasks are grouped by catalogue
      starts.push_back(0);
      for (const HostCat& h : c->cats) {
        const int64_t lo = std::max<int64_t>(p_begin, h.first), hi = std::min<int64_t>(p_end, h.first + h.n);
        starts.push_back(starts.back() + (uint32_t)std::max<int64_t>(0, hi - lo));
      }
    } else {
      starts = point_starts(c);
    }
    if ((rc = setup_det(c, starts, a))) return rc;
  }
  c->stats.waves = waves;
  // The null stream cannot be captured: batches on it launch eagerly. So do batches with shared
  // pivots, whose pivot count is read back on the host before the sweep.
  const bool graph = use_graph && !pivots && graphs_enabled() && c->stream != nullptr;
  if (graph) {
    // The whole device sequence (grid build + clears + persistent sweep) as one HIP graph,
    // captured once per batch shape and replayed afterwards.
    const std::string key = graph_key(c, a, waves) + (grid_in_run ? "g" : "-");
    if (!c->gexec || key != c->gkey) {
      if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
        c->gkey.clear();
      }
      hipGraph_t g = nullptr;
      HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      int rc1 = grid_in_run ? record_grid(c) : TPCF_OK;
      int rc2 = rc1 ? rc1 : record_sweep(c, a, waves);
      hipError_t e = hipStreamEndCapture(c->stream, &g);
      if (rc2) {
        if (g) (void)hipGraphDestroy(g);
        return rc2;
      }
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        c->gexec = nullptr;
        return hip_fail(c, e, "hipGraphInstantiate");
      }
      c->gkey = key;
    }
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
    if (grid_in_run) mark_grid(c);
    c->stats.ms_grid = -1.0;
  } else {
    if (grid_in_run) {
      HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
      if ((rc = record_grid(c))) return rc;
      HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
      mark_grid(c);
    }
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    if ((rc = record_sweep(c, a, waves))) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
  }
  const size_t cnt = (size_t)c->cd.size() * (c->lmax + 1) * c->nbins * c->nbins;
  if ((rc = copy_out(c, zeta, cnt, memspace))) return rc;
  rc = finish_stats(c, grid_in_run && !graph, ntask);
  if (pivots) c->dbg_valid = false;
  return rc;
}

// Shared body of tpcf_set_catalog and tpcf_set_catalog_f32 (arrays of double or float).
int set_catalog_impl(tpcf_ctx* c, int64_t n, const void* x, const void* y, const void* z, const void* w, double box,
                     int periodic, int memspace, bool f32) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (n < 0 || n >= kMaxPoints) return fail(c, TPCF_E_INVALID_ARG, "n must be in [0, 2^31)");
  if (!is_finite(box) || !(box > 0.0)) return fail(c, TPCF_E_INVALID_ARG, "box must be finite and > 0");
  if (n > 0 && (!x || !y || !z)) return fail(c, TPCF_E_INVALID_ARG, "NULL position array");
  if (memspace != TPCF_MEM_HOST && memspace != TPCF_MEM_DEVICE)
    return fail(c, TPCF_E_INVALID_ARG, "unknown memory space");
  if (c->bins_set && periodic && !(c->rmax < 0.5 * box))
    return fail(c, TPCF_E_INVALID_ARG, "periodic catalogue needs rmax < box/2");
  std::vector<HostCat> cats(1);
  cats[0].first = 0;
  cats[0].n = n;
  cats[0].box = box;
  cats[0].periodic = periodic ? 1 : 0;
  cats[0].sphere = 0;
  int rc = stage(c, cats, n, x, y, z, w, memspace, f32);
  if (!rc) c->err.clear();
  return rc;
}

// Shared body of tpcf_set_sphere_catalog and tpcf_set_sphere_catalog_f32.
int set_sphere_impl(tpcf_ctx* c, int64_t n, const void* x, const void* y, const void* z, const void* w,
                    int memspace, bool f32) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (n < 0 || n >= kMaxPoints) return fail(c, TPCF_E_INVALID_ARG, "n must be in [0, 2^31)");
  if (n > 0 && (!x || !y || !z)) return fail(c, TPCF_E_INVALID_ARG, "NULL position array");
  if (memspace != TPCF_MEM_HOST && memspace != TPCF_MEM_DEVICE)
    return fail(c, TPCF_E_INVALID_ARG, "unknown memory space");
  if (c->bins_set && !(c->rmax <= kPi))
    return fail(c, TPCF_E_INVALID_ARG, "angular bins on the sphere need theta_max <= pi");
  std::vector<HostCat> cats(1);
  cats[0].first = 0;
  cats[0].n = n;
  cats[0].box = 4.0;
  cats[0].periodic = 0;
  cats[0].sphere = 1;
  int rc = stage(c, cats, n, x, y, z, w, memspace, f32);
  if (!rc) c->err.clear();
  return rc;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// extern "C" entry points
// ------------------------------------------------------------------------------------------
extern "C" {

const char* tpcf_version(void) { return "tpcf 1.0.0 gfx950"; }

int tpcf_create(tpcf_ctx** out, int device, void* hip_stream) {
  if (!out || device < 0) return TPCF_E_INVALID_ARG;
  tpcf_ctx* c = new (std::nothrow) tpcf_ctx();
  if (!c) return TPCF_E_OUT_OF_MEMORY;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return TPCF_OK;
}

void tpcf_destroy(tpcf_ctx* c) {
  if (!c) return;
  if (c->dev_ready) {
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (DevBuf* b : all_bufs(c)) release(*b);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (auto& e : c->ev)
      if (e) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

int tpcf_set_bins(tpcf_ctx* c, int nbins, double rmin, double rmax, int lmax) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (nbins < 1 || nbins > TPCF_MAX_NBINS) return fail(c, TPCF_E_INVALID_ARG, "nbins must be in [1, 32]");
  if (lmax < 0 || lmax > TPCF_MAX_LMAX) return fail(c, TPCF_E_INVALID_ARG, "lmax must be in [0, 10]");
  if (!is_finite(rmin) || !is_finite(rmax) || rmin < 0.0 || !(rmax > rmin))
    return fail(c, TPCF_E_INVALID_ARG, "need finite 0 <= rmin < rmax");
  if (c->cat_set)
    for (const HostCat& h : c->cats) {
      if (h.periodic && !(rmax < 0.5 * h.box))
        return fail(c, TPCF_E_INVALID_ARG, "periodic catalogue needs rmax < box/2");
      if (h.sphere && !(rmax <= kPi))
        return fail(c, TPCF_E_INVALID_ARG, "angular bins on the sphere need theta_max <= pi");
    }
  c->nbins = nbins;
  c->rmin = rmin;
  c->rmax = rmax;
  c->lmax = lmax;
  c->bins_set = true;
  c->err.clear();
  return TPCF_OK;
}

int tpcf_set_precision(tpcf_ctx* c, int precision) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (precision != TPCF_PREC_FP64 && precision != TPCF_PREC_MIXED)
    return fail(c, TPCF_E_INVALID_ARG, "precision must be TPCF_PREC_FP64 or TPCF_PREC_MIXED");
  c->precision = precision;
  c->err.clear();
  return TPCF_OK;
}

// Upper bound of scratch blocks per wave. The sweep addresses a wave's scratch with 32-bit byte
// offsets from the wave's base.
constexpr int kMaxScratchBlocks = 8192;
static_assert((uint64_t)(kMaxScratchBlocks + kScratchTail) * kBlock * 4 < (1ull << 32),
              "a wave's scratch must stay below 4 GiB");

int tpcf_set_tuning(tpcf_ctx* c, double points_per_cell, int waves_per_cu, int scratch_blocks) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (!(points_per_cell >= 0.0) || !is_finite(points_per_cell) || waves_per_cu < 0 || scratch_blocks < 0 ||
      scratch_blocks % 64 != 0 || scratch_blocks > kMaxScratchBlocks || waves_per_cu > 64)
    return fail(c, TPCF_E_INVALID_ARG, "invalid tuning value");
  if (points_per_cell > 0.0) c->ppc = points_per_cell;
  if (waves_per_cu > 0) c->waves_per_cu = waves_per_cu;
  if (scratch_blocks > 0) c->scratch_blocks = scratch_blocks;
  c->err.clear();
  return TPCF_OK;
}

int tpcf_set_allocator(tpcf_ctx* c, tpcf_alloc_fn alloc, tpcf_free_fn free_, void* user) {
  if (!c) return TPCF_E_INVALID_ARG;
  if ((alloc == nullptr) != (free_ == nullptr))
    return fail(c, TPCF_E_INVALID_ARG, "alloc and free must both be set or both be NULL");
  c->alloc_fn = alloc;
  c->free_fn = free_;
  c->alloc_user = alloc ? user : nullptr;
  c->err.clear();
  return TPCF_OK;
}

int tpcf_set_deterministic(tpcf_ctx* c, int enable) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (enable != 0 && enable != 1) return fail(c, TPCF_E_INVALID_ARG, "enable must be 0 or 1");
  c->deterministic = enable == 1;
  c->err.clear();
  return TPCF_OK;
}

int tpcf_set_phase_aligned(tpcf_ctx* c, int mode) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (mode < -1 || mode > 1) return fail(c, TPCF_E_INVALID_ARG, "mode must be -1, 0 or 1");
  c->phase_mode = mode;
  c->err.clear();
  return TPCF_OK;
}

int tpcf_autotune(tpcf_ctx* c, double sample_fraction, tpcf_tuning* out) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (sample_fraction == 0.0) sample_fraction = 0.05;
  if (!(sample_fraction > 0.0 && sample_fraction <= 1.0))
    return fail(c, TPCF_E_INVALID_ARG, "sample_fraction must be in (0, 1]");
  if (!c->bins_set) return fail(c, TPCF_E_STATE, "set_bins has not been called");
  if (!c->cat_set) return fail(c, TPCF_E_STATE, "no catalogue set");
  int rc;
  if ((rc = check_periodic_range(c))) return rc;
  if ((rc = ensure_device(c))) return rc;
  const tpcf_stats saved_stats = c->stats;
  const bool saved_debug = c->debug;
  const double ppc0 = c->ppc;
  const int wpc_set = c->waves_per_cu;
  const int wpc0 = waves_per_cu_for(c);
  const int sb_set = c->scratch_blocks;
  const int sb0 = scratch_blocks_for(c);
  c->debug = false;

  // Up to 16 evenly spaced runs of consecutive cell-sorted points, sample_fraction of all: the
  // runs follow the catalogue's density (the positions are re-sorted per grid density), and
  // consecutive primaries keep the neighbour sharing in cache that the full sweep sees.
  std::vector<uint32_t> list;
  {
    const uint64_t n = (uint64_t)c->ntot;
    const uint64_t want = std::max<uint64_t>(1, (uint64_t)llround((double)n * sample_fraction));
    const uint64_t runs = std::max<uint64_t>(1, std::min<uint64_t>(16, want / 2048));
    for (uint64_t r = 0; r < runs && n > 0; ++r) {
      const uint64_t start = n * r / runs;
      const uint64_t len = want * (r + 1) / runs - want * r / runs;
      for (uint64_t s = start; s < std::min(n, start + len); ++s) list.push_back((uint32_t)s);
    }
  }
  const uint32_t ntask = (uint32_t)list.size();
  if ((rc = ensure(c, c->tasks, std::max<size_t>(1, list.size()) * 4, "task list"))) return rc;
  if (ntask) HIP_TRY(c, hipMemcpyAsync(c->tasks.p, list.data(), list.size() * 4, hipMemcpyHostToDevice, c->stream));

  // Times one configuration: grid for it, one untimed sweep of the sample, then the faster
  // of two timed sweeps.
  auto time_config = [&](double ppc, int wpc, int sb, double& ms) -> int {
    c->ppc = ppc;
    c->waves_per_cu = wpc;
    c->scratch_blocks = sb;
    int r;
    if (!grid_current(c)) {
      if ((r = prepare_grid(c)) || (r = record_grid(c))) return r;
      mark_grid(c);
    }
    SweepArgs a;
    int waves = 0;
    if ((r = prepare_sweep(c, (const uint32_t*)c->tasks.p, ntask, a, waves))) return r;
    if ((r = record_sweep(c, a, waves))) return r;
    ms = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
      HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
      if ((r = record_sweep(c, a, waves))) return r;
      HIP_TRY(c, hipEventRecord(c->ev[3], c->stream));
      HIP_TRY(c, hipEventSynchronize(c->ev[3]));
      float f = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&f, c->ev[2], c->ev[3]));
      ms = std::min(ms, (double)f);
    }
    return TPCF_OK;
  };
  double ms_default = 0.0;
  rc = time_config(ppc0, wpc0, sb0, ms_default);
  if (rc == TPCF_OK)
    log_msg(3, "autotune: %g points per cell, %d waves per CU, %d scratch blocks: %.3f ms (in force)", ppc0, wpc0, sb0,
         ms_default);
  double best_ms = ms_default, best_ppc = ppc0;
  int best_wpc = wpc0, best_sb = sb0, tried = 1;
  auto consider = [&](double ppc, int wpc, int sb) {
    double ms = 0.0;
    rc = time_config(ppc, wpc, sb, ms);
    ++tried;
    if (rc == TPCF_OK) log_msg(3, "autotune: %g points per cell, %d waves per CU, %d scratch blocks: %.3f ms", ppc, wpc, sb, ms);
    if (rc == TPCF_OK && ms < best_ms) {
      best_ms = ms;
      best_ppc = ppc;
      best_wpc = wpc;
      best_sb = sb;
    }
  };
  // Grid densities and wave counts first (12 and 8 per CU), then the pair-list length at the best
  // of them.
  const double ppcs[] = {3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0, 48.0};
  // More waves than fit at once still help the FP64 3D sweep a little: the later ones start as
  // the first finish and keep the tail of the queue short.
  const int wpcs[] = {wpc0, wpc0 == 12 ? 8 : 12};
  for (int wi = 0; wi < 2 && rc == TPCF_OK; ++wi)
    for (int pi = 0; pi < 9 && rc == TPCF_OK; ++pi)
      if (!(ppcs[pi] == ppc0 && wpcs[wi] == wpc0)) consider(ppcs[pi], wpcs[wi], sb0);
  const int sbs[] = {(sb0 / 2) & ~63, (sb0 * 2) & ~63};  // set_tuning takes multiples of 64
  for (int si = 0; si < 2 && rc == TPCF_OK; ++si)
    if (sbs[si] >= kMinRegionBlocks * c->nbins && sbs[si] <= kMaxScratchBlocks && sbs[si] != sb0)
      consider(best_ppc, best_wpc, sbs[si]);
  c->debug = saved_debug;
  c->stats = saved_stats;
  c->dbg_valid = false;  // debug output is kept by sorted position, and the grid was rebuilt
  if (rc) {
    c->ppc = ppc0;
    c->waves_per_cu = wpc_set;
    c->scratch_blocks = sb_set;
    return rc;
  }
  c->ppc = best_ppc;
  c->waves_per_cu = best_wpc;
  c->scratch_blocks = best_sb;
  log_msg(2, "autotune: %g points per cell, %d waves per CU, %d scratch blocks: %.3f ms on the sample (%.3f ms before), "
       "%d configurations", best_ppc, best_wpc, best_sb, best_ms, ms_default, tried);
  if (out) {
    out->points_per_cell = best_ppc;
    out->waves_per_cu = best_wpc;
    out->scratch_blocks = best_sb;
    out->candidates = tried;
    out->ms_best = best_ms;
    out->ms_default = ms_default;
  }
  c->err.clear();
  return TPCF_OK;
}

int tpcf_degenerate(tpcf_ctx* c, double* D, int memspace) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (!c->bins_set) return fail(c, TPCF_E_STATE, "set_bins has not been called");
  if (!c->cat_set) return fail(c, TPCF_E_STATE, "no catalogue set");
  if (!D) return fail(c, TPCF_E_INVALID_ARG, "D is NULL");
  if (memspace != TPCF_MEM_HOST && memspace != TPCF_MEM_DEVICE)
    return fail(c, TPCF_E_INVALID_ARG, "unknown memory space");
  int rc;
  if ((rc = check_periodic_range(c))) return rc;
  if ((rc = ensure_device(c))) return rc;
  if (!grid_current(c)) {
    if ((rc = prepare_grid(c)) || (rc = record_grid(c))) return rc;
    mark_grid(c);
  }
  const size_t n = (size_t)c->ntot;
  const int ncat = (int)c->cd.size(), nb = c->nbins, L = c->lmax;
  if ((rc = ensure(c, c->dg_rec, (n + 1) * sizeof(uint4), "degenerate term")) ||
      (rc = ensure(c, c->dg_w64, (n + 1) * 8, "degenerate term")) ||
      (rc = ensure(c, c->dg_zeta, (size_t)ncat * nb * nb * 8, "degenerate term")) ||
      (rc = ensure(c, c->dg_stats, 16, "degenerate term")) ||
      (rc = ensure(c, c->dg_pairs, (size_t)ncat * nb * 8, "degenerate term")) ||
      (rc = ensure(c, c->dg_dd, (size_t)ncat * nb * 8, "degenerate term")))
    return rc;
  HIP_TRY(c, square_weights((const uint4*)c->rec.p, (const double*)c->w64.p, (uint32_t)(n + 1), (uint4*)c->dg_rec.p,
                            (double*)c->dg_w64.p, c->stream));
  // The sweep at l_max = 0 in FP64 over every point as a primary (its own record and weight),
  // with the squared weights on the secondaries: its two-point by-product is then
  // sum_p w_p sum_{j in b} w_j^2 per bin. The last compute call's outputs stay untouched.
  const int saved_L = c->lmax, saved_prec = c->precision;
  const bool saved_debug = c->debug;
  c->lmax = 0;
  c->precision = TPCF_PREC_FP64;
  c->debug = false;
  SweepArgs a;
  int waves = 0;
  rc = prepare_sweep(c, nullptr, (uint32_t)n, a, waves);
  if (!rc) {
    a.rec = (const uint4*)c->dg_rec.p;
    a.w64 = (const double*)c->dg_w64.p;
    a.prim_rec = (const uint4*)c->rec.p;
    a.prim_w64 = (const double*)c->w64.p;
    a.zeta = (double*)c->dg_zeta.p;
    a.stats = (unsigned long long*)c->dg_stats.p;
    a.bin_pairs = (unsigned long long*)c->dg_pairs.p;
    a.bin_dd = (double*)c->dg_dd.p;
    if (c->deterministic) rc = setup_det(c, point_starts(c), a);
    if (!rc) rc = record_sweep(c, a, waves);
  }
  c->lmax = saved_L;
  c->precision = saved_prec;
  c->debug = saved_debug;
  if (rc) return rc;
  std::vector<double> dd((size_t)ncat * nb), out((size_t)ncat * (L + 1) * nb);
  HIP_TRY(c, hipMemcpyAsync(dd.data(), c->dg_dd.p, dd.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const bool sph = is_sphere(c);
  for (int k = 0; k < ncat; ++k)
    for (int l = 0; l <= L; ++l)
      for (int b = 0; b < nb; ++b)
        out[((size_t)k * (L + 1) + l) * nb + b] = (sph ? 1.0 : (2.0 * l + 1.0) / (4.0 * kPi)) * dd[(size_t)k * nb + b];
  if (memspace == TPCF_MEM_HOST) {
    memcpy(D, out.data(), out.size() * 8);
  } else {
    HIP_TRY(c, hipMemcpyAsync(D, out.data(), out.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  c->err.clear();
  return TPCF_OK;
}

int tpcf_pair_sums(tpcf_ctx* c, int64_t capacity, int64_t* npairs, double* dd) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (!c->sums_valid) return fail(c, TPCF_E_STATE, "no compute call yet");
  const size_t cnt = (size_t)c->sums_ncat * c->sums_nb;
  if (capacity < (int64_t)cnt) return fail(c, TPCF_E_INVALID_ARG, "capacity below ncat x nbins of the last compute call");
  if (npairs) HIP_TRY(c, hipMemcpyAsync(npairs, c->bin_pairs.p, cnt * 8, hipMemcpyDeviceToHost, c->stream));
  if (dd) HIP_TRY(c, hipMemcpyAsync(dd, c->bin_dd.p, cnt * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->err.clear();
  return TPCF_OK;
}

}  // extern "C"

namespace {

// Shared body of the two edge corrections: argument checks, host staging, the launch.
int edge_correct_impl(tpcf_ctx* c, int ncat, const double* N, const double* R, double* zeta, int memspace,
                      bool sphere) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (ncat < 1) return fail(c, TPCF_E_INVALID_ARG, "ncat must be >= 1");
  if (!N || !R || !zeta) return fail(c, TPCF_E_INVALID_ARG, "NULL array");
  if (memspace != TPCF_MEM_HOST && memspace != TPCF_MEM_DEVICE)
    return fail(c, TPCF_E_INVALID_ARG, "unknown memory space");
  if (!c->bins_set) return fail(c, TPCF_E_STATE, "set_bins has not been called");
  if (!sphere && is_sphere(c))
    return fail(c, TPCF_E_UNSUPPORTED,
                "the 3D edge correction couples spherical-harmonic multipoles; use tpcf_edge_correct_sphere");
  int rc;
  if ((rc = ensure_device(c))) return rc;
  const int L = c->lmax, nb = c->nbins;
  const size_t cnt = (size_t)ncat * (L + 1) * nb * nb;
  const double* t3 = nullptr;
  if (!sphere) {
    if (c->edge_lmax != L) {
      const std::vector<double> t = threej_squared_table(L);
      if ((rc = ensure(c, c->edge_tab, t.size() * 8, "3j table"))) return rc;
      HIP_TRY(c, hipMemcpyAsync(c->edge_tab.p, t.data(), t.size() * 8, hipMemcpyHostToDevice, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      c->edge_lmax = L;
    }
    t3 = (const double*)c->edge_tab.p;
  }
  auto launch = [&](const double* n, const double* r, double* z) {
    return sphere ? launch_edge_correct_sphere(ncat, L, nb, n, r, z, c->stream)
                  : launch_edge_correct(ncat, L, nb, n, r, t3, z, c->stream);
  };
  if (memspace == TPCF_MEM_DEVICE) {
    HIP_TRY(c, launch(N, R, zeta));
  } else {
    if ((rc = ensure(c, c->edge_io, cnt * 3 * 8, "edge correction staging"))) return rc;
    double* dN = (double*)c->edge_io.p;
    double* dR = dN + cnt;
    double* dZ = dR + cnt;
    HIP_TRY(c, hipMemcpyAsync(dN, N, cnt * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dR, R, cnt * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch(dN, dR, dZ));
    HIP_TRY(c, hipMemcpyAsync(zeta, dZ, cnt * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  c->err.clear();
  return TPCF_OK;
}

}  // namespace

extern "C" {

int tpcf_edge_correct(tpcf_ctx* c, int ncat, const double* N, const double* R, double* zeta, int memspace) {
  return edge_correct_impl(c, ncat, N, R, zeta, memspace, false);
}

int tpcf_edge_correct_sphere(tpcf_ctx* c, int ncat, const double* N, const double* R, double* zeta, int memspace) {
  return edge_correct_impl(c, ncat, N, R, zeta, memspace, true);
}

int tpcf_set_pivot_cell(tpcf_ctx* c, double side) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (!is_finite(side)) return fail(c, TPCF_E_INVALID_ARG, "pivot cell side must be finite");
  c->pivot_h = side < 0.0 ? -1.0 : side;
  c->err.clear();
  return TPCF_OK;
}

int tpcf_set_debug(tpcf_ctx* c, int enable) {
  if (!c) return TPCF_E_INVALID_ARG;
  c->debug = enable != 0;
  return TPCF_OK;
}

int tpcf_set_catalog(tpcf_ctx* c, int64_t n, const double* x, const double* y, const double* z, const double* w,
                     double box, int periodic, int memspace) {
  return set_catalog_impl(c, n, x, y, z, w, box, periodic, memspace, false);
}

int tpcf_set_catalog_f32(tpcf_ctx* c, int64_t n, const float* x, const float* y, const float* z, const float* w,
                         double box, int periodic, int memspace) {
  return set_catalog_impl(c, n, x, y, z, w, box, periodic, memspace, true);
}

int tpcf_set_sphere_catalog(tpcf_ctx* c, int64_t n, const double* x, const double* y, const double* z,
                            const double* w, int memspace) {
  return set_sphere_impl(c, n, x, y, z, w, memspace, false);
}

int tpcf_set_sphere_catalog_f32(tpcf_ctx* c, int64_t n, const float* x, const float* y, const float* z,
                                const float* w, int memspace) {
  return set_sphere_impl(c, n, x, y, z, w, memspace, true);
}

int tpcf_compute_zeta(tpcf_ctx* c, double* zeta, int memspace) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (c->cat_set && c->cats.size() != 1) return fail(c, TPCF_E_STATE, "context holds a batch; use compute_batch");
  int rc = compute(c, 0, c->ntot, zeta, memspace, false);
  if (!rc) c->err.clear();
  return rc;
}

int tpcf_compute_zeta_range(tpcf_ctx* c, int64_t p_begin, int64_t p_end, double* zeta, int memspace) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (!c->cat_set) return fail(c, TPCF_E_STATE, "no catalogue set");
  if (c->cats.size() != 1) return fail(c, TPCF_E_STATE, "context holds a batch; use compute_batch");
  if (p_begin < 0 || p_end > c->ntot || p_begin > p_end)
    return fail(c, TPCF_E_INVALID_ARG, "primary range outside [0, n]");
  int rc = compute(c, p_begin, p_end, zeta, memspace, false);
  if (!rc) c->err.clear();
  return rc;
}

}  // extern "C"

namespace {

// Validation shared by the batch entry points: the per-catalogue host description.
int batch_cats(tpcf_ctx* c, int ncat, const int64_t* offsets, const double* x, const double* y,
               const double* z, const double* box_side, const int* periodic, const double* zeta,
               std::vector<HostCat>& cats) {
  if (ncat < 1 || !offsets || !box_side || !periodic) return fail(c, TPCF_E_INVALID_ARG, "invalid batch description");
  if (!c->bins_set) return fail(c, TPCF_E_STATE, "set_bins has not been called");
  if (offsets[0] != 0) return fail(c, TPCF_E_INVALID_ARG, "offsets[0] must be 0");
  cats.assign(ncat, HostCat{});
  for (int k = 0; k < ncat; ++k) {
    if (offsets[k + 1] < offsets[k]) return fail(c, TPCF_E_INVALID_ARG, "offsets must be non-decreasing");
    if (!is_finite(box_side[k]) || !(box_side[k] > 0.0))
      return fail(c, TPCF_E_INVALID_ARG, "box must be finite and > 0");
    if (periodic[k] && !(c->rmax < 0.5 * box_side[k]))
      return fail(c, TPCF_E_INVALID_ARG, "periodic catalogue needs rmax < box/2");
    cats[k].first = offsets[k];
    cats[k].n = offsets[k + 1] - offsets[k];
    cats[k].box = box_side[k];
    cats[k].periodic = periodic[k] ? 1 : 0;
    cats[k].sphere = 0;
  }
  const int64_t ntot = offsets[ncat];
  if (ntot >= kMaxPoints) return fail(c, TPCF_E_INVALID_ARG, "total points must be < 2^31");
  if (ntot > 0 && (!x || !y || !z)) return fail(c, TPCF_E_INVALID_ARG, "NULL position array");
  if (!zeta) return fail(c, TPCF_E_INVALID_ARG, "zeta is NULL");
  return TPCF_OK;
}

// Device memory of tpcf_compute_batch_noalloc: a fixed array in the library's code object, one
// copy per GPU, held from the first launch of the library's kernels on that GPU until the process
// ends. Host code never uses the array's name as an address (on the host it stands for a host-side
// shadow): the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoallocScratchBytes = TPCF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::vector<char*> g_scratch_at;  // [device]: device address of that device's copy of scratch

// The device address of scratch on the context's device (current after ensure_device).
int scratch_address(tpcf_ctx* c, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)c->device >= g_scratch_at.size()) g_scratch_at.resize((size_t)c->device + 1, nullptr);
  if (!g_scratch_at[c->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(c, TPCF_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_at[c->device] = static_cast<char*>(p);
  }
  *out = g_scratch_at[c->device];
  return TPCF_OK;
}

}  // namespace

extern "C" {

int tpcf_compute_batch(tpcf_ctx* c, int ncat, const int64_t* offsets, const double* x, const double* y,
                       const double* z, const double* w, const double* box_side, const int* periodic,
                       double* zeta, int memspace) {
  if (!c) return TPCF_E_INVALID_ARG;
  std::vector<HostCat> cats;
  int rc = batch_cats(c, ncat, offsets, x, y, z, box_side, periodic, zeta, cats);
  if (rc) return rc;
  rc = stage(c, cats, offsets[ncat], x, y, z, w, memspace);
  if (rc) return rc;
  rc = compute(c, 0, c->ntot, zeta, memspace, true);
  if (!rc) c->err.clear();
  return rc;
}

int tpcf_compute_batch_noalloc(tpcf_ctx* c, int ncat, const int64_t* offsets, const double* x, const double* y,
                               const double* z, const double* w, const double* box_side, const int* periodic,
                               double* zeta, int memspace) {
  if (!c) return TPCF_E_INVALID_ARG;
  std::vector<HostCat> cats;
  int rc = batch_cats(c, ncat, offsets, x, y, z, box_side, periodic, zeta, cats);
  if (rc) return rc;
  if ((rc = ensure_device(c))) return rc;
  char* base = nullptr;
  if ((rc = scratch_address(c, &base))) return rc;
  // Every device buffer of this call is a slice of scratch; the context's own buffers, catalogue,
  // grid and caches are put back afterwards, whatever happens.
  const tpcf_ctx saved = *c;
  for (DevBuf* b : all_bufs(c)) *b = DevBuf{};
  c->grid_valid = false;
  c->conv_lmax = -1;
  c->regions_key = -1;
  c->edge_lmax = -1;
  c->arena.on = true;
  c->arena.base = base;
  c->arena.cap = kNoallocScratchBytes;
  c->arena.used = 0;
  rc = stage(c, cats, offsets[ncat], x, y, z, w, memspace);
  if (!rc) rc = compute(c, 0, c->ntot, zeta, memspace, false);  // returns after the stream has drained
  if (rc) (void)hipStreamSynchronize(c->stream);  // nothing queued may still use the array after a failure
  const tpcf_stats stats = c->stats;
  const std::string err = rc ? c->err : std::string();
  *c = saved;
  c->stats = stats;
  c->err = err;
  c->sums_valid = false;  // the two-point sums and debug output of this call lived in scratch
  c->dbg_valid = false;
  return rc;
}

int tpcf_compute_sphere_batch(tpcf_ctx* c, int ncat, const int64_t* offsets, const double* x, const double* y,
                              const double* z, const double* w, double* zeta, int memspace) {
  if (!c) return TPCF_E_INVALID_ARG;
  if (ncat < 1 || !offsets) return fail(c, TPCF_E_INVALID_ARG, "invalid batch description");
  if (!c->bins_set) return fail(c, TPCF_E_STATE, "set_bins has not been called");
  if (!(c->rmax <= kPi)) return fail(c, TPCF_E_INVALID_ARG, "angular bins on the sphere need theta_max <= pi");
  if (offsets[0] != 0) return fail(c, TPCF_E_INVALID_ARG, "offsets[0] must be 0");
  std::vector<HostCat> cats(ncat);
  for (int k = 0; k < ncat; ++k) {
    if (offsets[k + 1] < offsets[k]) return fail(c, TPCF_E_INVALID_ARG, "offsets must be non-decreasing");
    cats[k].first = offsets[k];
    cats[k].n = offsets[k + 1] - offsets[k];
    cats[k].box = 4.0;
    cats[k].periodic = 0;
    cats[k].sphere = 1;
  }
  const int64_t ntot = offsets[ncat];
  if (ntot >= kMaxPoints) return fail(c, TPCF_E_INVALID_ARG, "total points must be < 2^31");
  if (ntot > 0 && (!x || !y || !z)) return fail(c, TPCF_E_INVALID_ARG, "NULL position array");
  if (!zeta) return fail(c, TPCF_E_INVALID_ARG, "zeta is NULL");
  int rc = stage(c, cats, ntot, x, y, z, w, memspace);
  if (rc) return rc;
  rc = compute(c, 0, c->ntot, zeta, memspace, true);
  if (!rc) c->err.clear();
  return rc;
}

int tpcf_debug_pair_counts(tpcf_ctx* c, int64_t* counts) {
  if (!c || !counts) return TPCF_E_INVALID_ARG;
  if (!c->dbg_valid) return fail(c, TPCF_E_STATE, "no compute call with debug output enabled");
  int rc;
  DevBuf tmp;
  const size_t tot = (size_t)c->ntot * c->dbg_nb;
  if ((rc = ensure_device(c)) || (rc = ensure(c, tmp, std::max<size_t>(8, tot * 8), "debug staging"))) return rc;
  unsort_counts((const int32_t*)c->counts32.p, (const uint32_t*)c->perm.p, (int64_t*)tmp.p, (uint32_t)c->ntot,
                c->dbg_nb, c->stream);
  hipError_t e = hipMemcpyAsync(counts, tmp.p, tot * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) (void)hipStreamSynchronize(c->stream);
  release(tmp);
  if (e != hipSuccess) return hip_fail(c, e, "tpcf_debug_pair_counts");
  return TPCF_OK;
}

int tpcf_debug_alm(tpcf_ctx* c, double* alm) {
  if (!c || !alm) return TPCF_E_INVALID_ARG;
  if (!c->dbg_valid) return fail(c, TPCF_E_STATE, "no compute call with debug output enabled");
  int rc;
  DevBuf tmp;
  const int row = c->dbg_nb * c->dbg_nc;
  const size_t tot = (size_t)c->ntot * row;
  if ((rc = ensure_device(c)) || (rc = ensure(c, tmp, std::max<size_t>(8, tot * 8), "debug staging"))) return rc;
  unsort_alm(c->alm_dbg.p, c->dbg_f64, (const uint32_t*)c->perm.p, (double*)tmp.p, (uint32_t)c->ntot, row,
             c->stream);
  hipError_t e = hipMemcpyAsync(alm, tmp.p, tot * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) (void)hipStreamSynchronize(c->stream);
  release(tmp);
  if (e != hipSuccess) return hip_fail(c, e, "tpcf_debug_alm");
  return TPCF_OK;
}

int tpcf_get_stats(const tpcf_ctx* c, tpcf_stats* out) {
  if (!c || !out) return TPCF_E_INVALID_ARG;
  *out = c->stats;
  return TPCF_OK;
}

const char* tpcf_last_error(const tpcf_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

}  // extern "C"
