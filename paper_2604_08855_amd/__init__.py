"""Three-point correlation function multipoles on MI355X (gfx950).

Python binding of ``libtpcf.so`` (the C ABI declared in ``include/tpcf.h``). This module only
marshals arguments: numpy arrays are passed as host memory, torch CUDA/HIP tensors as device
memory on the tensor's device and the current stream. Every step of the computation runs in the
library's HIP kernels; when the library is missing, importing this package fails.

    import paper_2604_08855_amd as tpcf
    z = tpcf.zeta(x, y, z, w, box=1000.0, periodic=True, rmin=10.0, rmax=200.0, nbins=20,
                  lmax=10, precision="mixed")      # -> float64 [(lmax+1), nbins, nbins]
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Context", "zeta", "TpcfError", "library_path", "exported_symbols", "PREC_FP64", "PREC_MIXED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# TPCF_LIBRARY_PATH may name another build of the same library (for example one with host-side
# sanitizers); by default the in-tree libtpcf.so is loaded.
_LIB_PATH = os.environ.get("TPCF_LIBRARY_PATH") or os.path.join(_HERE, "libtpcf.so")

TPCF_OK = 0
ERRORS = {1: "INVALID_ARG", 2: "STATE", 3: "OUT_OF_MEMORY", 4: "DEVICE", 5: "UNSUPPORTED"}
PREC_FP64, PREC_MIXED = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1

# Every function the header declares.
EXPORTS = [
    "tpcf_version", "tpcf_create", "tpcf_destroy", "tpcf_set_bins", "tpcf_set_precision",
    "tpcf_set_tuning", "tpcf_set_catalog", "tpcf_compute_zeta", "tpcf_compute_zeta_range",
    "tpcf_compute_batch", "tpcf_debug_pair_counts", "tpcf_debug_alm", "tpcf_set_debug",
    "tpcf_get_stats", "tpcf_last_error", "tpcf_autotune", "tpcf_pair_sums", "tpcf_edge_correct",
    "tpcf_set_sphere_catalog", "tpcf_set_pivot_cell", "tpcf_edge_correct_sphere", "tpcf_compute_sphere_batch",
    "tpcf_set_phase_aligned", "tpcf_set_deterministic", "tpcf_degenerate", "tpcf_set_allocator", "tpcf_set_catalog_f32",
    "tpcf_set_sphere_catalog_f32", "tpcf_compute_batch_noalloc",
]


class TpcfError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"tpcf error {ERRORS.get(code, code)}: {message}")
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [
        ("points_per_cell", ctypes.c_double),
        ("waves_per_cu", ctypes.c_int),
        ("scratch_blocks", ctypes.c_int),
        ("candidates", ctypes.c_int),
        ("ms_best", ctypes.c_double),
        ("ms_default", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_int64),
        ("n_candidates", ctypes.c_int64),
        ("n_primaries", ctypes.c_int64),
        ("ms_grid", ctypes.c_double),
        ("ms_sweep", ctypes.c_double),
        ("ms_total", ctypes.c_double),
        ("cells_per_axis", ctypes.c_int),
        ("waves", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("lmax", ctypes.c_int),
        ("nbins", ctypes.c_int),
    ]


def library_path() -> str:
    return _LIB_PATH


def _load() -> ctypes.CDLL:
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is not built: run `python paper_2604_08855_amd/build.py` (needs hipcc)")
    # torch wheels bundle their own HIP runtime. Loading torch first lets the library bind to
    # that runtime (same soname), so a process never holds two HIP runtimes side by side.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "tpcf_version": ([], ctypes.c_char_p),
        "tpcf_create": ([ctypes.POINTER(vp), i, vp], i),
        "tpcf_destroy": ([vp], None),
        "tpcf_set_bins": ([vp, i, d, d, i], i),
        "tpcf_set_precision": ([vp, i], i),
        "tpcf_set_tuning": ([vp, d, i, i], i),
        "tpcf_set_phase_aligned": ([vp, i], i),
        "tpcf_set_deterministic": ([vp, i], i),
        "tpcf_degenerate": ([vp, vp, i], i),
        "tpcf_set_allocator": ([vp, vp, vp, vp], i),
        "tpcf_set_catalog_f32": ([vp, i64, vp, vp, vp, vp, d, i, i], i),
        "tpcf_set_sphere_catalog_f32": ([vp, i64, vp, vp, vp, vp, i], i),
        "tpcf_set_catalog": ([vp, i64, vp, vp, vp, vp, d, i, i], i),
        "tpcf_compute_zeta": ([vp, vp, i], i),
        "tpcf_compute_zeta_range": ([vp, i64, i64, vp, i], i),
        "tpcf_compute_batch": ([vp, i, vp, vp, vp, vp, vp, vp, vp, vp, i], i),
        "tpcf_compute_batch_noalloc": ([vp, i, vp, vp, vp, vp, vp, vp, vp, vp, i], i),
        "tpcf_debug_pair_counts": ([vp, vp], i),
        "tpcf_debug_alm": ([vp, vp], i),
        "tpcf_set_debug": ([vp, i], i),
        "tpcf_get_stats": ([vp, ctypes.POINTER(Stats)], i),
        "tpcf_last_error": ([vp], ctypes.c_char_p),
        "tpcf_autotune": ([vp, d, ctypes.POINTER(Tuning)], i),
        "tpcf_pair_sums": ([vp, i64, vp, vp], i),
        "tpcf_edge_correct": ([vp, i, vp, vp, vp, i], i),
        "tpcf_set_sphere_catalog": ([vp, i64, vp, vp, vp, vp, i], i),
        "tpcf_set_pivot_cell": ([vp, d], i),
        "tpcf_edge_correct_sphere": ([vp, i, vp, vp, vp, i], i),
        "tpcf_compute_sphere_batch": ([vp, i, vp, vp, vp, vp, vp, vp, i], i),
    }
    missing = [name for name in sig if not hasattr(lib, name)]
    if missing:
        raise ImportError(f"{_LIB_PATH} is stale (no {', '.join(missing)}): rebuild it with "
                          "`python paper_2604_08855_amd/build.py`")
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def exported_symbols() -> list:
    """Names of the C-ABI functions present in the loaded library."""
    return [n for n in EXPORTS if hasattr(_lib, n)]


def version() -> str:
    return _lib.tpcf_version().decode()


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _host_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr_np(a) -> ctypes.c_void_p:
    return a.ctypes.data_as(ctypes.c_void_p)


# tpcf_alloc_fn / tpcf_free_fn
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Context:
    """One library context (one device, one stream). Not thread-safe."""

    def __init__(self, device: int = 0, stream=None):
        self._h = ctypes.c_void_p()
        self.device = device
        sh = None
        if stream is None:
            # Device tensors are produced on torch's current stream: use it when torch is in use.
            import sys
            torch = sys.modules.get("torch")
            if torch is not None and torch.cuda.is_available():
                stream = torch.cuda.current_stream(device)
        if stream is not None:
            sh = getattr(stream, "cuda_stream", stream)
        self._check(_lib.tpcf_create(ctypes.byref(self._h), int(device),
                                     ctypes.c_void_p(sh) if sh else None))
        self._stream_ptr = int(sh) if sh else 0
        self.nbins = self.lmax = None
        self.n = 0
        self.ncat = 0
        self.sphere = False
        self._keep = []

    # -- plumbing
    def _check(self, rc: int):
        if rc != TPCF_OK:
            msg = _lib.tpcf_last_error(self._h).decode() if self._h else ""
            raise TpcfError(rc, msg)

    def close(self):
        if self._h:
            _lib.tpcf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- configuration
    def set_bins(self, nbins: int, rmin: float, rmax: float, lmax: int):
        self._check(_lib.tpcf_set_bins(self._h, int(nbins), float(rmin), float(rmax), int(lmax)))
        self.nbins, self.rmin, self.rmax, self.lmax = int(nbins), float(rmin), float(rmax), int(lmax)

    def set_precision(self, precision):
        p = {"fp64": PREC_FP64, "mixed": PREC_MIXED}.get(precision, precision)
        self._check(_lib.tpcf_set_precision(self._h, int(p)))

    def set_tuning(self, points_per_cell: float = 0.0, waves_per_cu: int = 0, scratch_blocks: int = 0):
        self._check(_lib.tpcf_set_tuning(self._h, float(points_per_cell), int(waves_per_cu),
                                         int(scratch_blocks)))

    def use_torch_allocator(self):
        """Routes the context's device buffers through torch's caching allocator on the context's
        stream (tpcf_set_allocator), so that they show in torch's memory statistics and reuse its
        pool. The callbacks stay referenced by the context."""
        import torch

        dev, stream = self.device, self._stream_ptr

        @_ALLOC_FN
        def _alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            except Exception:  # out of memory or a bad size: the library reports the failure
                return None

        @_FREE_FN
        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc_cbs = (_alloc, _free)
        self._check(_lib.tpcf_set_allocator(self._h, ctypes.cast(_alloc, ctypes.c_void_p),
                                            ctypes.cast(_free, ctypes.c_void_p), None))

    def set_deterministic(self, enable: bool = True):
        """Bit-for-bit reproducible results: fixed tiles and a fixed-order reduction
        (see tpcf_set_deterministic)."""
        self._check(_lib.tpcf_set_deterministic(self._h, 1 if enable else 0))

    def set_phase_aligned(self, mode: int = -1):
        """Phase-aligned stencil sweeps: -1 by neighbourhood size (default), 0 off, 1 on
        (see tpcf_set_phase_aligned)."""
        self._check(_lib.tpcf_set_phase_aligned(self._h, int(mode)))

    def autotune(self, sample_fraction: float = 0.0) -> dict:
        """Times the sweep on a sample of primaries of the staged catalogue(s) for several grid
        densities and wave counts and keeps the fastest (see tpcf_autotune)."""
        t = Tuning()
        self._check(_lib.tpcf_autotune(self._h, float(sample_fraction), ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def set_pivot_cell(self, side: float):
        """Shared pivots (approximate): pivot cells of this side (catalogue units); a negative value
        means the mean separation, 0 the exact estimator (see tpcf_set_pivot_cell)."""
        self._check(_lib.tpcf_set_pivot_cell(self._h, float(side)))

    def set_debug(self, enable: bool = True):
        self._check(_lib.tpcf_set_debug(self._h, int(bool(enable))))

    # -- inputs
    def _arrays(self, x, y, z, w):
        """(pointers, memspace, keep-alive list) for host numpy or device torch arrays."""
        if _is_torch(x):
            import torch
            ts = [t.contiguous().to(torch.float64) for t in (x, y, z)]
            wt = None if w is None else w.contiguous().to(torch.float64)
            if not ts[0].is_cuda:
                ts = [t.numpy() for t in ts]
                wt = None if wt is None else wt.numpy()
                return self._arrays(*ts, wt)
            keep = ts + ([wt] if wt is not None else [])
            ptrs = [ctypes.c_void_p(t.data_ptr()) for t in ts]
            ptrs.append(ctypes.c_void_p(wt.data_ptr()) if wt is not None else None)
            return ptrs, MEM_DEVICE, keep
        arrs = [_host_f64(a) for a in (x, y, z)]
        wa = None if w is None else _host_f64(w)
        ptrs = [_ptr_np(a) for a in arrs] + [_ptr_np(wa) if wa is not None else None]
        return ptrs, MEM_HOST, arrs + ([wa] if wa is not None else [])

    def _f32_arrays(self, x, y, z, w):
        """(pointers, memspace, keep-alive list) when every array is FP32 (numpy, or torch on the
        device), else None: FP32 inputs go to the _f32 entry points, which widen them exactly."""
        arrs = [a for a in (x, y, z, w) if a is not None]
        if all(_is_torch(a) for a in arrs):
            import torch

            if not all(a.is_cuda and a.dtype == torch.float32 for a in arrs):
                return None
            ts = [a.contiguous() for a in (x, y, z)]
            wt = None if w is None else w.contiguous()
            ptrs = [ctypes.c_void_p(t.data_ptr()) for t in ts]
            ptrs.append(ctypes.c_void_p(wt.data_ptr()) if wt is not None else None)
            return ptrs, MEM_DEVICE, ts + ([wt] if wt is not None else [])
        if all(isinstance(a, np.ndarray) and a.dtype == np.float32 for a in arrs):
            hs = [np.ascontiguousarray(a) for a in (x, y, z)]
            wh = None if w is None else np.ascontiguousarray(w)
            ptrs = [_ptr_np(a) for a in hs] + [_ptr_np(wh) if wh is not None else None]
            return ptrs, MEM_HOST, hs + ([wh] if wh is not None else [])
        return None

    def set_catalog(self, x, y, z, w=None, *, box: float, periodic: bool = True):
        n = len(x)
        if len(y) != n or len(z) != n or (w is not None and len(w) != n):
            raise ValueError("x, y, z, w must have the same length")
        f32 = self._f32_arrays(x, y, z, w)
        if f32 is not None:
            ptrs, mem, keep = f32
            self._check(_lib.tpcf_set_catalog_f32(self._h, int(n), *ptrs, float(box), int(bool(periodic)), mem))
            self.n, self.ncat, self.sphere = n, 1, False
            return
        ptrs, mem, keep = self._arrays(x, y, z, w)
        self._check(_lib.tpcf_set_catalog(self._h, int(n), *ptrs, float(box), int(bool(periodic)), mem))
        self.n, self.ncat, self.sphere = n, 1, False

    def set_sphere_catalog(self, x, y, z, w=None):
        """A projected field on the unit sphere: unit vectors x, y, z and field values w (see
        tpcf_set_sphere_catalog). The bins of set_bins are then angles in radians and lmax is
        m_max; compute_zeta returns zeta_m(b1, b2), m = 0..m_max."""
        n = len(x)
        if len(y) != n or len(z) != n or (w is not None and len(w) != n):
            raise ValueError("x, y, z, w must have the same length")
        f32 = self._f32_arrays(x, y, z, w)
        if f32 is not None:
            ptrs, mem, keep = f32
            self._check(_lib.tpcf_set_sphere_catalog_f32(self._h, int(n), *ptrs, mem))
        else:
            ptrs, mem, keep = self._arrays(x, y, z, w)
            self._check(_lib.tpcf_set_sphere_catalog(self._h, int(n), *ptrs, mem))
        self.n, self.ncat, self.sphere = n, 1, True

    # -- compute
    def _out(self, like_device: bool, shape):
        if like_device:
            import torch
            t = torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.device}")
            return t, ctypes.c_void_p(t.data_ptr()), MEM_DEVICE
        a = np.zeros(shape)
        return a, _ptr_np(a), MEM_HOST

    def compute_zeta(self, device_output: bool = False):
        out, p, mem = self._out(device_output, (self.lmax + 1, self.nbins, self.nbins))
        self._check(_lib.tpcf_compute_zeta(self._h, p, mem))
        return out

    def compute_zeta_range(self, p_begin: int, p_end: int, device_output: bool = False):
        out, p, mem = self._out(device_output, (self.lmax + 1, self.nbins, self.nbins))
        self._check(_lib.tpcf_compute_zeta_range(self._h, int(p_begin), int(p_end), p, mem))
        return out

    def compute_batch(self, offsets, x, y, z, w, box, periodic, device_output: bool = False):
        return self._batch(_lib.tpcf_compute_batch, offsets, x, y, z, w, box, periodic, device_output)

    def compute_batch_noalloc(self, offsets, x, y, z, w, box, periodic, out=None):
        """compute_batch through tpcf_compute_batch_noalloc: the library allocates no device memory
        (its buffers are slices of a fixed static array per GPU). With torch CUDA inputs pass `out`,
        a preallocated float64 CUDA tensor [ncat, (lmax+1), nbins, nbins], to keep the call free of
        allocations on the Python side as well."""
        return self._batch(_lib.tpcf_compute_batch_noalloc, offsets, x, y, z, w, box, periodic, False, out)

    def _batch(self, fn, offsets, x, y, z, w, box, periodic, device_output, out=None):
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        ncat = len(offsets) - 1
        box = np.ascontiguousarray(np.broadcast_to(np.asarray(box, dtype=np.float64), (ncat,)))
        per = np.ascontiguousarray(np.broadcast_to(np.asarray(periodic, dtype=np.int32), (ncat,)))
        ptrs, mem, keep = self._arrays(x, y, z, w)
        shape = (ncat, self.lmax + 1, self.nbins, self.nbins)
        if out is not None:
            if not (_is_torch(out) and out.is_cuda and mem == MEM_DEVICE):
                raise ValueError("out must be a CUDA tensor, with CUDA inputs")
            import torch
            if tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous():
                raise ValueError(f"out must be a contiguous float64 tensor of shape {shape}")
            p, omem = ctypes.c_void_p(out.data_ptr()), MEM_DEVICE
        else:
            out, p, omem = self._out(device_output or mem == MEM_DEVICE, shape)
        if omem != mem:
            raise ValueError("batch inputs and output must be in the same memory space")
        self._check(fn(self._h, ncat, _ptr_np(offsets), *ptrs, _ptr_np(box), _ptr_np(per), p, mem))
        self.n, self.ncat, self.sphere = int(offsets[-1]), ncat, False
        return out

    def compute_sphere_batch(self, offsets, x, y, z, w=None, device_output: bool = False):
        """ncat independent maps on the sphere in one launch (see tpcf_compute_sphere_batch):
        zeta [ncat, (m_max+1), nbins, nbins]."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        ncat = len(offsets) - 1
        ptrs, mem, keep = self._arrays(x, y, z, w)
        out, p, omem = self._out(device_output or mem == MEM_DEVICE, (ncat, self.lmax + 1, self.nbins, self.nbins))
        if omem != mem:
            raise ValueError("batch inputs and output must be in the same memory space")
        self._check(_lib.tpcf_compute_sphere_batch(self._h, ncat, _ptr_np(offsets), *ptrs, p, mem))
        self.n, self.ncat, self.sphere = int(offsets[-1]), ncat, True
        return out

    def degenerate(self):
        """The j = k part of zeta's diagonal for the staged catalogue(s) (see tpcf_degenerate):
        float64 [ncat, (lmax+1), nbins]; zeta_l(b, b) - D_l(b) counts triangles of distinct points."""
        L, nb = (self.lmax or 0), (self.nbins or 1)
        D = np.zeros((max(self.ncat, 1), L + 1, nb))
        self._check(_lib.tpcf_degenerate(self._h, _ptr_np(D), MEM_HOST))
        return D

    def pair_sums(self):
        """Two-point by-product of the last compute call: (npairs int64 [ncat, nbins] ordered
        pairs per bin, dd float64 [ncat, nbins] sum of w_p w_j per bin)."""
        nb = self.stats()["nbins"]
        npairs = np.zeros((max(self.ncat, 1), max(nb, 1)), dtype=np.int64)
        dd = np.zeros(npairs.shape)
        self._check(_lib.tpcf_pair_sums(self._h, npairs.size, _ptr_np(npairs), _ptr_np(dd)))
        return npairs, dd

    def edge_correct(self, N, R):
        """Edge-corrected multipoles N(mu)/R(mu) per bin pair (see tpcf_edge_correct; on the
        sphere tpcf_edge_correct_sphere, the cosine coefficients of N(phi)/R(phi)). N, R:
        [(lmax+1), nbins, nbins] or [ncat, (lmax+1), nbins, nbins], numpy (host) or torch
        CUDA tensors (device); the result has the same shape and kind."""
        fn = _lib.tpcf_edge_correct_sphere if self.sphere else _lib.tpcf_edge_correct
        if _is_torch(N):
            import torch
            Nt = N.contiguous().to(torch.float64)
            Rt = R.contiguous().to(torch.float64)
            if Nt.shape != Rt.shape:
                raise ValueError("N and R must have the same shape")
            out = torch.empty_like(Nt)
            ncat = 1 if Nt.dim() == 3 else Nt.shape[0]
            self._check(fn(self._h, ncat, ctypes.c_void_p(Nt.data_ptr()), ctypes.c_void_p(Rt.data_ptr()),
                           ctypes.c_void_p(out.data_ptr()), MEM_DEVICE))
            return out
        Na, Ra = _host_f64(N), _host_f64(R)
        if Na.shape != Ra.shape:
            raise ValueError("N and R must have the same shape")
        out = np.zeros_like(Na)
        ncat = 1 if Na.ndim == 3 else Na.shape[0]
        self._check(fn(self._h, ncat, _ptr_np(Na), _ptr_np(Ra), _ptr_np(out), MEM_HOST))
        return out

    # -- debug and statistics
    def pair_counts(self) -> np.ndarray:
        out = np.zeros((self.n, self.nbins), dtype=np.int64)
        self._check(_lib.tpcf_debug_pair_counts(self._h, _ptr_np(out)))
        return out

    def alm_real(self) -> np.ndarray:
        nc = 2 * self.lmax + 1 if self.sphere else (self.lmax + 1) ** 2
        out = np.zeros((self.n, self.nbins, nc))
        self._check(_lib.tpcf_debug_alm(self._h, _ptr_np(out)))
        return out

    def alm(self) -> np.ndarray:
        """a_lm for m >= 0 as complex [n, nbins, lmax+1, lmax+1] (index [.., l, m]); on the sphere
        a_m as complex [n, nbins, m_max+1]."""
        r = self.alm_real()
        L = self.lmax
        if self.sphere:
            out = np.zeros(r.shape[:2] + (L + 1,), dtype=np.complex128)
            out[..., 0] = r[..., 0]
            for m in range(1, L + 1):
                out[..., m] = r[..., 2 * m - 1] + 1j * r[..., 2 * m]
            return out
        out = np.zeros(r.shape[:2] + (L + 1, L + 1), dtype=np.complex128)
        for l in range(L + 1):
            out[..., l, 0] = r[..., l * l]
            for m in range(1, l + 1):
                out[..., l, m] = r[..., l * l + 2 * m - 1] + 1j * r[..., l * l + 2 * m]
        return out

    def stats(self) -> dict:
        s = Stats()
        self._check(_lib.tpcf_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}


def zeta_sphere(x, y=None, z=None, w=None, *, theta_min: float, theta_max: float, nbins: int, mmax: int,
                precision="fp64", device: int = 0, stream=None):
    """zeta_m(b1, b2) of a field on the unit sphere (unit vectors x, y, z or one [N, 3] array x;
    angles in radians), float64 [(mmax+1), nbins, nbins]."""
    if y is None and z is None:
        x, y, z = _columns(x)
    with Context(device, stream) as ctx:
        ctx.set_bins(nbins, theta_min, theta_max, mmax)
        ctx.set_precision(precision)
        ctx.set_sphere_catalog(x, y, z, w)
        return ctx.compute_zeta(device_output=_is_torch(x) and x.is_cuda)


def _columns(pos):
    """(x, y, z) of an [N, 3] position array (numpy or torch), each contiguous."""
    if _is_torch(pos):
        return tuple(pos[:, k].contiguous() for k in range(3))
    pos = np.asarray(pos, dtype=np.float64)
    if pos.ndim != 2 or pos.shape[1] != 3:
        raise ValueError("positions must be an [N, 3] array or three arrays x, y, z")
    return tuple(np.ascontiguousarray(pos[:, k]) for k in range(3))


def _concat(cats):
    """offsets and concatenated x, y, z, w (w None if no catalogue has weights) of a sequence of
    catalogues, each (x, y, z), (x, y, z, w) or ([N, 3] positions, w)."""
    parts = []
    for c in cats:
        c = tuple(c)
        if len(c) == 2:
            parts.append((*_columns(c[0]), c[1]))
        elif len(c) in (3, 4):
            parts.append((c[0], c[1], c[2], c[3] if len(c) == 4 else None))
        else:
            raise ValueError("a catalogue is (x, y, z), (x, y, z, w) or (positions, w)")
    host = [tuple(None if a is None else (a.detach().cpu().numpy() if _is_torch(a) else np.asarray(a, dtype=np.float64))
                  for a in p) for p in parts]
    n = [len(p[0]) for p in host]
    offsets = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    xyz = [np.concatenate([p[k] for p in host]) if host else np.zeros(0) for k in range(3)]
    w = None
    if any(p[3] is not None for p in host):
        w = np.concatenate([p[3] if p[3] is not None else np.ones(len(p[0])) for p in host])
    return offsets, xyz[0], xyz[1], xyz[2], w


def zeta_batch(catalogues, *, box, periodic=True, rmin: float, rmax: float, nbins: int, lmax: int,
               precision="mixed", device: int = 0, stream=None):
    """zeta_l of many independent catalogues in one persistent launch (tpcf_compute_batch):
    catalogues is a sequence of (x, y, z), (x, y, z, w) or ([N, 3] positions, w); box and periodic
    are one value or one per catalogue. float64 [ncat, (lmax+1), nbins, nbins]."""
    offsets, x, y, z, w = _concat(catalogues)
    with Context(device, stream) as ctx:
        ctx.set_bins(nbins, rmin, rmax, lmax)
        ctx.set_precision(precision)
        return ctx.compute_batch(offsets, x, y, z, w, box, periodic)


def zeta_sphere_batch(maps, *, theta_min: float, theta_max: float, nbins: int, mmax: int, precision="mixed",
                      device: int = 0, stream=None):
    """zeta_m of many independent maps on the unit sphere in one launch (tpcf_compute_sphere_batch):
    maps is a sequence of (x, y, z), (x, y, z, w) or ([N, 3] unit vectors, w).
    float64 [nmaps, (mmax+1), nbins, nbins]."""
    offsets, x, y, z, w = _concat(maps)
    with Context(device, stream) as ctx:
        ctx.set_bins(nbins, theta_min, theta_max, mmax)
        ctx.set_precision(precision)
        return ctx.compute_sphere_batch(offsets, x, y, z, w)


def zeta(x, y=None, z=None, w=None, *, box: float, periodic: bool = True, rmin: float, rmax: float,
         nbins: int, lmax: int, precision="fp64", device: int = 0, stream=None):
    """zeta_l(b1, b2) of one catalogue, float64 [(lmax+1), nbins, nbins]. Positions are x, y, z or
    one [N, 3] array x (numpy or torch) with y = z = None."""
    if y is None and z is None:
        x, y, z = _columns(x)
    with Context(device, stream) as ctx:
        ctx.set_bins(nbins, rmin, rmax, lmax)
        ctx.set_precision(precision)
        ctx.set_catalog(x, y, z, w, box=box, periodic=periodic)
        return ctx.compute_zeta(device_output=_is_torch(x) and x.is_cuda)
