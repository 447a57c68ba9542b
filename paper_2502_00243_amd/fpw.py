"""ctypes binding of libfpw (include/fpw.h), with torch tensors for device memory.

Argument marshalling only: every step of the periodogram runs in the HIP
library.  Loading fails loudly when ``libfpw.so`` has not been built; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpw.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fpw.h")

# status codes
OK, EINVAL, ENOMEM, EHIP, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "FPW_OK", -1: "FPW_EINVAL", -2: "FPW_ENOMEM", -3: "FPW_EHIP", -4: "FPW_ESTATE", -5: "FPW_EUNSUPPORTED"}

CENTER = {"weighted": 0, "mean": 1, "none": 2}
TREF = {"zero": 0, "first": 1, "given": 2}
PHASE = {"fp64": 0, "fp64_listing": 1, "df32": 2, "fp32": 3}
STAT = {"eq1": 0, "listing_half": 1}
SHARED_KERNEL = {"auto": 0, "general": 1, "matrix": 2}
SUM_FORMAT = {"auto": 0, "wide": 1}
MAX_BINS = 255
MAX_TOPK = 16


class FpwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("n_bins", ctypes.c_int32),
        ("center", ctypes.c_int32),
        ("tref_mode", ctypes.c_int32),
        ("phase", ctypes.c_int32),
        ("stat_scale", ctypes.c_int32),
        ("topk", ctypes.c_int32),
        ("inv_alpha2", ctypes.c_double),
        ("t_ref", ctypes.c_double),
        ("autotune", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("freqs_per_lane", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
        ("chunk_freqs", ctypes.c_int32),
        ("tune_cache", ctypes.c_char_p),
        ("point_source", ctypes.c_int32),
        ("derived_bins", ctypes.c_int32 * 4),
        ("all_offsets", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("shared_kernel", ctypes.c_int32),
        ("baseline_terms", ctypes.c_int32),
        ("baseline_scale", ctypes.c_double),
        ("hist_share", ctypes.c_int32),
        ("fuse_prepare", ctypes.c_int32),
        ("sum_format", ctypes.c_int32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_curves", ctypes.c_int64),
        ("n_freq", ctypes.c_int64),
        ("n_points", ctypes.c_int64),
        ("evals", ctypes.c_int64),
        ("n_bins", ctypes.c_int32),
        ("topk", ctypes.c_int32),
        ("phase", ctypes.c_int32),
        ("freqs_per_lane", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
        ("chunk_freqs", ctypes.c_int32),
        ("grid_groups", ctypes.c_int32),
        ("work_items", ctypes.c_int32),
        ("lds_bytes", ctypes.c_int32),
        ("tuned", ctypes.c_int32),
        ("point_source", ctypes.c_int32),
        ("n_variants", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("hist_share", ctypes.c_int32),
        ("fuse_prepare", ctypes.c_int32),
        ("n_wide_curves", ctypes.c_int32),
        ("n_wide_points", ctypes.c_int64),
    ]


_lib = None


def header_functions() -> list[str]:
    """Names of the functions include/fpw.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fpw_[a-z0-9_]+)\s*\(", text)))


def load(path: str = LIB_PATH):
    """Loads libfpw.so (once).  torch is imported first so both share one HIP runtime."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (binds the process to torch's HIP runtime first)
    except ImportError:
        pass
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_2502_00243_amd.build_lib` "
            "(the FPW periodogram has no CPU fallback)"
        )
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    dp = ctypes.POINTER(ctypes.c_double)
    lib.fpw_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.fpw_options_default.restype = None
    lib.fpw_plan.argtypes = [ctypes.POINTER(P), i64, ctypes.POINTER(i64), dp, dp, dp, i64, dp, ctypes.POINTER(Options), P]
    lib.fpw_plan.restype = ctypes.c_int
    lib.fpw_plan_shared.argtypes = [ctypes.POINTER(P), i64, i64, dp, dp, dp, i64, dp, ctypes.POINTER(Options), P]
    lib.fpw_plan_shared.restype = ctypes.c_int
    lib.fpw_eval_batch.argtypes = [P, P, P, P, P]
    lib.fpw_eval_batch.restype = ctypes.c_int
    lib.fpw_topk.argtypes = [P, P, i32, P, P, P]
    lib.fpw_topk.restype = ctypes.c_int
    lib.fpw_eval_fp64.argtypes = [P, P, P]
    lib.fpw_eval_fp64.restype = ctypes.c_int
    lib.fpw_debug_bins.argtypes = [P, i32, i64, i64, i64, P, P]
    lib.fpw_debug_bins.restype = ctypes.c_int
    lib.fpw_pass_timings.argtypes = [P, ctypes.POINTER(ctypes.c_float)]
    lib.fpw_pass_timings.restype = ctypes.c_int
    lib.fpw_pass_wide_ms.argtypes = [P, ctypes.POINTER(ctypes.c_float)]
    lib.fpw_pass_wide_ms.restype = ctypes.c_int
    lib.fpw_phase_entropy.argtypes = [P, P, i32, P, P, P, P]
    lib.fpw_phase_entropy.restype = ctypes.c_int
    lib.fpw_variant.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.fpw_variant.restype = ctypes.c_int
    lib.fpw_get_plan_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    lib.fpw_get_plan_info.restype = ctypes.c_int
    lib.fpw_eval_static.argtypes = [i64, P, i64, P, P, P, i64, P, ctypes.POINTER(Options), P, P, P, P]
    lib.fpw_eval_static.restype = ctypes.c_int
    lib.fpw_plan_destroy.argtypes = [P]
    lib.fpw_plan_destroy.restype = None
    lib.fpw_last_error.argtypes = []
    lib.fpw_last_error.restype = ctypes.c_char_p
    lib.fpw_version.argtypes = []
    lib.fpw_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        raise FpwError(status, load().fpw_last_error().decode())


def default_options() -> Options:
    o = Options()
    load().fpw_options_default(ctypes.byref(o))
    return o


def make_options(n_bins: int, center="weighted", tref="zero", t_ref=0.0, phase="fp64", stat_scale="eq1", topk=0,
                 inv_alpha2=0.0, autotune=False, use_graph=True, freqs_per_lane=0, waves_per_group=0, chunk_freqs=0,
                 tune_cache=None, profile=False, point_source=0, derived_bins=(), all_offsets=False,
                 shared_kernel=0, baseline_terms=0, baseline_scale=1.0, hist_share=0,
                 fuse_prepare=0, sum_format=0) -> Options:
    o = default_options()
    o.n_bins = int(n_bins)
    o.center = CENTER[center] if isinstance(center, str) else int(center)
    o.tref_mode = TREF[tref] if isinstance(tref, str) else int(tref)
    o.t_ref = float(t_ref)
    o.phase = PHASE[phase] if isinstance(phase, str) else int(phase)
    o.stat_scale = STAT[stat_scale] if isinstance(stat_scale, str) else int(stat_scale)
    o.topk = int(topk)
    o.inv_alpha2 = float(inv_alpha2)
    o.autotune = int(bool(autotune))
    o.use_graph = int(bool(use_graph))
    o.freqs_per_lane = int(freqs_per_lane)
    o.waves_per_group = int(waves_per_group)
    o.chunk_freqs = int(chunk_freqs)
    o.tune_cache = tune_cache.encode() if tune_cache else None
    o.profile = int(bool(profile))
    o.point_source = {"auto": 0, "scalar": 1, "dpp": 2}[point_source] if isinstance(point_source, str) else int(point_source)
    if len(derived_bins) > 4:
        raise ValueError("at most 4 derived bin counts")
    for i in range(4):
        o.derived_bins[i] = int(derived_bins[i]) if i < len(derived_bins) else 0
    o.all_offsets = int(bool(all_offsets))
    o.shared_kernel = SHARED_KERNEL[shared_kernel] if isinstance(shared_kernel, str) else int(shared_kernel)
    o.baseline_terms = int(baseline_terms)
    o.baseline_scale = float(baseline_scale)
    o.hist_share = int(hist_share)
    o.fuse_prepare = int(fuse_prepare)
    o.sum_format = SUM_FORMAT[sum_format] if isinstance(sum_format, str) else int(sum_format)
    return o


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check_out(t, dtype, numel, name):
    """Output buffers the kernels write: device, contiguous, of the plan's dtype and size."""
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name} must be a contiguous device tensor of {numel} {dtype} elements "
                         f"(got {tuple(t.shape)} {t.dtype} on {t.device})")


def _stream_handle(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A planned batch: light curves (CSR offsets + concatenated t, y, dy) and a frequency grid."""

    def __init__(self, offsets, t, y, dy, freqs, n_bins, stream=None, **opts):
        lib = load()
        self._offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self._t, self._y, self._dy, self._freqs = _f64(t), _f64(y), _f64(dy), _f64(freqs)
        self.options = make_options(n_bins, **opts)
        self.n_curves = len(self._offsets) - 1
        self.n_freq = len(self._freqs)
        self.n_bins = int(n_bins)
        self.topk_k = int(opts.get("topk", 0))
        h = ctypes.c_void_p()
        st = lib.fpw_plan(ctypes.byref(h), self.n_curves, _ptr(self._offsets, ctypes.c_int64), _ptr(self._t, ctypes.c_double),
                          _ptr(self._y, ctypes.c_double), _ptr(self._dy, ctypes.c_double), self.n_freq,
                          _ptr(self._freqs, ctypes.c_double), ctypes.byref(self.options), _stream_handle(stream))
        _check(st)
        self._h = h
        self.n_variants = self.info().n_variants

    @classmethod
    def shared(cls, t, y, dy, freqs, n_bins, stream=None, **opts):
        """A plan for curves observed at common times: t [n_points], y and dy [n_curves, n_points]."""
        lib = load()
        self = cls.__new__(cls)
        self._t = _f64(t)
        y2, dy2 = np.asarray(y, dtype=np.float64), np.asarray(dy, dtype=np.float64)
        if y2.ndim != 2 or y2.shape != dy2.shape or y2.shape[1] != len(self._t):
            raise ValueError("y and dy must be [n_curves, n_points] with n_points = len(t)")
        self._y, self._dy, self._freqs = _f64(y2), _f64(dy2), _f64(freqs)
        self.options = make_options(n_bins, **opts)
        self.n_curves = int(y2.shape[0])
        self.n_freq = len(self._freqs)
        self.n_bins = int(n_bins)
        self.topk_k = int(opts.get("topk", 0))
        self._offsets = np.arange(self.n_curves + 1, dtype=np.int64) * len(self._t)
        h = ctypes.c_void_p()
        st = lib.fpw_plan_shared(ctypes.byref(h), self.n_curves, len(self._t), _ptr(self._t, ctypes.c_double),
                                 _ptr(self._y, ctypes.c_double), _ptr(self._dy, ctypes.c_double), self.n_freq,
                                 _ptr(self._freqs, ctypes.c_double), ctypes.byref(self.options), _stream_handle(stream))
        _check(st)
        self._h = h
        self.n_variants = self.info().n_variants
        return self

    @classmethod
    def from_batch(cls, batch, stream=None, **opts):
        n_bins = opts.pop("n_bins", batch.n_bins)
        return cls(batch.offsets, batch.t, batch.y, batch.dy, batch.freqs, n_bins, stream=stream, **opts)

    # -------------------------------------------------------------- calls
    def eval(self, store_s=True, topk=None, S_out=None, idx_out=None, val_out=None, stream=None):
        """One pass; returns (S [n_curves, n_freq] float32 or None, idx, val) as device tensors."""
        import torch

        if topk is None:
            topk = self.topk_k > 0
        S = S_out
        nv = self.n_variants
        lead = (nv,) if nv > 1 else ()
        if S is not None:
            _check_out(S, torch.float32, nv * self.n_curves * self.n_freq, "S_out")
        elif store_s:
            S = torch.empty(lead + (self.n_curves, self.n_freq), dtype=torch.float32, device="cuda")
        idx = val = None
        if topk:
            shp = lead + (self.n_curves, self.topk_k)
            idx = idx_out if idx_out is not None else torch.empty(shp, dtype=torch.int32, device="cuda")
            val = val_out if val_out is not None else torch.empty(shp, dtype=torch.float32, device="cuda")
            _check_out(idx, torch.int32, nv * self.n_curves * self.topk_k, "idx_out")
            _check_out(val, torch.float32, nv * self.n_curves * self.topk_k, "val_out")
        _check(load().fpw_eval_batch(self._h, ctypes.c_void_p(S.data_ptr() if S is not None else 0),
                                     ctypes.c_void_p(idx.data_ptr() if idx is not None else 0),
                                     ctypes.c_void_p(val.data_ptr() if val is not None else 0), _stream_handle(stream)))
        return S, idx, val

    def topk(self, S, k, stream=None):
        """Peaks of a stored periodogram S (device float32 [n_curves, n_freq])."""
        import torch

        assert S.dtype == torch.float32 and S.is_cuda and S.is_contiguous()
        assert tuple(S.shape) == (self.n_curves, self.n_freq)
        idx = torch.empty((self.n_curves, k), dtype=torch.int32, device="cuda")
        val = torch.empty((self.n_curves, k), dtype=torch.float32, device="cuda")
        _check(load().fpw_topk(self._h, ctypes.c_void_p(S.data_ptr()), int(k), ctypes.c_void_p(idx.data_ptr()),
                               ctypes.c_void_p(val.data_ptr()), _stream_handle(stream)))
        return idx, val

    def eval_fp64(self, stream=None):
        """The plain per-curve FP64 comparator: S [n_curves, n_freq] float64 on the device."""
        import torch

        S = torch.empty((self.n_curves, self.n_freq), dtype=torch.float64, device="cuda")
        _check(load().fpw_eval_fp64(self._h, ctypes.c_void_p(S.data_ptr()), _stream_handle(stream)))
        return S

    def debug_bins(self, curve, f_begin, f_end, phase=None, stream=None):
        """Bin of every point of `curve` at frequencies f_begin..f_end-1: int32 [f_end-f_begin, N_curve]."""
        import torch

        if phase is None:
            phase = self.options.phase
        elif isinstance(phase, str):
            phase = PHASE[phase]
        n = int(self._offsets[curve + 1] - self._offsets[curve])
        out = torch.empty((f_end - f_begin, n), dtype=torch.int32, device="cuda")
        _check(load().fpw_debug_bins(self._h, int(phase), int(curve), int(f_begin), int(f_end),
                                     ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def timings(self):
        """(prepare, fold, merge) kernel milliseconds of the last eval (plan made with profile=True); the fold
        time covers the batched kernel and, with wide-format curves, the wide kernel (see wide_ms)."""
        ms = (ctypes.c_float * 3)()
        _check(load().fpw_pass_timings(self._h, ms))
        return float(ms[0]), float(ms[1]), float(ms[2])

    def wide_ms(self):
        """Milliseconds of the fold time of the last eval spent in the wide-format kernel (0 if none ran)."""
        ms = ctypes.c_float()
        _check(load().fpw_pass_wide_ms(self._h, ctypes.byref(ms)))
        return float(ms.value)

    def phase_entropy(self, freq_idx, stream=None):
        """(H, E, V) of the phase occupancy at freq_idx (device int32 [n_curves, k]), App. C."""
        import torch

        assert freq_idx.dtype == torch.int32 and freq_idx.is_cuda and freq_idx.is_contiguous()
        assert freq_idx.dim() == 2 and freq_idx.shape[0] == self.n_curves
        k = int(freq_idx.shape[1])
        H = torch.empty_like(freq_idx, dtype=torch.float32)
        E = torch.empty_like(H)
        V = torch.empty_like(H)
        _check(load().fpw_phase_entropy(self._h, ctypes.c_void_p(freq_idx.data_ptr()), k, ctypes.c_void_p(H.data_ptr()),
                                        ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                        _stream_handle(stream)))
        return H, E, V

    def variant(self, v):
        """(bin count, offset) of periodogram variant v."""
        m, o = ctypes.c_int32(), ctypes.c_int32()
        _check(load().fpw_variant(self._h, int(v), ctypes.byref(m), ctypes.byref(o)))
        return m.value, o.value

    def info(self) -> PlanInfo:
        inf = PlanInfo()
        _check(load().fpw_get_plan_info(self._h, ctypes.byref(inf)))
        return inf

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            load().fpw_plan_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def eval_static(offsets, t, y, dy, freqs, n_bins, store_s=True, stream=None, S_out=None, idx_out=None, val_out=None,
                **opts):
    """fpw_eval_static: one pass with no plan and no allocation by the library.

    offsets (int64), t, y, dy, freqs (float64) are device tensors; returns (S [n_curves, n_freq] or None,
    idx, val) as device tensors (peaks when opts has topk > 0).  Outputs may be passed preallocated."""
    import torch

    for name, a, dt in (("offsets", offsets, torch.int64), ("t", t, torch.float64), ("y", y, torch.float64),
                        ("dy", dy, torch.float64), ("freqs", freqs, torch.float64)):
        if not (a.is_cuda and a.dtype == dt and a.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dt} device tensor")
    n_curves, n_points, n_freq = offsets.numel() - 1, t.numel(), freqs.numel()
    if y.numel() != n_points or dy.numel() != n_points:
        raise ValueError("t, y and dy must have the same length")
    o = make_options(n_bins, **opts)
    S = S_out if S_out is not None else (
        torch.empty((n_curves, n_freq), dtype=torch.float32, device="cuda") if store_s else None)
    idx = val = None
    if o.topk > 0:
        idx = idx_out if idx_out is not None else torch.empty((n_curves, o.topk), dtype=torch.int32, device="cuda")
        val = val_out if val_out is not None else torch.empty((n_curves, o.topk), dtype=torch.float32, device="cuda")
    addr = lambda x: ctypes.c_void_p(x.data_ptr() if x is not None else 0)  # noqa: E731
    _check(load().fpw_eval_static(n_curves, addr(offsets), n_points, addr(t), addr(y), addr(dy), n_freq, addr(freqs),
                                  ctypes.byref(o), addr(S), addr(idx), addr(val), _stream_handle(stream)))
    return S, idx, val


def plan_status(offsets, t, y, dy, freqs, n_bins, **opts):
    """Calls fpw_plan and returns (status, message) without raising (for argument-check tests)."""
    lib = load()
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    t, y, dy, freqs = _f64(t), _f64(y), _f64(dy), _f64(freqs)
    o = make_options(n_bins, **opts)
    h = ctypes.c_void_p()
    st = lib.fpw_plan(ctypes.byref(h), len(offsets) - 1, _ptr(offsets, ctypes.c_int64), _ptr(t, ctypes.c_double),
                      _ptr(y, ctypes.c_double), _ptr(dy, ctypes.c_double), len(freqs), _ptr(freqs, ctypes.c_double),
                      ctypes.byref(o), ctypes.c_void_p(0))
    msg = lib.fpw_last_error().decode()
    if st == OK and h:
        lib.fpw_plan_destroy(h)
    return st, msg


def plan_shared_status(t, y, dy, freqs, n_bins, **opts):
    """Calls fpw_plan_shared and returns (status, message) without raising (for argument-check tests)."""
    lib = load()
    t, y, dy, freqs = _f64(t), _f64(y), _f64(dy), _f64(freqs)
    if y.ndim != 2 or y.shape != dy.shape or y.shape[1] != len(t):
        raise ValueError("y and dy must be [n_curves, n_points] with n_points = len(t)")
    n_curves = y.shape[0]
    o = make_options(n_bins, **opts)
    h = ctypes.c_void_p()
    st = lib.fpw_plan_shared(ctypes.byref(h), n_curves, len(t), _ptr(t, ctypes.c_double), _ptr(y, ctypes.c_double),
                             _ptr(dy, ctypes.c_double), len(freqs), _ptr(freqs, ctypes.c_double), ctypes.byref(o),
                             ctypes.c_void_p(0))
    msg = lib.fpw_last_error().decode()
    if st == OK and h:
        lib.fpw_plan_destroy(h)
    return st, msg
