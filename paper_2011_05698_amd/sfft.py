"""Python binding of libsfft.so (ctypes): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory and
streams.  The module-level functions carry the C entry points' names; Plan and
Batch wrap them for convenience.  If the library has not been built, importing
this module raises ImportError: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsfft.so")

SFFT_OK = 0
STATUS = {0: "SFFT_OK", 1: "SFFT_ERR_PARAM", 2: "SFFT_ERR_UNSUPPORTED", 3: "SFFT_ERR_ALLOC",
          4: "SFFT_ERR_LAUNCH", 5: "SFFT_ERR_CAPACITY", 6: "SFFT_ERR_STATE"}
DTYPES = {"c64": 0, "c128": 1, "f16x2": 2}
SFFT_PLAN_HOST_ONLY = 1
MAX_ROUNDS = 48

EXPORTED = [
    "sfft_default_options", "sfft_plan", "sfft_execute", "sfft_execute_noalloc", "sfft_hash_to_bins", "sfft_recover",
    "sfft_get_plan_info", "sfft_get_iter_info", "sfft_plan_dump_tables", "sfft_destroy",
    "sfft_batch_create", "sfft_execute_batch", "sfft_batch_launch_stage", "sfft_batch_destroy",
    "sfft_batch_create_interleaved", "sfft_execute_interleaved", "sfft_plan_set_fold_config", "sfft_batch_set_fold_config", "sfft_batch_autotune", "sfft_batch_get_tuning", "sfft_batch_set_tuning", "sfft_status_string",
    "sfft_last_error",
]


class SfftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("seed", ctypes.c_uint64), ("dtype", ctypes.c_int32),
                ("kahan", ctypes.c_int32), ("b_min", ctypes.c_int32), ("combine", ctypes.c_int32),
                ("eta", ctypes.c_double), ("rho", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("location", ctypes.c_uint32)]


class FoldConfig(ctypes.Structure):
    _fields_ = [("unroll", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("fold_ms", ctypes.c_double)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("fused_chunk", ctypes.c_int32), ("fold_unroll", ctypes.c_int32),
                ("fold_wg_per_cu", ctypes.c_int32), ("fft_group_points", ctypes.c_int32),
                ("fused_available", ctypes.c_int32), ("step_ms", ctypes.c_double), ("fold_lanes", ctypes.c_int32)]


BATCH_MODES = {"stages": 0, "fused": 1}


class PlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("K", ctypes.c_int64), ("B", ctypes.c_int64), ("w", ctypes.c_int64),
                ("loops", ctypes.c_int32), ("multiscale", ctypes.c_int32), ("extension", ctypes.c_double),
                ("delta", ctypes.c_double), ("dtype", ctypes.c_int32), ("kahan", ctypes.c_int32),
                ("samples", ctypes.c_int64), ("yhat_elems", ctypes.c_int64), ("rec_capacity", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("seed", ctypes.c_uint64)]


class IterInfo(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int64), ("L", ctypes.c_int64), ("w", ctypes.c_int64), ("h", ctypes.c_int64),
                ("e", ctypes.c_int64), ("R", ctypes.c_int64), ("d_delta", ctypes.c_double),
                ("sigma", ctypes.c_uint64), ("sigma_inv", ctypes.c_uint64), ("tau0", ctypes.c_uint64),
                ("y_offset", ctypes.c_int64), ("T", ctypes.c_int64 * MAX_ROUNDS),
                ("tau", ctypes.c_int64 * MAX_ROUNDS), ("len", ctypes.c_int64 * MAX_ROUNDS),
                ("last_kind", ctypes.c_int32), ("pad", ctypes.c_int32)]


def _hip_runtimes():
    """Distinct HIP runtime files mapped into this process (Linux)."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({os.path.realpath(ln.split()[-1]) for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # Device buffers and streams come from torch, so the library must run on
    # the HIP runtime torch carries: loading torch first makes the loader
    # bind libsfft's libamdhip64.so.7 to that same copy (equal soname).  Two
    # runtimes in one process see separate device contexts.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError("two HIP runtimes are loaded (" + ", ".join(rts) + "); import torch before any "
                          "library that links the system HIP runtime, then load libsfft")
    vp, i64, i32, f64, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_float
    sig = {
        "sfft_default_options": (None, [ctypes.POINTER(Options)]),
        "sfft_plan": (i32, [ctypes.POINTER(vp), i64, i64, i64, i64, i32, i32, f64, ctypes.POINTER(Options)]),
        "sfft_execute": (i32, [vp, vp, f32, vp, vp, vp, vp]),
        "sfft_execute_noalloc": (i32, [vp, vp, f32, vp, vp, vp, vp]),
        "sfft_hash_to_bins": (i32, [vp, vp, f32, vp, vp]),
        "sfft_recover": (i32, [vp, vp, vp, vp, vp, vp]),
        "sfft_get_plan_info": (i32, [vp, ctypes.POINTER(PlanInfo)]),
        "sfft_get_iter_info": (i32, [vp, i32, ctypes.POINTER(IterInfo)]),
        "sfft_plan_dump_tables": (i32, [vp, i32, vp, vp]),
        "sfft_destroy": (i32, [vp]),
        "sfft_batch_create": (i32, [ctypes.POINTER(vp), ctypes.POINTER(vp), i32]),
        "sfft_execute_batch": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(f32), ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), vp, vp]),
        "sfft_batch_launch_stage": (i32, [vp, i32, vp]),
        "sfft_plan_set_fold_config": (i32, [vp, ctypes.POINTER(FoldConfig)]),
        "sfft_batch_set_fold_config": (i32, [vp, ctypes.POINTER(FoldConfig)]),
        "sfft_batch_autotune": (i32, [vp, vp, ctypes.POINTER(FoldConfig)]),
        "sfft_batch_get_tuning": (i32, [vp, ctypes.POINTER(BatchTuning)]),
        "sfft_batch_set_tuning": (i32, [vp, ctypes.POINTER(BatchTuning)]),
        "sfft_batch_create_interleaved": (i32, [ctypes.POINTER(vp), vp, i32]),
        "sfft_execute_interleaved": (i32, [vp, vp, i64, vp, vp, vp, vp, vp]),
        "sfft_batch_destroy": (i32, [vp]),
        "sfft_status_string": (ctypes.c_char_p, [i32]),
        "sfft_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _check(status):
    if status != SFFT_OK:
        raise SfftError(status, _lib.sfft_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------- C entry points --
def sfft_default_options() -> Options:
    o = Options()
    _lib.sfft_default_options(ctypes.byref(o))
    return o


def sfft_plan(N, K, B, w, loops, multiscale, extension, opt: Options | None = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(_lib.sfft_plan(ctypes.byref(h), N, K, B, w, loops, multiscale, float(extension),
                          None if opt is None else ctypes.byref(opt)))
    return h


def sfft_execute(plan, x, scale, idx, val, count, stream=None):
    _check(_lib.sfft_execute(plan, _ptr(x), float(scale), _ptr(idx), _ptr(val), _ptr(count), _stream(stream)))


def sfft_execute_noalloc(plan, x, scale, idx, val, count, stream=None):
    _check(_lib.sfft_execute_noalloc(plan, _ptr(x), float(scale), _ptr(idx), _ptr(val), _ptr(count),
                                     _stream(stream)))


def sfft_hash_to_bins(plan, x, scale, yhat, stream=None):
    _check(_lib.sfft_hash_to_bins(plan, _ptr(x), float(scale), _ptr(yhat), _stream(stream)))


def sfft_recover(plan, yhat, idx, val, count, stream=None):
    _check(_lib.sfft_recover(plan, _ptr(yhat), _ptr(idx), _ptr(val), _ptr(count), _stream(stream)))


def sfft_get_plan_info(plan) -> PlanInfo:
    info = PlanInfo()
    _check(_lib.sfft_get_plan_info(plan, ctypes.byref(info)))
    return info


def sfft_get_iter_info(plan, m) -> IterInfo:
    info = IterInfo()
    _check(_lib.sfft_get_iter_info(plan, m, ctypes.byref(info)))
    return info


def sfft_plan_dump_tables(plan, m, window: np.ndarray | None, ghat: np.ndarray | None):
    wp = None if window is None else window.ctypes.data_as(ctypes.c_void_p)
    gp = None if ghat is None else ghat.ctypes.data_as(ctypes.c_void_p)
    _check(_lib.sfft_plan_dump_tables(plan, m, wp, gp))


def sfft_destroy(plan):
    _check(_lib.sfft_destroy(plan))


def sfft_batch_create(plans) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(plans))(*[p.value for p in plans])
    h = ctypes.c_void_p()
    _check(_lib.sfft_batch_create(ctypes.byref(h), arr, len(plans)))
    return h


def sfft_execute_batch(batch, xs, scales, idxs, vals, counts, stream=None):
    n = len(xs)
    px = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xs])
    pi = (ctypes.c_void_p * n)(*[t.data_ptr() for t in idxs])
    pv = (ctypes.c_void_p * n)(*[t.data_ptr() for t in vals])
    ps = None if scales is None else (ctypes.c_float * n)(*[float(s) for s in scales])
    _check(_lib.sfft_execute_batch(batch, px, ps, pi, pv, _ptr(counts), _stream(stream)))


def sfft_batch_create_interleaved(plan, nsig):
    h = ctypes.c_void_p()
    _check(_lib.sfft_batch_create_interleaved(ctypes.byref(h), plan, nsig))
    return h


def sfft_execute_interleaved(batch, x, ld, scales, idx, val, counts, stream=None):
    n = len(scales) if scales is not None else None
    ps = None if scales is None else (ctypes.c_float * n)(*[float(s) for s in scales])
    _check(_lib.sfft_execute_interleaved(batch, _ptr(x), ld, ps, _ptr(idx), _ptr(val), _ptr(counts), _stream(stream)))


def sfft_batch_launch_stage(batch, stage, stream=None):
    _check(_lib.sfft_batch_launch_stage(batch, stage, _stream(stream)))


def sfft_plan_set_fold_config(plan, unroll, wg_per_cu):
    c = FoldConfig(unroll, wg_per_cu, 0.0)
    _check(_lib.sfft_plan_set_fold_config(plan, ctypes.byref(c)))


def sfft_batch_set_fold_config(batch, unroll, wg_per_cu):
    c = FoldConfig(unroll, wg_per_cu, 0.0)
    _check(_lib.sfft_batch_set_fold_config(batch, ctypes.byref(c)))


def sfft_batch_autotune(batch, stream=None) -> dict:
    c = FoldConfig()
    _check(_lib.sfft_batch_autotune(batch, _stream(stream), ctypes.byref(c)))
    return {"unroll": c.unroll, "wg_per_cu": c.wg_per_cu, "fold_ms": c.fold_ms}


def sfft_batch_get_tuning(batch) -> dict:
    t = BatchTuning()
    _check(_lib.sfft_batch_get_tuning(batch, ctypes.byref(t)))
    return {"mode": {v: k for k, v in BATCH_MODES.items()}[t.mode], "fused_chunk": t.fused_chunk,
            "fold_unroll": t.fold_unroll, "fold_wg_per_cu": t.fold_wg_per_cu, "fft_group_points": t.fft_group_points,
            "fused_available": bool(t.fused_available), "step_ms": t.step_ms, "fold_lanes": t.fold_lanes}


def sfft_batch_set_tuning(batch, mode, fused_chunk, fold_unroll, fold_wg_per_cu, fft_group_points, fold_lanes=0):
    t = BatchTuning(BATCH_MODES[mode], fused_chunk, fold_unroll, fold_wg_per_cu, fft_group_points, 0, 0.0, fold_lanes)
    _check(_lib.sfft_batch_set_tuning(batch, ctypes.byref(t)))


def sfft_batch_destroy(batch):
    _check(_lib.sfft_batch_destroy(batch))


def sfft_status_string(status) -> str:
    return _lib.sfft_status_string(status).decode()


def sfft_last_error() -> str:
    return _lib.sfft_last_error().decode()


# ------------------------------------------------------------ wrappers --
class Plan:
    """A plan for signals of length N (see sfft_plan in include/sfft.h)."""

    def __init__(self, N, K, B, w, loops, multiscale, extension, *, delta=1e-6, seed=0, dtype="c64",
                 kahan=False, b_min=16, eta=1e-4, rho=0.25, host_only=False, location="multiscale",
                 combine="sum"):
        o = sfft_default_options()
        o.delta, o.seed, o.dtype, o.kahan, o.b_min = delta, seed, DTYPES[dtype], int(kahan), b_min
        o.eta, o.rho = eta, rho
        o.flags = SFFT_PLAN_HOST_ONLY if host_only else 0
        o.location = {"multiscale": 0, "direct": 1}[location]
        o.combine = {"sum": 0, "vote": 1}[combine]
        self.dtype = dtype
        self.handle = sfft_plan(N, K, B, w, loops, multiscale, float(Fraction(extension)), o)
        i = sfft_get_plan_info(self.handle)
        self.N, self.K, self.B, self.w, self.loops = i.N, i.K, i.B, i.w, i.loops
        self.samples, self.yhat_elems = i.samples, i.yhat_elems
        self.workspace_bytes = i.workspace_bytes

    def close(self):
        if self.handle is not None:
            sfft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iteration(self, m) -> dict:
        it = sfft_get_iter_info(self.handle, m)
        R = it.R
        return dict(B=it.B, L=it.L, w=it.w, h=it.h, e=it.e, R=R, d_delta=it.d_delta, sigma=it.sigma,
                    sigma_inv=it.sigma_inv, tau0=it.tau0, y_offset=it.y_offset,
                    T=list(it.T[:R + 1]), tau=list(it.tau[:R + 1]), len=list(it.len[:R + 1]),
                    last_kind=it.last_kind)

    def tables(self, m):
        it = self.iteration(m)
        G = np.zeros(it["h"] + 1)
        Ghat = np.zeros(it["L"] // 2 + it["e"] + 1)
        sfft_plan_dump_tables(self.handle, m, G, Ghat)
        return G, Ghat

    # -- device execution (torch tensors) --
    def _out(self, device):
        import torch
        vdt = torch.complex128 if self.dtype == "c128" else torch.complex64
        return (torch.zeros(self.K, dtype=torch.int64, device=device),
                torch.zeros(self.K, dtype=vdt, device=device),
                torch.zeros(1, dtype=torch.int64, device=device))

    def execute(self, x, scale=1.0, stream=None):
        """Returns device tensors (idx[K], val[K], count[1]); valid after the stream syncs."""
        idx, val, count = self._out(x.device)
        sfft_execute(self.handle, x, scale, idx, val, count, stream)
        return idx, val, count

    def hash_to_bins(self, x, scale=1.0, stream=None):
        import torch
        vdt = torch.complex128 if self.dtype == "c128" else torch.complex64
        y = torch.empty(self.yhat_elems, dtype=vdt, device=x.device)
        sfft_hash_to_bins(self.handle, x, scale, y, stream)
        return y

    def recover(self, yhat, stream=None):
        idx, val, count = self._out(yhat.device)
        sfft_recover(self.handle, yhat, idx, val, count, stream)
        return idx, val, count


class Batch:
    """Many plans executed together (see sfft_batch_create)."""

    def __init__(self, plans):
        self.plans = list(plans)
        self.handle = sfft_batch_create([p.handle for p in self.plans])

    def close(self):
        if self.handle is not None:
            sfft_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def outputs(self, device):
        import torch
        idxs, vals = [], []
        for p in self.plans:
            i, v, _ = p._out(device)
            idxs.append(i)
            vals.append(v)
        counts = torch.zeros(len(self.plans), dtype=torch.int64, device=device)
        return idxs, vals, counts

    def launch_stage(self, stage, stream=None):
        sfft_batch_launch_stage(self.handle, stage, stream)

    def autotune(self, stream=None) -> dict:
        """Time the fold stage over its launch shapes and keep the fastest
        (needs buffers bound by a prior execute)."""
        return sfft_batch_autotune(self.handle, stream)

    def tuning(self) -> dict:
        return sfft_batch_get_tuning(self.handle)

    def set_tuning(self, **kw):
        """Changes some fields of the batch's tuning (see sfft_batch_tuning)."""
        t = self.tuning()
        t.update(kw)
        sfft_batch_set_tuning(self.handle, t["mode"], t["fused_chunk"], t["fold_unroll"], t["fold_wg_per_cu"],
                              t["fft_group_points"], t["fold_lanes"])

    def set_fold_config(self, unroll, wg_per_cu):
        sfft_batch_set_fold_config(self.handle, unroll, wg_per_cu)

    def execute(self, xs, scales=None, outs=None, stream=None):
        if outs is None:
            outs = self.outputs(xs[0].device)
        idxs, vals, counts = outs
        sfft_execute_batch(self.handle, xs, scales, idxs, vals, counts, stream)
        return idxs, vals, counts


class InterleavedBatch(Batch):
    """nsig signals sharing one plan, stored position-major: x[c, s] is sample
    c of signal s (a tensor of shape [N, ld] with ld >= nsig, or [N, ld, 2]
    float16 for the F16X2 form; see sfft_batch_create_interleaved)."""

    def __init__(self, plan, nsig):
        self.plans = [plan] * nsig
        self.plan = plan
        self.nsig = nsig
        self.handle = sfft_batch_create_interleaved(plan.handle, nsig)

    def outputs(self, device):
        import torch
        vdt = torch.complex128 if self.plan.dtype == "c128" else torch.complex64
        return (torch.zeros((self.nsig, self.plan.K), dtype=torch.int64, device=device),
                torch.zeros((self.nsig, self.plan.K), dtype=vdt, device=device),
                torch.zeros(self.nsig, dtype=torch.int64, device=device))

    def execute(self, x, scales=None, outs=None, stream=None):
        if outs is None:
            outs = self.outputs(x.device)
        pair = x.dim() == 3  # float16 (re, im) pairs
        ok = x.shape[0] == self.plan.N and x.shape[1] >= self.nsig and (
            (not pair and x.dim() == 2 and x.stride(1) == 1) or
            (pair and x.shape[2] == 2 and x.stride(2) == 1 and x.stride(1) == 2 and x.stride(0) % 2 == 0))
        if not ok:
            raise ValueError("x must be [N, ld] (or [N, ld, 2] float16) with ld >= nsig, contiguous along signals")
        idx, val, counts = outs
        ld = x.stride(0) // 2 if pair else x.stride(0)
        sfft_execute_interleaved(self.handle, x, ld, scales, idx, val, counts, stream)
        return idx, val, counts
