"""Python binding of libqfca, the gfx950 implementation of the Quantized FCA
score-map path (Ardelean, Rueckbeil, Weyrich, "Quantized FCA: Efficient
Zero-Shot Texture Anomaly Detection").

Argument marshalling only: every step runs in the HIP library.  The entry
points keep the C names (qfca_fit_pca, qfca_quantize, qfca_score_map, ...);
tensors are torch tensors on a HIP device, passed by pointer on the context's
stream (by default torch's current stream).  There is no CPU fallback: if the
library is not built, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqfca.so")

QFCA_PRE_NONE, QFCA_PRE_RESIDUAL, QFCA_PRE_COORDS = 0, 1, 2
QFCA_PREC_FP32, QFCA_PREC_BF16 = 0, 1
QFCA_REF_MEDIAN_QUAN, QFCA_REF_MEAN_QUAN, QFCA_REF_QUAN_MEDIAN, QFCA_REF_QUAN_MEAN = 0, 1, 2, 3

STATUS = {0: "QFCA_OK", 1: "QFCA_E_ARG", 2: "QFCA_E_SHAPE", 3: "QFCA_E_NOMEM", 4: "QFCA_E_DEVICE",
          5: "QFCA_E_STATE", 6: "QFCA_E_NONFINITE", 7: "QFCA_E_UNSUPPORTED"}

# Symbols declared in include/qfca.h
EXPORTS = ("qfca_status_str", "qfca_last_error", "qfca_version", "qfca_ctx_create",
           "qfca_ctx_set_stream", "qfca_ctx_destroy", "qfca_fit_pca", "qfca_model_create",
           "qfca_fit_reference", "qfca_quantize", "qfca_score_map", "qfca_model_params",
           "qfca_model_read", "qfca_model_destroy", "qfca_model_export", "qfca_model_import",
           "qfca_host_sym_eig", "qfca_host_sym_eig_top", "qfca_ctx_profile",
           "qfca_ctx_profile_read", "qfca_ctx_set_tile", "qfca_score_batch", "qfca_batch_error",
           "qfca_autotune", "qfca_clock", "qfca_server_create", "qfca_server_submit",
           "qfca_server_poll", "qfca_server_drain", "qfca_server_stats", "qfca_server_destroy",
           "qfca_inspect_windows", "qfca_score_map_noalloc", "qfca_model_set_reference")

KERNELS = {"score": 0, "proj": 1, "finish": 2}


class QfcaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("C", ctypes.c_int32), ("k", ctypes.c_int32), ("B", ctypes.c_int32),
                ("T", ctypes.c_int32), ("q_lo", ctypes.c_float), ("q_hi", ctypes.c_float),
                ("sigma_s", ctypes.c_float), ("preproc", ctypes.c_int32),
                ("proj_prec", ctypes.c_int32), ("sigma_p", ctypes.c_float), ("reference", ctypes.c_int32)]

    @classmethod
    def make(cls, C, k=10, B=16, T=9, q_lo=0.01, q_hi=0.99, sigma_s=1.0,
             preproc=QFCA_PRE_RESIDUAL, proj_prec=QFCA_PREC_FP32, sigma_p=float("inf"),
             reference=QFCA_REF_MEDIAN_QUAN):
        return cls(int(C), int(k), int(B), int(T), float(q_lo), float(q_hi), float(sigma_s),
                   int(preproc), int(proj_prec), float(sigma_p), int(reference))

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Job(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("X", ctypes.c_void_p), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32), ("score", ctypes.c_void_p), ("bins", ctypes.c_void_p),
                ("amap", ctypes.c_void_p), ("achan", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("Ws", ctypes.c_int32), ("Hb", ctypes.c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("deferred_memory", ctypes.c_uint64),
                ("max_inflight_seen", ctypes.c_int32), ("max_batch_seen", ctypes.c_int32),
                ("arena_bytes", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64),
                ("device_busy_s", ctypes.c_double), ("device_span_s", ctypes.c_double),
                ("overlapped", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libqfca.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        L.qfca_status_str.restype = ctypes.c_char_p
        L.qfca_status_str.argtypes = [i32]
        L.qfca_last_error.restype = ctypes.c_char_p
        L.qfca_version.restype = i32
        L.qfca_ctx_create.argtypes = [i32, P, ctypes.POINTER(P)]
        L.qfca_ctx_set_stream.argtypes = [P, P]
        L.qfca_ctx_destroy.argtypes = [P]
        L.qfca_fit_pca.argtypes = [P, ctypes.POINTER(Params), P, i32, i32, ctypes.POINTER(P)]
        L.qfca_model_create.argtypes = [P, ctypes.POINTER(Params), P, P, P, P, P, ctypes.POINTER(P)]
        L.qfca_fit_reference.argtypes = [P, P, P, i32, i32]
        L.qfca_quantize.argtypes = [P, P, P, i32, i32, P, P]
        L.qfca_score_map.argtypes = [P, P, P, i32, i32, P, P, P, P]
        L.qfca_inspect_windows.argtypes = [P, P, P, i32, i32, P, P]
        L.qfca_score_map_noalloc.argtypes = [P, P, P, i32, i32, P, P, P, P]
        L.qfca_model_set_reference.argtypes = [P, P, P]
        L.qfca_model_params.argtypes = [P, ctypes.POINTER(Params)]
        L.qfca_model_read.argtypes = [P, i32, P, sz]
        L.qfca_model_destroy.argtypes = [P]
        L.qfca_model_export.argtypes = [P, P, ctypes.POINTER(sz)]
        L.qfca_model_import.argtypes = [P, P, sz, ctypes.POINTER(P)]
        L.qfca_host_sym_eig.argtypes = [P, i32, P, P]
        L.qfca_host_sym_eig.restype = i32
        L.qfca_host_sym_eig_top.argtypes = [P, i32, i32, P, P]
        L.qfca_host_sym_eig_top.restype = i32
        L.qfca_ctx_profile.argtypes = [P, i32]
        L.qfca_ctx_set_tile.argtypes = [P, i32, i32, i32, i32]
        L.qfca_score_batch.argtypes = [P, ctypes.POINTER(Job), i32]
        L.qfca_batch_error.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.qfca_autotune.argtypes = [P, ctypes.POINTER(Job), i32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
        L.qfca_ctx_profile_read.argtypes = [P, i32, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int64)]
        L.qfca_clock.restype = ctypes.c_double
        L.qfca_clock.argtypes = []
        L.qfca_server_create.argtypes = [i32, ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]
        L.qfca_server_submit.argtypes = [P, P, P, i32, i32, P, ctypes.POINTER(ctypes.c_uint64)]
        L.qfca_server_poll.argtypes = [P, ctypes.POINTER(Completion), i32, ctypes.POINTER(ctypes.c_int32)]
        L.qfca_server_drain.argtypes = [P]
        L.qfca_server_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
        L.qfca_server_destroy.argtypes = [P]
        for name in ("qfca_server_create", "qfca_server_submit", "qfca_server_poll", "qfca_server_drain",
                     "qfca_server_stats", "qfca_server_destroy"):
            getattr(L, name).restype = i32
        for name in ("qfca_ctx_create", "qfca_ctx_set_stream", "qfca_ctx_destroy", "qfca_fit_pca",
                     "qfca_model_create", "qfca_fit_reference", "qfca_quantize", "qfca_score_map",
                     "qfca_model_params", "qfca_model_read", "qfca_model_destroy", "qfca_model_export",
                     "qfca_model_import",
                     "qfca_ctx_profile", "qfca_ctx_profile_read", "qfca_ctx_set_tile",
                     "qfca_score_batch", "qfca_batch_error", "qfca_autotune", "qfca_inspect_windows",
                     "qfca_score_map_noalloc", "qfca_model_set_reference"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise QfcaError(rc, lib().qfca_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_tensor(t, dtype, name, ndim=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return t


class Context:
    """A libqfca context on one device, issuing work on a HIP stream (torch's
    current stream of that device unless given)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().qfca_ctx_create(self.device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().qfca_ctx_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))

    def set_tile(self, Ws=0, Hb=0, S=0, variant=1):
        """Pin the score kernel's tile (Ws=0 restores the automatic choice)."""
        _check(lib().qfca_ctx_set_tile(self.handle, int(Ws), int(Hb), int(S), int(variant)))

    def profile(self, enable: bool = True, kernels=None):
        """Event timing of every kernel, or of the named ones (see KERNELS)."""
        mask = 0 if not enable else (-1 if kernels is None else sum(1 << KERNELS[k] for k in kernels))
        _check(lib().qfca_ctx_profile(self.handle, mask))

    def profile_read(self, kernel: str):
        """(total_ms, launches) of one kernel since the previous read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().qfca_ctx_profile_read(self.handle, KERNELS[kernel], ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().qfca_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


FIELDS = {"mu": (0, np.float32), "V": (1, np.float32), "edges": (2, np.float32),
          "delta": (3, np.float64), "cR": (4, np.int32), "evals": (5, np.float64),
          "lo": (6, np.float64), "hi": (7, np.float64), "cRw": (8, np.float64)}


class Model:
    def __init__(self, handle):
        self.handle = handle
        p = Params()
        _check(lib().qfca_model_params(handle, ctypes.byref(p)))
        self.params = p

    @property
    def planes(self) -> int:
        """Histogrammed planes: the k principal coordinates (PRE_COORDS) or the C channels."""
        p = self.params
        return p.k if p.preproc == QFCA_PRE_COORDS else p.C

    def read(self, field: str) -> np.ndarray:
        fid, dt = FIELDS[field]
        p = self.params
        P = self.planes
        shape = {"mu": (p.C,), "V": (p.C, p.k), "edges": (P, max(p.B - 1, 0)), "delta": (P,),
                 "cR": (P, p.B), "evals": (p.C,), "lo": (P,), "hi": (P,), "cRw": (P, p.B)}[field]
        out = np.zeros(shape, dt)
        _check(lib().qfca_model_read(self.handle, fid, out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().qfca_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)

def qfca_model_set_reference(ctx: Context, model: Model, cRw):
    """General reference: cumulative weights [C, B] (host, float64)."""
    w = np.ascontiguousarray(cRw, dtype=np.float64)
    if w.shape != (model.params.C, model.params.B):
        raise ValueError("cRw must be [C, B]")
    _check(lib().qfca_model_set_reference(ctx.handle, model.handle, w.ctypes.data_as(ctypes.c_void_p)))


def qfca_fit_pca(ctx: Context, params: Params, X) -> Model:
    import torch
    X = _dev_tensor(X, torch.float32, "X", 3)
    C, H, W = X.shape
    if C != params.C:
        raise ValueError("X.shape[0] != params.C")
    h = ctypes.c_void_p()
    _check(lib().qfca_fit_pca(ctx.handle, ctypes.byref(params), _ptr(X), H, W, ctypes.byref(h)))
    return Model(h)


def qfca_model_create(ctx: Context, params: Params, mu, V, edges, delta, cR=None) -> Model:
    def host(a, dt):
        return None if a is None else np.ascontiguousarray(a, dtype=dt)
    mu, V, edges = host(mu, np.float32), host(V, np.float32), host(edges, np.float32)
    delta, cR = host(delta, np.float64), host(cR, np.int32)
    C, B, k = params.C, params.B, params.k
    P = k if params.preproc == QFCA_PRE_COORDS else C  # histogrammed planes
    if edges is not None and edges.size != P * max(B - 1, 0):
        raise ValueError("edges must be [planes, B-1]")
    if delta is None or delta.size != P:
        raise ValueError("delta must be [planes]")
    if cR is not None and cR.size != P * B:
        raise ValueError("cR must be [planes, B]")
    if params.preproc != QFCA_PRE_NONE and k > 0:
        if mu is None or V is None or mu.size != C or V.size != C * k:
            raise ValueError("mu [C] and V [C, k] are required")

    def p(a):
        return None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    h = ctypes.c_void_p()
    _check(lib().qfca_model_create(ctx.handle, ctypes.byref(params), p(mu), p(V), p(edges), p(delta),
                                   p(cR), ctypes.byref(h)))
    return Model(h)


def qfca_model_export(model: Model) -> bytes:
    """Serialised model (host bytes); see qfca_model_export in include/qfca.h."""
    n = ctypes.c_size_t(0)
    _check(lib().qfca_model_export(model.handle, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().qfca_model_export(model.handle, buf, ctypes.byref(n)))
    return buf.raw[: n.value]


def qfca_model_import(ctx: Context, blob: bytes) -> Model:
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    h = ctypes.c_void_p()
    _check(lib().qfca_model_import(ctx.handle, buf, len(blob), ctypes.byref(h)))
    return Model(h)


def qfca_fit_reference(ctx: Context, model: Model, bins):
    import torch
    bins = _dev_tensor(bins, torch.uint8, "bins", 3)
    _check(lib().qfca_fit_reference(ctx.handle, model.handle, _ptr(bins), bins.shape[1], bins.shape[2]))


def qfca_quantize(ctx: Context, model: Model, X, bins=None, resid=None, want_bins=True):
    """Returns (bins uint8 [C,H,W] or None, resid float32 [C,H,W] or None).
    Pass resid=True to allocate the residual output."""
    import torch
    X = _dev_tensor(X, torch.float32, "X", 3)
    C, H, W = X.shape
    if C != model.params.C:
        raise ValueError("X.shape[0] != model C")
    P = model.planes
    if bins is None and want_bins:
        bins = torch.empty((P, H, W), dtype=torch.uint8, device=X.device)
    if resid is True:
        resid = torch.empty((P, H, W), dtype=torch.float32, device=X.device)
    elif resid is False:
        resid = None
    if bins is not None:
        _dev_tensor(bins, torch.uint8, "bins", 3)
    if resid is not None:
        _dev_tensor(resid, torch.float32, "resid", 3)
    _check(lib().qfca_quantize(ctx.handle, model.handle, _ptr(X), H, W, _ptr(bins), _ptr(resid)))
    return bins, resid


@dataclass
class ScoreMaps:
    score: object
    amap: object = None
    w1: object = None
    achan: object = None


def qfca_score_map(ctx: Context, model: Model, bins, amap=False, w1=False, achan=False,
                   out: ScoreMaps | None = None) -> ScoreMaps:
    import torch
    bins = _dev_tensor(bins, torch.uint8, "bins", 3)
    C, H, W = bins.shape
    if C != model.planes:
        raise ValueError("bins.shape[0] != the model's histogrammed planes")
    dev = bins.device
    if out is None:
        out = ScoreMaps(torch.empty((H, W), dtype=torch.float32, device=dev))
        if amap:
            out.amap = torch.empty((H, W), dtype=torch.float32, device=dev)
        if w1:
            out.w1 = torch.empty((H, W), dtype=torch.float32, device=dev)
        if achan:
            out.achan = torch.empty((C, H, W), dtype=torch.float32, device=dev)
    _check(lib().qfca_score_map(ctx.handle, model.handle, _ptr(bins), H, W, _ptr(out.score),
                                _ptr(out.amap), _ptr(out.w1), _ptr(out.achan)))
    return out


def _jobs(items):
    """items: sequence of (model, X, score[, bins[, amap[, achan]]])."""
    arr = (Job * len(items))()
    for i, it in enumerate(items):
        model, X, score = it[0], it[1], it[2]
        bins = it[3] if len(it) > 3 else None
        amap = it[4] if len(it) > 4 else None
        achan = it[5] if len(it) > 5 else None
        import torch
        _dev_tensor(X, torch.float32, "X", 3)
        _dev_tensor(score, torch.float32, "score", 2)
        C, H, W = X.shape
        if C != model.params.C or tuple(score.shape) != (H, W):
            raise ValueError("job shapes do not match")
        if bins is not None:
            _dev_tensor(bins, torch.uint8, "bins", 3)
        if amap is not None:
            _dev_tensor(amap, torch.float32, "amap", 2)
        if achan is not None:
            _dev_tensor(achan, torch.float32, "achan", 3)
            if tuple(achan.shape) != (C, H, W):
                raise ValueError("achan shape does not match")
        arr[i] = Job(model.handle.value if hasattr(model.handle, "value") else model.handle,
                     X.data_ptr(), H, W, score.data_ptr(), bins.data_ptr() if bins is not None else None,
                     amap.data_ptr() if amap is not None else None,
                     achan.data_ptr() if achan is not None else None)
    return arr


def qfca_score_map_noalloc(ctx: Context, model: Model, bins, out: ScoreMaps):
    """qfca_score_map without device allocation: out (a ScoreMaps whose
    score and any of amap, w1, achan are preallocated device tensors)
    receives the maps."""
    import torch
    bins = _dev_tensor(bins, torch.uint8, "bins", 3)
    C, H, W = bins.shape
    if C != model.planes:
        raise ValueError("bins.shape[0] != the model's histogrammed planes")
    _dev_tensor(out.score, torch.float32, "score", 2)
    for name, nd in (("amap", 2), ("w1", 2), ("achan", 3)):
        if getattr(out, name) is not None:
            _dev_tensor(getattr(out, name), torch.float32, name, nd)
    _check(lib().qfca_score_map_noalloc(ctx.handle, model.handle, _ptr(bins), H, W, _ptr(out.score),
                                        _ptr(out.amap), _ptr(out.w1), _ptr(out.achan)))
    return out


def qfca_inspect_windows(ctx: Context, model: Model, bins):
    """Integer stages of the score path for every window: (cp, I), each a
    [C, H, W, B] int32 device tensor (see qfca.h)."""
    import torch
    _dev_tensor(bins, torch.uint8, "bins", 3)
    C, H, W = bins.shape
    if C != model.params.C:
        raise ValueError("bins do not match the model's channel count")
    B = model.params.B
    cp = torch.empty((C, H, W, B), dtype=torch.int32, device=bins.device)
    I = torch.empty((C, H, W, B), dtype=torch.int32, device=bins.device)
    _check(lib().qfca_inspect_windows(ctx.handle, model.handle, _ptr(bins), H, W, _ptr(cp), _ptr(I)))
    return cp, I


def qfca_score_batch(ctx: Context, items):
    """Quantise and score a batch.  items: sequence of (model, X [C,H,W],
    score [H,W] out[, bins [C,H,W] out[, amap [H,W] out[, achan [C,H,W] out]]])."""
    arr = _jobs(items)
    _check(lib().qfca_score_batch(ctx.handle, arr, len(items)))


def qfca_batch_error(ctx: Context) -> int:
    v = ctypes.c_int32()
    _check(lib().qfca_batch_error(ctx.handle, ctypes.byref(v)))
    return v.value


def qfca_autotune(ctx: Context, items):
    """Returns (Ws, Hb, ms) of the fastest score tile for this batch and keeps it."""
    arr = _jobs(items)
    ws, hb, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().qfca_autotune(ctx.handle, arr, len(items), ctypes.byref(ws), ctypes.byref(hb), ctypes.byref(ms)))
    return ws.value, hb.value, ms.value


def qfca_clock() -> float:
    """Seconds of the host monotonic clock that completion times use."""
    return lib().qfca_clock()


class Server:
    """Continuous-batching server (qfca_server_*): requests are submitted one
    image at a time against resident models and complete asynchronously."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_inflight: int = 2,
                 max_batch: int = 64, Ws: int = 0, Hb: int = 0):
        cfg = ServerConfig(int(hbm_budget), int(max_inflight), int(max_batch), int(Ws), int(Hb))
        h = ctypes.c_void_p()
        _check(lib().qfca_server_create(int(device), ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._buf = (Completion * 1024)()
        self._live = {}  # ticket -> (X, score): kept alive until the ticket completes

    def submit(self, model: "Model", X, score) -> int:
        """X: [C, H, W] float32 and score: [H, W] float32 on the device; both
        must stay alive and untouched until the returned ticket completes."""
        import torch
        _dev_tensor(X, torch.float32, "X", 3)
        _dev_tensor(score, torch.float32, "score", 2)
        C, H, W = X.shape
        if C != model.params.C or tuple(score.shape) != (H, W):
            raise ValueError("request shapes do not match")
        t = ctypes.c_uint64()
        _check(lib().qfca_server_submit(self.handle, model.handle, _ptr(X), H, W, _ptr(score), ctypes.byref(t)))
        self._live[t.value] = (model, X, score)
        return t.value

    def poll(self):
        """Completions since the last poll, as dicts."""
        out = []
        n = ctypes.c_int32()
        while True:
            _check(lib().qfca_server_poll(self.handle, self._buf, len(self._buf), ctypes.byref(n)))
            for i in range(n.value):
                c = self._buf[i]
                out.append({f: getattr(c, f) for f, _ in Completion._fields_})
                self._live.pop(c.ticket, None)
            if n.value < len(self._buf):
                return out

    def drain(self):
        _check(lib().qfca_server_drain(self.handle))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().qfca_server_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().qfca_server_destroy(self.handle)  # drains first
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def host_sym_eig(A: np.ndarray):
    """The library's host eigensolver (no GPU needed): (evals desc, vecs)."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    ev = np.zeros(n)
    V = np.zeros((n, n))
    rc = lib().qfca_host_sym_eig(A.ctypes.data_as(ctypes.c_void_p), n, ev.ctypes.data_as(ctypes.c_void_p),
                                 V.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise QfcaError(4, "eigensolver failed")
    return ev, V


def host_sym_eig_top(A: np.ndarray, k: int):
    """The fit's host eigensolver (no GPU needed): (all evals desc, the k
    leading eigenvectors as columns)."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    ev = np.zeros(n)
    V = np.zeros((n, k))
    rc = lib().qfca_host_sym_eig_top(A.ctypes.data_as(ctypes.c_void_p), n, k, ev.ctypes.data_as(ctypes.c_void_p),
                                     V.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise QfcaError(4, "eigensolver failed")
    return ev, V


# short aliases
fit_pca = qfca_fit_pca
model_create = qfca_model_create
fit_reference = qfca_fit_reference
quantize = qfca_quantize
score_map = qfca_score_map
score_batch = qfca_score_batch
