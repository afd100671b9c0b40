"""FP64 CPU oracle for the QFCA score-map path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``qfca_oracle.c`` (plain C, FP64, OpenMP over
channels) through ctypes and shares no code with the HIP library.

Every function follows a passage of "Quantized FCA" (Ardelean et al.):
PCA residual (Sec. 3.3), quantisation (Sec. 3.1), the per-bin mismatch of
Alg. 1 as the monotone coupling of two cumulative histograms (Alg. 1 and the
supplementary proof), the four reference choices (Sec. 3.2, Sec. 4.5.3,
Tab. 3), the association with box or Gaussian sigma_p weights (Eq. 2,
Sec. 3.1, Sec. 4.5.4), the sigma_s blur (Sec. 4.5.4), the principal-
coordinate histograms scored by the window 1-Wasserstein distance (Sec. 3.3,
Sec. 3.1) and FCA's sort-based comparison (Sec. 3.1).  Pins for each live in
tests/test_oracle_pins.py and tests/test_oracle_pins_variants.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qfca_oracle.c")
_LIB = os.path.join(_HERE, "libqfca_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int, ctypes.c_long, ctypes.c_double
        L.orc_pca.argtypes = [P, i32, i64, i32, P, P, P]
        L.orc_pca.restype = i32
        L.orc_residual.argtypes = [P, i32, i64, P, P, i32, i32, P]
        L.orc_quantile.argtypes = [P, i64, f64]
        L.orc_quantile.restype = f64
        L.orc_edges.argtypes = [P, i32, i64, i32, f64, f64, P, P, P, P]
        L.orc_quantize.argtypes = [P, i32, i64, i32, P, P]
        L.orc_bin_mismatch.argtypes = [P, P, i32, P, P]
        L.orc_bin_mismatch.restype = i32
        L.orc_reference_values.argtypes = [P, i32, i32, i32, i32, i32, P]
        L.orc_reference_literal.argtypes = [P, i32, i32, i32, i32, i32, P, i32, P]
        L.orc_reference_cdf.argtypes = [P, i32, i32, i32, i32, i32, P]
        L.orc_reference_hist.argtypes = [P, i32, i32, i32, i32, i32, i32, P]
        L.orc_channel_map.argtypes = [P, i32, i32, i32, i32, P, f64, P, P]
        L.orc_channel_map.restype = i32
        L.orc_window_errors.argtypes = [P, i32, i32, i32, i32, P, i32, i32, P, P, P]
        L.orc_window_errors.restype = i32
        L.orc_blur.argtypes = [P, i32, i32, f64, P]
        L.orc_score.argtypes = [P, i32, i32, i32, i32, i32, P, P, f64, f64, P, P, P, P]
        L.orc_score.restype = i32
        L.orc_amap_pixels.argtypes = [P, i32, i32, i32, i32, i32, P, P, f64, i32, P, P, P, P]
        L.orc_project.argtypes = [P, i32, i64, P, P, i32, P]
        L.orc_w1_score.argtypes = [P, i32, i32, i32, i32, i32, P, P, f64, P, P]
        L.orc_fca_window.argtypes = [P, i32, i32, i32, P, i32, i32, P]
        L.orc_fca_window.restype = i32
        L.orc_fca_score.argtypes = [P, i32, i32, i32, i32, P, f64, P, P, P]
        L.orc_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return int(_load().orc_num_threads())


# --------------------------------------------------------------------------
# PCA residual preprocessing (Sec. 3.3)

def pca(X, k):
    """X: [C, H, W] or [C, N] float32.  Returns (mu[C], V[C,k], evals[C] desc)."""
    X = _c(X, np.float32)
    C = X.shape[0]
    N = X.size // C
    mu = np.zeros(C)
    V = np.zeros((C, max(k, 0)))
    ev = np.zeros(C)
    rc = _load().orc_pca(_p(X), C, N, k, _p(mu), _p(V), _p(ev))
    if rc < 0:
        raise ValueError("bad PCA arguments")
    return mu, V, ev


def residual(X, mu, V, preproc=1):
    """r = (x - mu) - V V^T (x - mu) per pixel (preproc=1), or x (preproc=0)."""
    X = _c(X, np.float32)
    C = X.shape[0]
    N = X.size // C
    k = 0 if V is None else V.shape[1]
    mu = _c(mu if mu is not None else np.zeros(C), np.float64)
    Vc = _c(V if V is not None and k > 0 else np.zeros((C, 1)), np.float64)
    R = np.zeros(X.shape, np.float64)
    _load().orc_residual(_p(X), C, N, _p(mu), _p(Vc), k, int(preproc), _p(R))
    return R


# --------------------------------------------------------------------------
# Quantisation (Sec. 3.1)

def quantile(v, q):
    v = _c(v, np.float64).ravel()
    return float(_load().orc_quantile(_p(v), v.size, float(q)))


def edges(R, B, q_lo=0.01, q_hi=0.99):
    """Returns (lo[C], hi[C], delta[C], edges[C, B-1] float32)."""
    R = _c(R, np.float64)
    C = R.shape[0]
    N = R.size // C
    lo, hi, de = np.zeros(C), np.zeros(C), np.zeros(C)
    e = np.zeros((C, max(B - 1, 1)), np.float32)
    _load().orc_edges(_p(R), C, N, B, float(q_lo), float(q_hi), _p(lo), _p(hi), _p(de), _p(e))
    return lo, hi, de, e[:, : B - 1]


def quantize(R, B, e):
    R = _c(R, np.float64)
    C = R.shape[0]
    N = R.size // C
    e = _c(e if B > 1 else np.zeros((C, 1)), np.float32)
    out = np.zeros(R.shape, np.uint8)
    _load().orc_quantize(_p(R), C, N, B, _p(e), _p(out))
    return out


# --------------------------------------------------------------------------
# Per-bin mismatch (Alg. 1)

def bin_mismatch(P, R, numerators=False):
    """Per-bin mismatch of a patch histogram P against a reference R (equal
    total mass, any nonnegative weights), Q_i = i: the monotone coupling of
    the two cumulative histograms (Alg. 1 and the supplementary proof).
    Returns (E[B] in bin units, cells) or, with numerators=True,
    (E, I, cells) with I_i = E_i P_i."""
    P = _c(P, np.float64)
    R = _c(R, np.float64)
    E = np.zeros(P.size)
    I = np.zeros(P.size)
    cells = _load().orc_bin_mismatch(_p(P), _p(R), P.size, _p(E), _p(I))
    return (E, I, int(cells)) if numerators else (E, int(cells))


# --------------------------------------------------------------------------
# Reference (Sec. 3.2, Sec. 4.5.3, Tab. 3)

REF_KINDS = ("median_quan", "mean_quan", "quan_median", "quan_mean")


def reference_values(R, T, kind="median"):
    """Full-precision reference vectors [C, T*T]: the rank-wise lower median
    (kind "median") or mean (kind "mean") of the sorted full windows."""
    R = _c(R, np.float64)
    C, H, W = R.shape
    Y = np.zeros((C, T * T))
    _load().orc_reference_values(_p(R), C, H, W, T, 0 if kind == "median" else 1, _p(Y))
    return Y


def reference_literal(R, T, B, e, kind="median"):
    """median -> quan (kind "median") or mean -> quan (kind "mean"):
    cumulative integer reference [C, B] of mass T*T."""
    R = _c(R, np.float64)
    C, H, W = R.shape
    e = _c(e if B > 1 else np.zeros((C, 1)), np.float32)
    cR = np.zeros((C, B), np.int32)
    _load().orc_reference_literal(_p(R), C, H, W, T, B, _p(e), 0 if kind == "median" else 1, _p(cR))
    return cR


def reference_cdf(bins, T, B):
    bins = _c(bins, np.uint8)
    C, H, W = bins.shape
    cR = np.zeros((C, B), np.int32)
    _load().orc_reference_cdf(_p(bins), C, H, W, T, B, _p(cR))
    return cR


def reference_hist(bins, T, B, kind="median"):
    """quan -> median (kind "median": bin-wise lower median of the full-window
    histograms) or quan -> mean (kind "mean": their mean).  Cumulative
    reference weights [C, B] (float64); the median's mass is the sum of the
    medians."""
    bins = _c(bins, np.uint8)
    C, H, W = bins.shape
    cR = np.zeros((C, B))
    _load().orc_reference_hist(_p(bins), C, H, W, T, B, 0 if kind == "median" else 1, _p(cR))
    return cR


# --------------------------------------------------------------------------
# Comparison, association, aggregation, blur

def channel_map(bins_c, T, B, cR_c, want_w1=False, sigma_p=np.inf):
    bins_c = _c(bins_c, np.uint8)
    H, W = bins_c.shape
    cR_c = _c(cR_c, np.float64)
    A = np.zeros((H, W))
    W1 = np.zeros((H, W)) if want_w1 else None
    cells = _load().orc_channel_map(_p(bins_c), H, W, T, B, _p(cR_c), float(sigma_p), _p(A), _p(W1))
    return A, W1, int(cells)


def window_errors(bins_c, T, B, cR_c, py, px, numerators=False):
    """Per-bin mismatch E[B] of one window (and, with numerators=True, the
    numerators I[B] and the scaled patch weights P~[B]) plus the cell count."""
    bins_c = _c(bins_c, np.uint8)
    H, W = bins_c.shape
    cR_c = _c(cR_c, np.float64)
    E, I, Pt = np.zeros(B), np.zeros(B), np.zeros(B)
    cells = _load().orc_window_errors(_p(bins_c), H, W, T, B, _p(cR_c), int(py), int(px), _p(E), _p(I),
                                      _p(Pt))
    return (E, I, Pt, int(cells)) if numerators else (E, int(cells))


def blur(A, sigma):
    A = _c(A, np.float64)
    H, W = A.shape
    out = np.zeros_like(A)
    _load().orc_blur(_p(A), H, W, float(sigma), _p(out))
    return out


@dataclass
class ScoreOut:
    A: np.ndarray        # [H, W] channel-mean association map (feature units)
    score: np.ndarray    # [H, W] blurred score
    W1: np.ndarray | None
    Achan: np.ndarray | None
    max_steps: int       # largest number of transport cells of a window (<= 2B - 1)


def score(bins, T, B, cR, delta, sigma_s=1.0, want_w1=False, want_chan=False, sigma_p=np.inf):
    bins = _c(bins, np.uint8)
    C, H, W = bins.shape
    cR = _c(cR, np.float64)
    delta = _c(delta, np.float64)
    A = np.zeros((H, W))
    S = np.zeros((H, W))
    W1 = np.zeros((H, W)) if want_w1 else None
    Ach = np.zeros((C, H, W)) if want_chan else None
    cells = _load().orc_score(_p(bins), C, H, W, T, B, _p(cR), _p(delta), float(sigma_p), float(sigma_s),
                              _p(A), _p(S), _p(W1), _p(Ach))
    return ScoreOut(A, S, W1, Ach, int(cells))


def amap_pixels(bins, T, B, cR, delta, ys, xs, want_chan=False, sigma_p=np.inf):
    bins = _c(bins, np.uint8)
    C, H, W = bins.shape
    ys = _c(ys, np.int32)
    xs = _c(xs, np.int32)
    out = np.zeros(ys.size)
    ch = np.zeros((ys.size, C)) if want_chan else None
    _load().orc_amap_pixels(_p(bins), C, H, W, T, B, _p(_c(cR, np.float64)), _p(_c(delta, np.float64)),
                            float(sigma_p), ys.size, _p(ys), _p(xs), _p(out), _p(ch))
    return (out, ch) if want_chan else out


# --------------------------------------------------------------------------
# Principal-coordinate histograms scored by the window W1 (Sec. 3.3, Sec. 3.1)

def project(X, mu, V):
    """z = V^T (x - mu) per pixel: [k, H, W] (or [k, N]) float64."""
    X = _c(X, np.float32)
    C = X.shape[0]
    N = X.size // C
    k = V.shape[1]
    Z = np.zeros((k,) + X.shape[1:])
    _load().orc_project(_p(X), C, N, _p(_c(mu, np.float64)), _p(_c(V, np.float64)), k, _p(Z))
    return Z


def w1_score(bins, T, B, cR, delta, sigma_s=1.0):
    """Window W1 of every coordinate plane, box smoothed, averaged over the
    planes and blurred.  Returns (A, score)."""
    bins = _c(bins, np.uint8)
    K, H, W = bins.shape
    A = np.zeros((H, W))
    S = np.zeros((H, W))
    _load().orc_w1_score(_p(bins), K, H, W, T, B, _p(_c(cR, np.int32)), _p(_c(delta, np.float64)),
                         float(sigma_s), _p(A), _p(S))
    return A, S


# --------------------------------------------------------------------------
# FCA's sort-based comparison (Sec. 3.1)

def fca_window(Rc, T, Y, py, px):
    """Per-element errors of one window (raster order of its pixels)."""
    Rc = _c(Rc, np.float64)
    H, W = Rc.shape
    err = np.zeros(T * T)
    n = _load().orc_fca_window(_p(Rc), H, W, T, _p(_c(Y, np.float64)), int(py), int(px), _p(err))
    return err[:n]


def fca_score(R, T, Y, sigma_s=1.0, want_chan=False):
    """FCA map: R [C, H, W] real features, Y [C, T*T] sorted references.
    Returns (A, score, Achan or None)."""
    R = _c(R, np.float64)
    C, H, W = R.shape
    A = np.zeros((H, W))
    S = np.zeros((H, W))
    Ach = np.zeros((C, H, W)) if want_chan else None
    _load().orc_fca_score(_p(R), C, H, W, T, _p(_c(Y, np.float64)), float(sigma_s), _p(A), _p(S), _p(Ach))
    return A, S, Ach


# --------------------------------------------------------------------------
# Whole zero-shot fit + score, composed from the steps above.

@dataclass
class OracleModel:
    mu: np.ndarray       # [C]
    V: np.ndarray        # [C, k]
    evals: np.ndarray    # [C]
    lo: np.ndarray
    hi: np.ndarray
    delta: np.ndarray    # [C]
    edges: np.ndarray    # [C, B-1] float32
    cR: np.ndarray       # [C, B] int32 (float64 for the quan -> median / mean references)
    T: int
    B: int
    preproc: int


def fit(X, k, B, T, q_lo=0.01, q_hi=0.99, preproc=1, reference="cdf"):
    """Zero-shot fit on the image itself.  Returns (model, residual, bins).
    reference: "cdf" (median -> quan from the bins), "literal" (median -> quan
    by sorting), "mean_quan", "quan_median" or "quan_mean" (Tab. 3)."""
    X = _c(X, np.float32)
    C = X.shape[0]
    if preproc:
        mu, V, ev = pca(X, k)
    else:
        mu, V, ev = np.zeros(C), np.zeros((C, 0)), np.zeros(C)
    R = residual(X, mu, V, preproc)
    lo, hi, de, e = edges(R, B, q_lo, q_hi)
    bins = quantize(R, B, e)
    if reference == "literal":
        cR = reference_literal(R, T, B, e)
    elif reference == "mean_quan":
        cR = reference_literal(R, T, B, e, kind="mean")
    elif reference == "quan_median":
        cR = reference_hist(bins, T, B, kind="median")
    elif reference == "quan_mean":
        cR = reference_hist(bins, T, B, kind="mean")
    else:
        cR = reference_cdf(bins, T, B)
    return OracleModel(mu, V, ev, lo, hi, de, e, cR, T, B, preproc), R, bins


@dataclass
class CoordModel:
    mu: np.ndarray       # [C]
    V: np.ndarray        # [C, k]
    lo: np.ndarray       # [k]
    hi: np.ndarray
    delta: np.ndarray    # [k]
    edges: np.ndarray    # [k, B-1] float32
    cR: np.ndarray       # [k, B] int32
    T: int
    B: int


def fit_coords(X, k, B, T, q_lo=0.01, q_hi=0.99):
    """Zero-shot fit of the principal-coordinate variant: PCA, the k
    coordinates z, their [q_lo, q_hi] quantile edges, bins and the median ->
    quan reference of every coordinate.  Returns (model, Z, bins)."""
    X = _c(X, np.float32)
    mu, V, _ = pca(X, k)
    Z = project(X, mu, V)
    lo, hi, de, e = edges(Z, B, q_lo, q_hi)
    bins = quantize(Z, B, e)
    cR = reference_cdf(bins, T, B)
    return CoordModel(mu, V, lo, hi, de, e, cR, T, B), Z, bins
