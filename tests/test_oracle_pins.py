"""Pins for the FP64 oracle, against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-worked
Algorithm 1 traces, a brute-force "FCA on quantised values" (the paper's
correctness argument in Sec. S4), library routines (numpy.linalg.eigh,
numpy.quantile, numpy.searchsorted, scipy.ndimage.gaussian_filter1d),
closed forms for special cases (B = 1, T = 1, periodic textures) and
invariances (permutation inside a window, transposes, channel order, scale).
"""
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Algorithm 1

def test_alg1_hand_worked_cases():
    """The oracle's coupling form against Alg. 1 traces worked by hand; every
    loop iteration of a trace that moves mass is one transport cell."""
    cases = json.load(open(os.path.join(GOLD, "alg1_hand.json")))["cases"]
    for c in cases:
        E, cells = oracle.bin_mismatch(c["P"], c["R"])
        np.testing.assert_allclose(E, c["E"], rtol=0, atol=1e-15)
        assert cells <= c["steps"] <= 2 * len(c["P"]) - 1


def fca_on_quantised(px, ry):
    """Brute-force FCA (Sec. 3.1 / Sec. S4) on bin-index values: px are the patch
    values, ry the reference values.  Both are replicated to equal mass, sorted,
    matched rank by rank, and the per-element errors |x - y| averaged per bin
    (ties averaged).  Returns E[bin]."""
    n, m = len(px), len(ry)
    xs = np.sort(np.repeat(np.asarray(px), m))
    ys = np.sort(np.repeat(np.asarray(ry), n))
    err = np.abs(xs - ys).astype(np.float64)
    B = int(max(px.max(), ry.max())) + 1
    E = np.zeros(B)
    for b in range(B):
        sel = xs == b
        if sel.any():
            E[b] = err[sel].mean()
    return E


@pytest.mark.parametrize("seed", range(40))
def test_alg1_equals_fca_on_quantised_values(seed):
    g = rng(seed)
    B = int(g.integers(1, 12))
    n = int(g.integers(1, 30))
    m = int(g.integers(1, 30))
    px = g.integers(0, B, n)
    ry = g.integers(0, B, m)
    # histograms scaled to equal mass, as for clipped border windows
    P = np.bincount(px, minlength=B) * m
    R = np.bincount(ry, minlength=B) * n
    E, cells = oracle.bin_mismatch(P, R)
    assert cells <= 2 * B - 1
    ref = fca_on_quantised(px, ry)
    ref = np.pad(ref, (0, B - ref.size))
    np.testing.assert_allclose(E, ref, rtol=1e-13, atol=1e-13)


def closed_form_numerators(cP, cR_scaled):
    """Per-bin transport numerators I_i = sum_j |i-j| pi_ij written as integrals
    of |i - J(u)| over the patch bin's quantile interval, with
    Phi(t) = sum_k (t - c_k)^+ (the identity the GPU kernel evaluates)."""
    B = len(cP)
    c = np.asarray(cR_scaled, np.int64)

    def Phi(t):
        return int(np.maximum(t - c[: B - 1], 0).sum())

    I = np.zeros(B, np.int64)
    for i in range(B):
        a = int(cP[i - 1]) if i else 0
        b = int(cP[i])
        cm = int(c[i - 1]) if i else 0
        s = min(max(cm, a), b)
        I[i] = Phi(a) + Phi(b) - 2 * Phi(s) + i * (2 * s - a - b)
    return I


@pytest.mark.parametrize("seed", range(40))
def test_alg1_closed_form_and_cdf_l1(seed):
    g = rng(1000 + seed)
    B = int(g.integers(1, 20))
    n = int(g.integers(1, 50))
    m = int(g.integers(1, 50))
    P = np.bincount(g.integers(0, B, n), minlength=B) * m
    R = np.bincount(g.integers(0, B, m), minlength=B) * n
    E, _ = oracle.bin_mismatch(P, R)
    I = closed_form_numerators(np.cumsum(P), np.cumsum(R))
    np.testing.assert_allclose(E * P, I, rtol=0, atol=1e-9)
    # sum_i P_i E_i is the L1 distance between the cumulative histograms
    assert abs((E * P).sum() - np.abs(np.cumsum(P) - np.cumsum(R)).sum()) < 1e-9


def test_alg1_identical_histograms_zero():
    P = np.array([3, 0, 5, 1, 7])
    E, cells = oracle.bin_mismatch(P, P)
    assert np.all(E == 0) and cells <= 9


# ---------------------------------------------------------------------------
# Window 1-Wasserstein by-product

def test_window_w1_equals_sorted_transport():
    g = rng(7)
    H, W, T, B = 11, 9, 5, 7
    bins = g.integers(0, B, (H, W)).astype(np.uint8)
    refvals = np.sort(g.integers(0, B, T * T))
    cR = np.cumsum(np.bincount(refvals, minlength=B)).astype(np.int32)
    A, W1, _ = oracle.channel_map(bins, T, B, cR, want_w1=True)
    r = T // 2
    for (py, px) in [(0, 0), (5, 4), (10, 8), (2, 7)]:
        vals = bins[max(0, py - r): py + r + 1, max(0, px - r): px + r + 1].ravel()
        n, m = vals.size, T * T
        xs = np.sort(np.repeat(vals, m)).astype(float)
        ys = np.sort(np.repeat(refvals, n)).astype(float)
        w1 = np.abs(xs - ys).mean()   # 1-D Wasserstein between empirical laws
        assert abs(W1[py, px] - w1) < 1e-12


# ---------------------------------------------------------------------------
# PCA residual (Sec. 3.3)

def test_pca_against_eigh_and_residual_properties():
    g = rng(11)
    C, N, k = 12, 500, 4
    X = (g.standard_normal((C, C)) @ g.standard_normal((C, N)) + g.standard_normal((C, 1))).astype(np.float32)
    mu, V, ev = oracle.pca(X, k)
    Xd = X.astype(np.float64)
    np.testing.assert_allclose(mu, Xd.mean(1), rtol=0, atol=1e-12)
    cov = np.cov(Xd, bias=True)
    w, U = np.linalg.eigh(cov)
    np.testing.assert_allclose(ev, w[::-1], rtol=1e-10, atol=1e-10)
    Uk = U[:, ::-1][:, :k]
    np.testing.assert_allclose(V @ V.T, Uk @ Uk.T, atol=1e-9)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-12)
    R = oracle.residual(X, mu, V)
    np.testing.assert_allclose(V.T @ R, 0, atol=1e-10)
    np.testing.assert_allclose(R.sum(1), 0, atol=1e-9)
    # residual = projection onto the orthogonal complement of the top-k axes
    ref = (np.eye(C) - Uk @ Uk.T) @ (Xd - Xd.mean(1, keepdims=True))
    np.testing.assert_allclose(R, ref, atol=1e-9)
    # k = 0: the residual is the centred feature
    R0 = oracle.residual(X, mu, np.zeros((C, 0)))
    np.testing.assert_allclose(R0, Xd - Xd.mean(1, keepdims=True), atol=1e-12)
    # plain QFCA (no preprocessing) keeps the features
    np.testing.assert_array_equal(oracle.residual(X, mu, V, preproc=0), Xd)


# ---------------------------------------------------------------------------
# Quantisation (Sec. 3.1)

def test_quantile_matches_numpy_linear():
    g = rng(3)
    for n in (1, 2, 7, 100, 1001):
        v = g.standard_normal(n)
        for q in (0.0, 0.01, 0.5, 0.99, 1.0):
            assert abs(oracle.quantile(v, q) - np.quantile(v, q, method="linear")) < 1e-14


def test_edges_and_bins_match_searchsorted():
    g = rng(4)
    C, N, B = 5, 2000, 9
    R = g.standard_normal((C, N)) * g.uniform(0.1, 3, (C, 1))
    lo, hi, de, e = oracle.edges(R, B, 0.01, 0.99)
    for c in range(C):
        l = np.quantile(R[c], 0.01)
        h = np.quantile(R[c], 0.99)
        assert abs(lo[c] - l) < 1e-14 and abs(hi[c] - h) < 1e-14
        np.testing.assert_array_equal(e[c], (l + np.arange(1, B) * (h - l) / B).astype(np.float32))
    # put some values exactly on edges: ties go to the upper bin
    R[0, :8] = e[0, :8].astype(np.float64)
    bins = oracle.quantize(R, B, e)
    for c in range(C):
        ref = np.searchsorted(e[c].astype(np.float64), R[c], side="right")
        np.testing.assert_array_equal(bins[c], ref)
    assert np.all(bins[0, :8] == np.arange(1, 9))
    assert bins.max() == B - 1 and bins.min() == 0


def test_degenerate_channel_goes_to_bin_zero():
    R = np.ones((2, 50))
    R[1] = np.linspace(0, 1, 50)
    lo, hi, de, e = oracle.edges(R, 4)
    b = oracle.quantize(R, 4, e)
    assert de[0] == 0 and np.all(b[0] == 0)
    assert de[1] > 0 and b[1].max() == 3


# ---------------------------------------------------------------------------
# Reference (Sec. 3.2): per-rank lower median, then quantised

def brute_reference(R, T, B, e):
    C, H, W = R.shape
    out = np.zeros((C, B), np.int32)
    for c in range(C):
        wins = np.array([np.sort(R[c, y:y + T, x:x + T].ravel())
                         for y in range(H - T + 1) for x in range(W - T + 1)])
        nw = wins.shape[0]
        ref = np.sort(wins, axis=0)[(nw + 1) // 2 - 1]     # lower median per rank
        b = np.searchsorted(e[c].astype(np.float64), ref, side="right")
        out[c] = np.cumsum(np.bincount(b, minlength=B))
    return out


@pytest.mark.parametrize("shape", [(3, 9, 9, 3, 5), (2, 10, 13, 5, 6), (2, 8, 8, 1, 4), (1, 12, 7, 7, 3)])
def test_reference_literal_vs_bruteforce_and_cdf_form(shape):
    C, H, W, T, B = shape
    g = rng(sum(shape))
    R = g.standard_normal((C, H, W))
    _, _, _, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    lit = oracle.reference_literal(R, T, B, e)
    np.testing.assert_array_equal(lit, brute_reference(R, T, B, e))
    np.testing.assert_array_equal(oracle.reference_cdf(bins, T, B), lit)
    assert np.all(lit[:, -1] == T * T)


# ---------------------------------------------------------------------------
# Full pipeline: brute force of the whole score on tiny maps

def brute_score(bins, T, B, cR, delta, sigma):
    from scipy.ndimage import gaussian_filter1d
    C, H, W = bins.shape
    r = T // 2
    A = np.zeros((H, W))
    for c in range(C):
        refvals = np.repeat(np.arange(B), np.diff(np.concatenate([[0], cR[c]])))
        e = np.zeros((H, W, B))
        for py in range(H):
            for px in range(W):
                vals = bins[c, max(0, py - r): py + r + 1, max(0, px - r): px + r + 1].ravel()
                E = fca_on_quantised(vals, refvals)
                e[py, px, : E.size] = E
        for y in range(H):
            for x in range(W):
                win = e[max(0, y - r): y + r + 1, max(0, x - r): x + r + 1, bins[c, y, x]]
                A[y, x] += delta[c] * win.mean()
    A /= C
    if sigma > 0:
        def g(a):
            a = gaussian_filter1d(a, sigma, axis=0, mode="constant", truncate=3.0)
            return gaussian_filter1d(a, sigma, axis=1, mode="constant", truncate=3.0)
        S = g(A) / g(np.ones_like(A))
    else:
        S = A.copy()
    return A, S


@pytest.mark.parametrize("case", [(2, 9, 11, 3, 4), (3, 8, 8, 5, 6), (1, 10, 7, 7, 3), (2, 6, 9, 1, 5)])
def test_score_against_bruteforce_fca(case):
    C, H, W, T, B = case
    g = rng(100 + sum(case))
    R = g.standard_normal((C, H, W))
    _, _, delta, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    cR = oracle.reference_cdf(bins, T, B) if (H >= T and W >= T) else None
    out = oracle.score(bins, T, B, cR, delta, 1.0, want_chan=True)
    A, S = brute_score(bins, T, B, cR, delta, 1.0)
    np.testing.assert_allclose(out.A, A, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(out.score, S, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(out.Achan.mean(0), out.A, rtol=1e-13, atol=1e-15)
    assert out.max_steps <= 2 * B - 1
    ys, xs = np.array([0, H - 1, H // 2]), np.array([W - 1, 0, W // 2])
    np.testing.assert_allclose(oracle.amap_pixels(bins, T, B, cR, delta, ys, xs), out.A[ys, xs],
                               rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# Special cases and invariances

def test_single_bin_gives_zero_score():
    g = rng(5)
    bins = np.zeros((2, 9, 9), np.uint8)
    cR = np.full((2, 1), 25, np.int32)
    out = oracle.score(bins, 5, 1, cR, np.ones(2), 1.0)
    assert np.all(out.score == 0)


def test_T1_closed_form():
    """T = 1: every window is one pixel; the reference is the bin of the lower
    median pixel value m_c, so A_c(x) = delta_c |b_c(x) - m_c|."""
    g = rng(6)
    C, H, W, B = 3, 7, 8, 6
    R = g.standard_normal((C, H, W))
    _, _, delta, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    cR = oracle.reference_literal(R, 1, B, e)
    out = oracle.score(bins, 1, B, cR, delta, 0.0, want_chan=True)
    for c in range(C):
        v = np.sort(R[c].ravel())[(H * W + 1) // 2 - 1]
        mc = np.searchsorted(e[c].astype(np.float64), v, side="right")
        np.testing.assert_allclose(out.Achan[c], delta[c] * np.abs(bins[c].astype(int) - mc), atol=1e-14)


def test_periodic_texture_scores_zero_inside():
    """Plain QFCA on a T-periodic texture: every full window holds the same
    multiset of values, the reference equals every full-window histogram, and
    the map is 0 wherever all covering windows are full."""
    g = rng(8)
    C, T, B = 3, 5, 8
    H = W = 6 * T
    tile = g.standard_normal((C, T, T)).astype(np.float32)
    X = np.tile(tile, (1, H // T, W // T))
    m, R, bins = oracle.fit(X, 0, B, T, preproc=0)
    out = oracle.score(bins, T, B, m.cR, m.delta, 1.0)
    r = T // 2
    inner = out.A[2 * r: H - 2 * r, 2 * r: W - 2 * r]
    assert np.abs(inner).max() < 1e-14
    assert np.abs(out.A).max() > 0  # the clipped border windows do differ
    inner_s = out.score[2 * r + 3: H - 2 * r - 3, 2 * r + 3: W - 2 * r - 3]
    assert np.abs(inner_s).max() < 1e-14


def test_permutation_inside_window_invariance():
    g = rng(9)
    H, W, T, B = 13, 13, 5, 6
    bins = g.integers(0, B, (H, W)).astype(np.uint8)
    cR = np.cumsum(np.bincount(g.integers(0, B, T * T), minlength=B)).astype(np.int32)
    E0, _ = oracle.window_errors(bins, T, B, cR, 6, 6)
    b2 = bins.copy()
    sub = b2[4:9, 4:9].ravel()
    b2[4:9, 4:9] = g.permutation(sub).reshape(5, 5)
    E1, _ = oracle.window_errors(b2, T, B, cR, 6, 6)
    np.testing.assert_array_equal(E0, E1)


def test_transpose_flip_and_channel_order():
    g = rng(10)
    C, H, W, T, B = 3, 10, 12, 5, 6
    R = g.standard_normal((C, H, W))
    _, _, delta, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    cR = oracle.reference_cdf(bins, T, B)
    base = oracle.score(bins, T, B, cR, delta, 1.0)
    tr = oracle.score(np.ascontiguousarray(bins.transpose(0, 2, 1)), T, B, cR, delta, 1.0)
    np.testing.assert_allclose(tr.score, base.score.T, rtol=1e-12, atol=1e-14)
    fl = oracle.score(np.ascontiguousarray(bins[:, ::-1, :]), T, B, cR, delta, 1.0)
    np.testing.assert_allclose(fl.score, base.score[::-1], rtol=1e-12, atol=1e-14)
    p = g.permutation(C)
    pc = oracle.score(np.ascontiguousarray(bins[p]), T, B, cR[p], delta[p], 1.0)
    np.testing.assert_allclose(pc.score, base.score, rtol=1e-12, atol=1e-14)


def test_channel_scale_invariance_plain_mode():
    """x_c -> 2 x_c (exact in binary floating point) leaves the bins unchanged
    and doubles the channel's contribution."""
    g = rng(12)
    C, H, W, T, B = 2, 12, 12, 5, 8
    X = g.standard_normal((C, H, W)).astype(np.float32)
    m1, _, b1 = oracle.fit(X, 0, B, T, preproc=0)
    X2 = X.copy()
    X2[1] *= 2
    m2, _, b2 = oracle.fit(X2, 0, B, T, preproc=0)
    np.testing.assert_array_equal(b1, b2)
    np.testing.assert_array_equal(m1.cR, m2.cR)
    o1 = oracle.score(b1, T, B, m1.cR, m1.delta, 1.0, want_chan=True)
    o2 = oracle.score(b2, T, B, m2.cR, m2.delta, 1.0, want_chan=True)
    np.testing.assert_allclose(o2.Achan[0], o1.Achan[0], rtol=1e-14)
    np.testing.assert_allclose(o2.Achan[1], 2 * o1.Achan[1], rtol=1e-14)


def test_blur_library_pin_and_special_cases():
    from scipy.ndimage import gaussian_filter1d
    g = rng(13)
    A = g.standard_normal((9, 14))
    for sigma in (0.5, 1.0, 1.7):
        out = oracle.blur(A, sigma)
        R = int(np.ceil(3 * sigma))
        tr = R / sigma

        def f(a):
            a = gaussian_filter1d(a, sigma, axis=0, mode="constant", truncate=tr)
            return gaussian_filter1d(a, sigma, axis=1, mode="constant", truncate=tr)
        np.testing.assert_allclose(out, f(A) / f(np.ones_like(A)), rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(oracle.blur(A, 0.0), A)
    np.testing.assert_allclose(oracle.blur(np.full((7, 5), 3.25), 1.0), 3.25, rtol=1e-14)


def test_synthetic_anomaly_is_localised():
    """Smoke check of the whole zero-shot oracle on the 64x64 workload: the
    inserted square scores higher than the background (no paper number)."""
    import qfca_synth
    ts, p = qfca_synth.workload_small()
    t = ts[0]
    m, R, bins = oracle.fit(t.X, p["k"], p["B"], p["T"], p["q_lo"], p["q_hi"])
    out = oracle.score(bins, p["T"], p["B"], m.cR, m.delta, p["sigma_s"])
    from sklearn.metrics import roc_auc_score
    assert roc_auc_score(t.mask.ravel(), out.score.ravel()) > 0.9
