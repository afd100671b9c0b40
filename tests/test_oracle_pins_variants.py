"""Pins for the oracle's variants beside the default path, each against
something other than the oracle itself:

* finite sigma_p association (Eq. 2, Sec. 3.1, Sec. 4.5.4): a numpy brute
  force of the weighted mean, the sigma_p -> infinity and sigma_p -> 0 limits;
* the Tab. 3 reference choices (Sec. 4.5.3): numpy brute forces, their
  agreement on periodic textures, a hand-worked case, and the score with a
  fractional reference against the integral (closed) form of the numerators;
* the principal-coordinate histograms scored by the window W1 (Sec. 3.3,
  Sec. 3.1): numpy projection, sort-based 1-D Wasserstein per window, direct
  box smoothing and scipy's Gaussian;
* FCA's sort-based comparison (Sec. 3.1, supplementary proof): numpy sorting,
  the tie-averaged errors on quantised values against the histogram form,
  the window error sum against the sorted 1-D W1, and convergence of the
  quantised map to FCA's as the bins get finer.
"""
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def fca_on_quantised(px, ry):
    """Sorted rank matching of bin-index values replicated to equal mass; the
    per-element errors averaged per patch bin."""
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


def windows(H, W, T, y, x):
    r = T // 2
    return slice(max(0, y - r), y + r + 1), slice(max(0, x - r), x + r + 1)


# ---------------------------------------------------------------------------
# Finite sigma_p

def brute_channel_sigma(bins, T, B, cR, sigma_p):
    H, W = bins.shape
    r = T // 2
    refvals = np.repeat(np.arange(B), np.diff(np.concatenate([[0], cR])))
    e = np.zeros((H, W, B))
    for py in range(H):
        for px in range(W):
            sy, sx = windows(H, W, T, py, px)
            E = fca_on_quantised(bins[sy, sx].ravel(), refvals)
            e[py, px, :E.size] = E
    A = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            s = wsum = 0.0
            for py in range(max(0, y - r), min(H, y + r + 1)):
                for px in range(max(0, x - r), min(W, x + r + 1)):
                    w = 1.0 if np.isinf(sigma_p) else np.exp(-((py - y) ** 2 + (px - x) ** 2) / (2 * sigma_p ** 2))
                    s += w * e[py, px, bins[y, x]]
                    wsum += w
            A[y, x] = s / wsum
    return A, e


@pytest.mark.parametrize("sigma_p", [0.7, 1.5, 4.0, np.inf])
def test_sigma_p_association_bruteforce(sigma_p):
    g = rng(21)
    H, W, T, B = 9, 11, 5, 6
    bins = g.integers(0, B, (H, W)).astype(np.uint8)
    cR = np.cumsum(np.bincount(g.integers(0, B, T * T), minlength=B))
    A, _, _ = oracle.channel_map(bins, T, B, cR, sigma_p=sigma_p)
    ref, _ = brute_channel_sigma(bins, T, B, cR, sigma_p)
    np.testing.assert_allclose(A, ref, rtol=1e-12, atol=1e-13)


def test_sigma_p_limits():
    g = rng(22)
    H, W, T, B = 10, 10, 7, 5
    bins = g.integers(0, B, (H, W)).astype(np.uint8)
    cR = np.cumsum(np.bincount(g.integers(0, B, T * T), minlength=B))
    box, _, _ = oracle.channel_map(bins, T, B, cR)
    wide, _, _ = oracle.channel_map(bins, T, B, cR, sigma_p=1e7)
    np.testing.assert_allclose(wide, box, rtol=1e-10, atol=1e-12)
    # sigma_p -> 0: only the window centred at the pixel counts
    narrow, _, _ = oracle.channel_map(bins, T, B, cR, sigma_p=1e-2)
    for (y, x) in [(0, 0), (4, 5), (9, 3)]:
        E, _ = oracle.window_errors(bins, T, B, cR, y, x)
        assert abs(narrow[y, x] - E[bins[y, x]]) < 1e-12


# ---------------------------------------------------------------------------
# Reference choices (Tab. 3)

def full_windows(plane, T):
    H, W = plane.shape
    return [plane[y:y + T, x:x + T].ravel() for y in range(H - T + 1) for x in range(W - T + 1)]


def brute_mean_quan(R, T, B, e):
    out = []
    for c in range(R.shape[0]):
        wins = np.sort(np.array(full_windows(R[c], T)), axis=1)
        ref = wins.mean(0)
        b = np.searchsorted(e[c].astype(np.float64), ref, side="right")
        out.append(np.cumsum(np.bincount(b, minlength=B)))
    return np.array(out)


def brute_quan_hist(bins, T, B, kind):
    out = []
    for c in range(bins.shape[0]):
        hs = np.array([np.bincount(w, minlength=B) for w in full_windows(bins[c], T)])
        if kind == "median":
            v = np.sort(hs, axis=0)[(hs.shape[0] + 1) // 2 - 1]
        else:
            v = hs.mean(0)
        out.append(np.cumsum(v))
    return np.array(out, np.float64)


@pytest.mark.parametrize("shape", [(2, 9, 9, 3, 5), (2, 10, 13, 5, 6), (1, 12, 11, 7, 4)])
def test_reference_variants_bruteforce(shape):
    C, H, W, T, B = shape
    g = rng(30 + sum(shape))
    R = g.standard_normal((C, H, W))
    _, _, _, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    np.testing.assert_array_equal(oracle.reference_literal(R, T, B, e, kind="mean"), brute_mean_quan(R, T, B, e))
    np.testing.assert_allclose(oracle.reference_hist(bins, T, B, "median"), brute_quan_hist(bins, T, B, "median"),
                               rtol=0, atol=0)
    np.testing.assert_allclose(oracle.reference_hist(bins, T, B, "mean"), brute_quan_hist(bins, T, B, "mean"),
                               rtol=1e-14, atol=1e-12)
    # the mean of the window histograms has mass T^2
    assert np.allclose(oracle.reference_hist(bins, T, B, "mean")[:, -1], T * T)


def test_reference_variants_agree_on_periodic_texture():
    """Every full window of a T-periodic texture holds the same multiset of
    values, so all four reference choices give that multiset's histogram."""
    g = rng(31)
    C, T, B = 2, 5, 6
    tile = g.standard_normal((C, T, T))
    R = np.tile(tile, (1, 4, 5))
    _, _, _, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    base = oracle.reference_literal(R, T, B, e)
    np.testing.assert_array_equal(oracle.reference_literal(R, T, B, e, kind="mean"), base)
    np.testing.assert_array_equal(oracle.reference_hist(bins, T, B, "median"), base)
    np.testing.assert_allclose(oracle.reference_hist(bins, T, B, "mean"), base, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(oracle.reference_cdf(bins, T, B), base)


def test_reference_variants_hand_worked():
    cases = json.load(open(os.path.join(GOLD, "reference_hand.json")))["cases"]
    for c in cases:
        R = np.array(c["R"], np.float64)[None]
        e = np.array(c["edges"], np.float32)[None]
        T, B = c["T"], len(c["edges"]) + 1
        bins = oracle.quantize(R, B, e)
        np.testing.assert_array_equal(bins[0], np.array(c["bins"]))
        np.testing.assert_array_equal(oracle.reference_literal(R, T, B, e)[0], c["median_quan"])
        np.testing.assert_array_equal(oracle.reference_literal(R, T, B, e, kind="mean")[0], c["mean_quan"])
        np.testing.assert_array_equal(oracle.reference_hist(bins, T, B, "median")[0], c["quan_median"])
        np.testing.assert_allclose(oracle.reference_hist(bins, T, B, "mean")[0], c["quan_mean"], rtol=0,
                                   atol=1e-12)


def closed_form_numerators(cP, cRs):
    """Integral form of the per-bin numerators (exact for integer inputs):
    I_i = Phi(a) + Phi(b) - 2 Phi(s) + i (2 s - a - b), Phi(t) = sum_k (t - c_k)^+."""
    B = len(cP)
    c = np.asarray(cRs)

    def Phi(t):
        return np.maximum(t - c[: B - 1], 0).sum()

    I = np.zeros(B)
    for i in range(B):
        a = cP[i - 1] if i else 0
        b = cP[i]
        cm = c[i - 1] if i else 0
        s = min(max(cm, a), b)
        I[i] = Phi(a) + Phi(b) - 2 * Phi(s) + i * (2 * s - a - b)
    return I


def test_fractional_reference_numerators():
    """quan -> mean references are fractional; scaled by the window count they
    are integers, and the scale-free E must equal the integral form computed
    in exact integers on the scaled masses."""
    g = rng(32)
    H, W, T, B = 9, 10, 3, 5
    bins = g.integers(0, B, (1, H, W)).astype(np.uint8)
    cR = oracle.reference_hist(bins, T, B, "mean")[0]
    nw = (H - T + 1) * (W - T + 1)
    cRi = np.rint(cR * nw).astype(np.int64)
    assert np.allclose(cRi, cR * nw)
    for (y, x) in [(0, 0), (4, 4), (8, 9), (0, 5)]:
        E, I, Pt, _ = oracle.window_errors(bins[0], T, B, cR, y, x, numerators=True)
        sy, sx = windows(H, W, T, y, x)
        P = np.bincount(bins[0, sy, sx].ravel(), minlength=B)
        n = P.sum()
        cP_s = np.cumsum(P) * int(cRi[-1])      # P~ in units of 1/nw
        cR_s = cRi * n                          # R~ in units of 1/nw
        Iref = closed_form_numerators(cP_s, cR_s)
        with np.errstate(invalid="ignore", divide="ignore"):
            Eref = np.where(P > 0, Iref / (P * cRi[-1]), 0.0)
        np.testing.assert_allclose(E, Eref, rtol=1e-12, atol=1e-12)


def test_bin_mismatch_scale_free():
    g = rng(33)
    for _ in range(20):
        B = int(g.integers(2, 10))
        n, m = int(g.integers(1, 20)), int(g.integers(1, 20))
        P = np.bincount(g.integers(0, B, n), minlength=B) * m
        R = np.bincount(g.integers(0, B, m), minlength=B) * n
        E1, _ = oracle.bin_mismatch(P, R)
        E2, _ = oracle.bin_mismatch(P / 7.0, R / 7.0)
        np.testing.assert_allclose(E2, E1, rtol=1e-12, atol=1e-12)


def test_score_with_bin_median_reference_zero_on_periodic():
    g = rng(34)
    C, T, B = 2, 5, 4
    tile = g.standard_normal((C, T, T)).astype(np.float32)
    X = np.tile(tile, (1, 6, 6))
    for ref in ("quan_median", "quan_mean", "mean_quan"):
        m, R, bins = oracle.fit(X, 0, B, T, preproc=0, reference=ref)
        out = oracle.score(bins, T, B, m.cR, m.delta, 0.0)
        r = T // 2
        assert np.abs(out.A[2 * r:-2 * r, 2 * r:-2 * r]).max() < 1e-13, ref


# ---------------------------------------------------------------------------
# Principal-coordinate histograms and the window W1

def test_project_matches_numpy():
    g = rng(40)
    C, H, W, k = 10, 6, 7, 3
    X = g.standard_normal((C, H, W)).astype(np.float32)
    mu, V, _ = oracle.pca(X, k)
    Z = oracle.project(X, mu, V)
    ref = V.T @ (X.reshape(C, -1).astype(np.float64) - mu[:, None])
    np.testing.assert_allclose(Z.reshape(k, -1), ref, rtol=1e-12, atol=1e-12)


def brute_w1_score(bins, T, B, cR, delta, sigma):
    from scipy.ndimage import gaussian_filter1d
    K, H, W = bins.shape
    r = T // 2
    A = np.zeros((H, W))
    for j in range(K):
        refvals = np.repeat(np.arange(B), np.diff(np.concatenate([[0], cR[j]]))).astype(float)
        w1 = np.zeros((H, W))
        for py in range(H):
            for px in range(W):
                sy, sx = windows(H, W, T, py, px)
                vals = bins[j, sy, sx].ravel().astype(float)
                n, m = vals.size, refvals.size
                xs = np.sort(np.repeat(vals, m))
                ys = np.sort(np.repeat(refvals, n))
                w1[py, px] = delta[j] * np.abs(xs - ys).mean()
        for y in range(H):
            for x in range(W):
                sy, sx = windows(H, W, T, y, x)
                A[y, x] += w1[sy, sx].mean()
    A /= K

    def gf(a):
        a = gaussian_filter1d(a, sigma, axis=0, mode="constant", truncate=3.0)
        return gaussian_filter1d(a, sigma, axis=1, mode="constant", truncate=3.0)
    return A, gf(A) / gf(np.ones_like(A))


@pytest.mark.parametrize("case", [(3, 9, 10, 3, 5), (2, 8, 8, 5, 7), (1, 11, 7, 7, 4)])
def test_w1_score_bruteforce(case):
    K, H, W, T, B = case
    g = rng(41 + sum(case))
    Z = g.standard_normal((K, H, W))
    _, _, delta, e = oracle.edges(Z, B)
    bins = oracle.quantize(Z, B, e)
    cR = oracle.reference_cdf(bins, T, B)
    A, S = oracle.w1_score(bins, T, B, cR, delta, 1.0)
    Ar, Sr = brute_w1_score(bins, T, B, cR, delta, 1.0)
    np.testing.assert_allclose(A, Ar, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(S, Sr, rtol=1e-12, atol=1e-13)


def test_w1_score_periodic_zero_and_fit():
    g = rng(42)
    C, T, B, k = 6, 5, 6, 3
    tile = g.standard_normal((C, T, T)).astype(np.float32)
    X = np.tile(tile, (1, 6, 6))
    m, Z, bins = oracle.fit_coords(X, k, B, T)
    A, _ = oracle.w1_score(bins, T, B, m.cR, m.delta, 0.0)
    r = T // 2
    assert np.abs(A[2 * r:-2 * r, 2 * r:-2 * r]).max() < 1e-13
    assert A.max() > 0


# ---------------------------------------------------------------------------
# FCA's sort-based comparison

def test_fca_full_window_matches_numpy_sort():
    g = rng(50)
    H, W, T = 9, 9, 5
    Rc = g.standard_normal((H, W))
    Y = np.sort(g.standard_normal(T * T))
    err = oracle.fca_window(Rc, T, Y, 4, 4)
    vals = Rc[2:7, 2:7].ravel()
    rank = np.argsort(np.argsort(vals, kind="stable"), kind="stable")
    np.testing.assert_allclose(err, np.abs(vals - Y[rank]), rtol=0, atol=1e-15)
    # the error sum is T^2 times the sorted 1-D Wasserstein distance
    assert abs(err.sum() - np.abs(np.sort(vals) - Y).sum()) < 1e-12


def test_fca_border_window_mass_equalised():
    """Clipped window: each window element replicated T^2 times, each reference
    element n_p times, matched in sorted order; an element's error is the mean
    over its replicas."""
    g = rng(51)
    H, W, T = 8, 8, 5
    Rc = g.standard_normal((H, W))
    Y = np.sort(g.standard_normal(T * T))
    for (y, x) in [(0, 0), (1, 7), (7, 3)]:
        err = oracle.fca_window(Rc, T, Y, y, x)
        sy, sx = windows(H, W, T, y, x)
        vals = Rc[sy, sx].ravel()
        n, m = vals.size, T * T
        order = np.argsort(vals, kind="stable")
        reps = np.repeat(order, m)                  # element index of each replica, in sorted order
        ys = np.sort(np.repeat(Y, n))
        e = np.abs(vals[reps] - ys)
        ref = np.array([e[reps == i].mean() for i in range(n)])
        np.testing.assert_allclose(err, ref, rtol=1e-12, atol=1e-13)


def test_fca_on_quantised_values_averages_to_bin_mismatch():
    """Values on bin centres (integers): FCA's errors, averaged over the
    elements of each bin, equal the histogram mismatch of that bin (the
    supplementary correctness argument)."""
    g = rng(52)
    H, W, T, B = 10, 11, 5, 6
    bins = g.integers(0, B, (H, W)).astype(np.uint8)
    refv = np.sort(g.integers(0, B, T * T)).astype(np.float64)
    cR = np.cumsum(np.bincount(refv.astype(int), minlength=B))
    for (y, x) in [(5, 5), (0, 0), (9, 10), (2, 8)]:
        err = oracle.fca_window(bins.astype(np.float64), T, refv, y, x)
        E, _ = oracle.window_errors(bins, T, B, cR, y, x)
        sy, sx = windows(H, W, T, y, x)
        vals = bins[sy, sx].ravel()
        for b in np.unique(vals):
            assert abs(err[vals == b].mean() - E[b]) < 1e-12


def brute_fca(R, T, Y, sigma):
    from scipy.ndimage import gaussian_filter1d
    C, H, W = R.shape
    A = np.zeros((H, W))
    for c in range(C):
        acc = np.zeros((H, W))
        cnt = np.zeros((H, W))
        for py in range(H):
            for px in range(W):
                sy, sx = windows(H, W, T, py, px)
                err = oracle.fca_window(R[c], T, Y[c], py, px).reshape(R[c, sy, sx].shape)
                acc[sy, sx] += err
                cnt[sy, sx] += 1
        A += acc / cnt
    A /= C

    def gf(a):
        a = gaussian_filter1d(a, sigma, axis=0, mode="constant", truncate=3.0)
        return gaussian_filter1d(a, sigma, axis=1, mode="constant", truncate=3.0)
    return A, gf(A) / gf(np.ones_like(A))


def test_fca_score_assembly():
    g = rng(53)
    C, H, W, T = 2, 8, 9, 3
    R = g.standard_normal((C, H, W))
    Y = oracle.reference_values(R, T, "median")
    # the references are the rank-wise lower medians of the sorted windows
    for c in range(C):
        wins = np.sort(np.array(full_windows(R[c], T)), axis=1)
        np.testing.assert_array_equal(Y[c], np.sort(wins, axis=0)[(wins.shape[0] + 1) // 2 - 1])
    A, S, Ach = oracle.fca_score(R, T, Y, 1.0, want_chan=True)
    Ar, Sr = brute_fca(R, T, Y, 1.0)
    np.testing.assert_allclose(A, Ar, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(S, Sr, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(Ach.mean(0), A, rtol=1e-13, atol=1e-15)


def test_quantised_map_converges_to_fca():
    """As the bins get finer, QFCA's map (per-bin errors in feature units,
    median -> quan reference) approaches FCA's map on the same features."""
    g = rng(54)
    C, H, W, T = 2, 14, 14, 5
    R = g.standard_normal((C, H, W))
    Y = oracle.reference_values(R, T, "median")
    Af, _, _ = oracle.fca_score(R, T, Y, 0.0)
    errs = []
    for B in (4, 16, 64, 256):
        lo, hi = R.min(axis=(1, 2)), R.max(axis=(1, 2))
        d = (hi - lo) / B
        e = (lo[:, None] + np.arange(1, B)[None] * d[:, None]).astype(np.float32)
        bins = np.clip(oracle.quantize(R, B, e), 0, 255).astype(np.uint8) if B <= 256 else None
        cR = oracle.reference_literal(R, T, B, e)
        out = oracle.score(bins, T, B, cR, d, 0.0)
        errs.append(np.abs(out.A - Af).mean() / np.abs(Af).mean())
    assert errs[-1] < errs[0] and errs[-1] < 0.05, errs
