"""Edge cases of the HIP path: bins of values planted on and next to the
edges (through the MFMA projection), windows beyond the block-walk kernels
(T = 33, 63), the largest channel count, and the ABI's argument checks."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2510_15602_amd as q  # noqa: E402

RTOL, ATOL_REL = 1e-5, 1e-7


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return q.Context(0)


def close(g, o, what):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    tol = RTOL * np.abs(o) + ATOL_REL * max(np.abs(o).max(), 1e-30)
    assert (np.abs(g - o) <= tol).all(), f"{what}: worst {(np.abs(g - o) - tol).max()}"


def planted_values(edges, rng, n):
    """Values on every edge, one float32 step either side of it, and uniform
    ones over and beyond the edge range."""
    e = edges.astype(np.float32)
    vals = [e, np.nextafter(e, np.float32(np.inf)), np.nextafter(e, np.float32(-np.inf))]
    span = float(e[-1] - e[0]) if e.size > 1 else 1.0
    vals.append(rng.uniform(e[0] - span, e[-1] + span, n).astype(np.float32))
    v = np.concatenate(vals).astype(np.float32)
    return rng.permutation(np.resize(v, n))


@pytest.mark.parametrize("C,prec,grid,H,W", [(64, q.QFCA_PREC_FP32, True, 40, 48),
                                             (256, q.QFCA_PREC_FP32, True, 40, 48),
                                             (256, q.QFCA_PREC_BF16, True, 40, 48),
                                             (64, q.QFCA_PREC_FP32, False, 40, 48),
                                             (512, q.QFCA_PREC_BF16, True, 40, 48),
                                             (500, q.QFCA_PREC_BF16, False, 37, 41),
                                             (449, q.QFCA_PREC_BF16, True, 9, 12)],
                         ids=["C64_fp32", "C256_fp32", "C256_bf16", "C64_fp32_irregular_edges", "C512_bf16",
                              "C500_bf16_irregular_ragged", "C449_bf16_one_ragged_tile"])
def test_bins_of_values_on_edges(ctx, C, prec, grid, H, W):
    """With mu = 0 and an all-zero basis the residual is the feature itself,
    so values can be placed exactly on the edges; the bins must equal
    #{m : r >= e_m} for every one (regular grid edges take the arithmetic
    shortcut away from edges; irregular edges are always searched).  C > 256
    in BF16 runs the kernel whose wavefronts own whole tiles and write bins
    four pixels to a dword (byte by byte when a row is not a whole number of
    dwords: the 37 x 41 and 9 x 12 maps)."""
    rng = np.random.Generator(np.random.PCG64(C + prec + grid))
    B = 32
    lo = rng.uniform(-3, -1, C)
    delta = rng.uniform(0.05, 0.3, C)
    if grid:
        edges = np.stack([(lo[c] + delta[c] * np.arange(1, B)).astype(np.float32) for c in range(C)])
    else:
        edges = np.sort(rng.uniform(-2, 2, (C, B - 1)).astype(np.float32), axis=1)
    X = np.stack([planted_values(edges[c], rng, H * W).reshape(H, W) for c in range(C)]).astype(np.float32)
    prm = q.Params.make(C=C, k=32 if prec == q.QFCA_PREC_BF16 else 1, B=B, T=5, proj_prec=prec)
    V = np.zeros((C, prm.k), np.float32)
    cR = np.full((C, B), 25, np.int32)  # any valid reference of mass T*T
    m = q.qfca_model_create(ctx, prm, np.zeros(C, np.float32), V, edges, delta, cR)
    bins, resid = q.qfca_quantize(ctx, m, torch.from_numpy(X).cuda(), resid=True)
    torch.cuda.synchronize()
    r = resid.cpu().numpy()
    np.testing.assert_array_equal(r, X)  # the residual is exact here
    g = bins.cpu().numpy()
    for c in range(C):
        np.testing.assert_array_equal(g[c], np.searchsorted(edges[c], X[c], side="right"),
                                      err_msg=f"channel {c}")
    say(f"[edges] C={C} prec={prec} grid={grid} {H}x{W}: {g.size} bins exact")


@pytest.mark.parametrize("path", ["valu", "fp32", "bf16", "bf16_wide"])
def test_zero_width_channel(ctx, path):
    """A channel of zero width (delta = 0, every edge at one value) still
    takes #{m : r >= e_m}: bin 0 below the edge value, B - 1 at or above it,
    on the VALU projection, the MFMA projections and the wide BF16 kernel."""
    C = 300 if path == "bf16_wide" else 8
    B, H, W = 16, 9, 20
    rng = np.random.Generator(np.random.PCG64(77))
    lo = rng.uniform(-2, -1, C)
    delta = rng.uniform(0.1, 0.2, C)
    edges = np.stack([(lo[c] + delta[c] * np.arange(1, B)).astype(np.float32) for c in range(C)])
    z = 3  # the zero-width channel
    delta[z] = 0.0
    edges[z] = np.float32(0.5)
    X = rng.uniform(-3, 3, (C, H, W)).astype(np.float32)
    X[z] = rng.choice(np.array([0.25, 0.5, 0.75, np.nextafter(np.float32(0.5), np.float32(0))], np.float32),
                      (H, W))
    if path == "valu":
        prm = q.Params.make(C=C, k=0, B=B, T=3, preproc=q.QFCA_PRE_NONE)
        mu, V = None, None
    else:
        k = 1 if path == "fp32" else min(32, C - 1)
        prec = q.QFCA_PREC_FP32 if path == "fp32" else q.QFCA_PREC_BF16
        prm = q.Params.make(C=C, k=k, B=B, T=3, proj_prec=prec)
        mu, V = np.zeros(C, np.float32), np.zeros((C, k), np.float32)
    cR = np.full((C, B), 9, np.int32)
    m = q.qfca_model_create(ctx, prm, mu, V, edges, delta, cR)
    bins, _ = q.qfca_quantize(ctx, m, torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    g = bins.cpu().numpy()
    for c in range(C):
        np.testing.assert_array_equal(g[c], np.searchsorted(edges[c], X[c], side="right"), err_msg=f"channel {c}")


@pytest.mark.parametrize("C,k,H,W", [(512, 64, 48, 80), (512, 32, 33, 47), (300, 50, 20, 31)],
                         ids=["C512_k64", "C512_k32_ragged", "C300_k50"])
def test_bf16_projection_wide(ctx, C, k, H, W):
    """BF16 projection of the widest maps (C > 256) against the FP64
    oracle: the residual within the BF16 operand rounding, and the bins
    exactly #{m : r >= e_m} of the GPU's own residual."""
    rng = np.random.Generator(np.random.PCG64(C * 7 + k))
    say(f"[bf16 wide] C={C} k={k} {H}x{W}")
    X = rng.standard_normal((C, H, W)).astype(np.float32) * rng.uniform(0.5, 2.0, (C, 1, 1)).astype(np.float32)
    mu = X.reshape(C, -1).mean(1)
    V, _ = np.linalg.qr(rng.standard_normal((C, k)))
    B = 32
    Rr = oracle.residual(X, mu.astype(np.float32).astype(np.float64), V.astype(np.float32).astype(np.float64))
    _, _, delta, edges = oracle.edges(Rr, B)
    prm = q.Params.make(C=C, k=k, B=B, T=5, proj_prec=q.QFCA_PREC_BF16)
    cR = np.full((C, B), 25, np.int32)
    m = q.qfca_model_create(ctx, prm, mu.astype(np.float32), V.astype(np.float32), edges, delta, cR)
    bins, resid = q.qfca_quantize(ctx, m, torch.from_numpy(X).cuda(), resid=True)
    torch.cuda.synchronize()
    r = resid.cpu().numpy().astype(np.float64)
    # BF16 operands (8 significant bits) with FP32 accumulation: the
    # reconstruction's error is a few 2^-8 of |x - mu| summed over C
    scale = np.abs(X - mu[:, None, None]).reshape(C, -1).max()
    assert np.abs(r - Rr).max() <= 0.05 * scale
    g = bins.cpu().numpy()
    e32 = edges.astype(np.float32)
    for c in range(C):
        np.testing.assert_array_equal(g[c], np.searchsorted(e32[c], resid[c].cpu().numpy(), side="right"),
                                      err_msg=f"channel {c}")


def rand_problem(seed, C, H, W, T, B):
    g = np.random.Generator(np.random.PCG64(seed))
    R = g.standard_normal((C, H, W))
    _, _, delta, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    cR = oracle.reference_cdf(bins, T, B) if (H >= T and W >= T) else \
        np.cumsum(np.bincount(g.integers(0, B, T * T), minlength=B))[None].repeat(C, 0)
    return bins, delta, e, cR.astype(np.int32)


@pytest.mark.parametrize("case", [(2, 50, 47, 33, 8), (1, 70, 66, 63, 8), (3, 40, 40, 45, 5)],
                         ids=lambda c: "C%d_H%d_W%d_T%d_B%d" % c)
def test_large_windows_generic_kernel(ctx, case):
    C, H, W, T, B = case
    say(f"[large window] C={C} H={H} W={W} T={T} B={B}")
    bins, delta, e, cR = rand_problem(sum(case), C, H, W, T, B)
    ref = oracle.score(bins, T, B, cR, delta, 1.0, want_w1=True, want_chan=True)
    prm = q.Params.make(C=C, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE)
    m = q.qfca_model_create(ctx, prm, None, None, e, delta, cR)
    out = q.qfca_score_map(ctx, m, torch.from_numpy(bins).cuda(), amap=True, w1=True, achan=True)
    torch.cuda.synchronize()
    close(out.achan.cpu().numpy(), ref.Achan, "per-channel map")
    close(out.amap.cpu().numpy(), ref.A, "channel mean")
    close(out.score.cpu().numpy(), ref.score, "score")
    close(out.w1.cpu().numpy(), ref.W1, "W1")


def test_max_channels_plain(ctx):
    """C = 2048 (the largest accepted), plain QFCA: fit, quantise and score
    against the oracle's fit and score."""
    C, H, W, T, B = 2048, 20, 22, 5, 8
    rng = np.random.Generator(np.random.PCG64(2048))
    X = rng.standard_normal((C, H, W)).astype(np.float32)
    say(f"[max channels] C={C} {H}x{W} T={T} B={B}")
    om, R, obins = oracle.fit(X, 0, B, T, preproc=0)
    prm = q.Params.make(C=C, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE)
    m = q.qfca_fit_pca(ctx, prm, torch.from_numpy(X).cuda())
    np.testing.assert_array_equal(m.read("cR"), om.cR)
    bins, _ = q.qfca_quantize(ctx, m, torch.from_numpy(X).cuda())
    g = bins.cpu().numpy()
    assert (g == obins).mean() > 0.999
    ref = oracle.score(g, T, B, m.read("cR"), m.read("delta"), 1.0)
    out = q.qfca_score_map(ctx, m, bins, amap=True)
    torch.cuda.synchronize()
    close(out.amap.cpu().numpy(), ref.A, "channel mean")
    close(out.score.cpu().numpy(), ref.score, "score")


def test_abi_rejects_bad_arguments(ctx):
    X = torch.zeros((4, 8, 8), device="cuda")
    ok = q.Params.make(C=4, k=0, B=4, T=3, preproc=q.QFCA_PRE_NONE)
    cases = [
        (q.Params.make(C=4, k=0, B=4, T=4, preproc=q.QFCA_PRE_NONE), 7),    # even window
        (q.Params.make(C=4, k=0, B=65, T=3, preproc=q.QFCA_PRE_NONE), 7),   # more bins than a byte code allows
        (q.Params.make(C=4, k=4, B=4, T=3), 7),                             # k must stay below C
        (q.Params.make(C=4, k=0, B=4, T=3, q_lo=0.9, q_hi=0.1, preproc=q.QFCA_PRE_NONE), 1),
    ]
    for prm, status in cases:
        with pytest.raises(q.QfcaError) as err:
            q.qfca_fit_pca(ctx, prm, X)
        assert err.value.status == status, (prm.as_dict(), err.value)
    Xn = X.clone()
    Xn[1, 2, 3] = float("nan")
    with pytest.raises(q.QfcaError) as err:
        q.qfca_fit_pca(ctx, ok, Xn)
    assert err.value.status == 6
    with pytest.raises(q.QfcaError) as err:  # the reference needs a full window
        q.qfca_fit_pca(ctx, q.Params.make(C=4, k=0, B=4, T=9, preproc=q.QFCA_PRE_NONE), X)
    assert err.value.status == 2
    m = q.qfca_fit_pca(ctx, ok, X + torch.arange(64, device="cuda", dtype=torch.float32).reshape(8, 8))
    with pytest.raises(q.QfcaError) as err:  # an empty map (no storage: a null pointer, or H = 0)
        q.qfca_score_map(ctx, m, torch.zeros((4, 0, 8), dtype=torch.uint8, device="cuda"))
    assert err.value.status in (1, 2)
    torch.cuda.synchronize()
