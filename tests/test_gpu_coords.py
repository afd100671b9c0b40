"""The principal-coordinate variant (QFCA_PRE_COORDS): the k coordinates
z = V^T (x - mu) (Sec. 3.3 "PCA(W)") are histogrammed and every window is
scored by its 1-Wasserstein distance to the reference (Sec. 3.1), box-averaged
over the windows holding a pixel, averaged over the coordinates and blurred.
Against the FP64 oracle (oracle.fit_coords, oracle.project, oracle.w1_score)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2510_15602_amd as q  # noqa: E402
import qfca_synth  # noqa: E402


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
    tol = 1e-5 * np.abs(o) + 1e-7 * max(np.abs(o).max(), 1e-30)
    bad = np.abs(g - o) > tol
    if bad.any():
        i = np.unravel_index(np.argmax(np.abs(g - o) - tol), g.shape)
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside tolerance; worst at {i}: "
                             f"gpu {g[i]!r} oracle {o[i]!r}")


def coords_model(ctx, om, C, k, B, T, prec=q.QFCA_PREC_FP32):
    prm = q.Params.make(C=C, k=k, B=B, T=T, preproc=q.QFCA_PRE_COORDS, proj_prec=prec)
    return q.qfca_model_create(ctx, prm, om.mu, om.V, om.edges, om.delta, om.cR)


CASES = [(64, 16, 64, 64, 16, 7, 1), (48, 8, 40, 57, 8, 5, 2), (256, 32, 96, 80, 32, 15, 3),
         (100, 10, 50, 70, 16, 9, 4)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "C%d_k%d_H%d_W%d_B%d_T%d" % c[:6])
def test_coords_score_against_oracle(ctx, case):
    C, k, H, W, B, T, seed = case
    say(f"[coords] C={C} k={k} H={H} W={W} B={B} T={T}")
    t = qfca_synth.make_texture(C, H, W, 4000 + seed, anomalies=[("shift", 4, max(4, min(H, W) // 5))])
    om, Z, obins = oracle.fit_coords(t.X, k, B, T)
    m = coords_model(ctx, om, C, k, B, T)
    X = torch.from_numpy(t.X).cuda()
    # bins: exactly #{m : z >= e_m} of the GPU's own float32 z; against the
    # FP64 z only inside the float32 error band of an edge
    gb, gz = q.qfca_quantize(ctx, m, X, resid=True)
    torch.cuda.synchronize()
    gz, gb = gz.cpu().numpy(), gb.cpu().numpy()
    assert gb.shape == (k, H, W)
    for j in range(k):
        np.testing.assert_array_equal(gb[j], np.searchsorted(om.edges[j], gz[j], side="right"))
    scale = np.abs(t.X.astype(np.float64)).sum(0).max() * np.abs(om.V).max(0)
    assert (np.abs(gz - Z).reshape(k, -1).max(1) <= 1e-5 * scale).all()
    diff = gb != obins
    say(f"  bins differing from the FP64 oracle: {int(diff.sum())} of {diff.size}")
    assert diff.mean() < 1e-3
    # score of the oracle's bins
    A, S = oracle.w1_score(obins, T, B, om.cR, om.delta, 1.0)
    out = q.qfca_score_map(ctx, m, torch.from_numpy(obins).cuda(), amap=True, w1=True)
    torch.cuda.synchronize()
    close(out.amap.cpu().numpy(), A, "box-averaged W1 map")
    close(out.score.cpu().numpy(), S, "score")
    # the unsmoothed coordinate-mean window W1 map equals the residual path's
    # W1 by-product for the same bins and reference (same definition)
    prm0 = q.Params.make(C=k, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE)
    m0 = q.qfca_model_create(ctx, prm0, None, None, om.edges, om.delta, om.cR)
    o0 = q.qfca_score_map(ctx, m0, torch.from_numpy(obins).cuda(), w1=True)
    torch.cuda.synchronize()
    assert torch.equal(o0.w1, out.w1)


@pytest.mark.parametrize("C,k,H,W", [(512, 64, 40, 48), (500, 30, 37, 41), (512, 17, 9, 12)],
                         ids=["C512_k64", "C500_k30_ragged", "C512_k17_one_tile"])
def test_coords_bf16_wide(ctx, C, k, H, W):
    """BF16 coordinates of the widest maps (C > 256: every wavefront owns
    whole tiles): z within the BF16 operand rounding of the oracle's, and the
    bins exactly #{m : z >= e_m} of the GPU's own z, four pixels per dword
    store (byte stores where a row is not whole dwords)."""
    say(f"[coords bf16 wide] C={C} k={k} {H}x{W}")
    t = qfca_synth.make_texture(C, H, W, 4200 + k, anomalies=[])
    B, T = 16, 5
    rng = np.random.Generator(np.random.PCG64(4300 + k))
    V, _ = np.linalg.qr(rng.standard_normal((C, k)))  # any orthonormal basis serves
    mu = t.X.reshape(C, -1).mean(1).astype(np.float32)
    V32 = V.astype(np.float32)
    Z = oracle.project(t.X, mu.astype(np.float64), V32.astype(np.float64))
    _, _, delta, edges = oracle.edges(Z, B)
    cR = np.full((k, B), 0, np.int32)
    cR[:, -1] = T * T
    prm = q.Params.make(C=C, k=k, B=B, T=T, preproc=q.QFCA_PRE_COORDS, proj_prec=q.QFCA_PREC_BF16)
    m = q.qfca_model_create(ctx, prm, mu, V32, edges, delta, cR)
    gb, gz = q.qfca_quantize(ctx, m, torch.from_numpy(t.X).cuda(), resid=True)
    torch.cuda.synchronize()
    gz, gb = gz.cpu().numpy(), gb.cpu().numpy()
    assert gb.shape == (k, H, W)
    scale = np.abs(t.X.astype(np.float64) - mu[:, None, None]).max() * np.sqrt(C)
    assert np.abs(gz - Z).max() <= 0.02 * scale
    for j in range(k):
        np.testing.assert_array_equal(gb[j], np.searchsorted(edges[j], gz[j], side="right"),
                                      err_msg=f"component {j}")


def test_coords_tile_independent(ctx):
    C, k, H, W, B, T = 64, 16, 70, 81, 16, 9
    t = qfca_synth.make_texture(C, H, W, 4100, anomalies=[("shift", 4, 10)])
    om, Z, obins = oracle.fit_coords(t.X, k, B, T)
    m = coords_model(ctx, om, C, k, B, T)
    bd = torch.from_numpy(obins).cuda()
    a = q.qfca_score_map(ctx, m, bd, amap=True, w1=True)
    try:
        for (Ws, Hb, S) in [(9, 7, 1), (27, 40, 2), (45, 100, 4)]:
            ctx.set_tile(Ws, Hb, S, 1)
            b = q.qfca_score_map(ctx, m, bd, amap=True, w1=True)
            torch.cuda.synchronize()
            for f in ("score", "amap", "w1"):
                assert torch.equal(getattr(a, f), getattr(b, f)), f"{f} differs with tile {(Ws, Hb, S)}"
    finally:
        ctx.set_tile(0)


@pytest.mark.parametrize("prec", [q.QFCA_PREC_FP32, q.QFCA_PREC_BF16], ids=["fp32", "bf16"])
def test_coords_zero_shot_fit(ctx, prec):
    """qfca_fit_pca with PRE_COORDS: mean and subspace as the oracle's, the
    coordinates' quantiles within the coordinates' own difference, the
    reference exact for the GPU's own bins."""
    ts, p = qfca_synth.workload_small()
    X = ts[0].X
    C, k, B, T = p["C"], 16, p["B"], p["T"]
    qlo, qhi = float(np.float32(p["q_lo"])), float(np.float32(p["q_hi"]))
    om, Z, obins = oracle.fit_coords(X, k, B, T, q_lo=qlo, q_hi=qhi)
    prm = q.Params.make(C=C, k=k, B=B, T=T, preproc=q.QFCA_PRE_COORDS, proj_prec=prec)
    Xd = torch.from_numpy(X).cuda()
    m = q.qfca_fit_pca(ctx, prm, Xd)
    V = m.read("V").astype(np.float64)
    assert np.abs(V @ V.T - om.V @ om.V.T).max() <= 1e-5
    gb, gz = q.qfca_quantize(ctx, m, Xd, resid=True)
    torch.cuda.synchronize()
    gz = gz.cpu().numpy().astype(np.float64)
    lo, hi = m.read("lo"), m.read("hi")
    for j in range(k):  # coordinates are defined up to the eigenvector's sign
        ref = oracle.project(X, m.read("mu").astype(np.float64), V)[j]
        assert np.abs(gz[j] - ref).max() <= (1e-5 if prec == q.QFCA_PREC_FP32 else 5e-2) * np.abs(ref).max()
        v = np.sort(gz[j].ravel())
        n = v.size
        for qq, got in ((qlo, lo[j]), (qhi, hi[j])):
            h = (n - 1) * qq
            f = int(np.floor(h))
            want = v[f] + (h - f) * (v[min(f + 1, n - 1)] - v[f])
            assert abs(got - want) <= 1e-12 * max(abs(want), 1.0)
    np.testing.assert_array_equal(m.read("cR"), oracle.reference_cdf(gb.cpu().numpy(), T, B))
    out = q.qfca_score_map(ctx, m, gb, amap=True)
    torch.cuda.synchronize()
    A, S = oracle.w1_score(gb.cpu().numpy(), T, B, m.read("cR"), m.read("delta"), 1.0)
    close(out.score.cpu().numpy(), S, "zero-shot score")
