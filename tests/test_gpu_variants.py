"""The association and reference variants against the FP64 oracle, through
the C ABI: Gaussian association weights of finite sigma_p (Eq. 2, Sec. 4.5.4)
and the reference choices of Sec. 4.5.3 / Tab. 3 (mean -> quan, quan ->
median, quan -> mean) besides the default median -> quan."""
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


def problem(seed, C, H, W, T, B):
    g = np.random.Generator(np.random.PCG64(seed))
    R = g.standard_normal((C, H, W))
    _, _, delta, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    return R, bins, delta, e


@pytest.mark.parametrize("case", [(3, 40, 37, 5, 8, 1.0), (2, 64, 70, 7, 16, 2.0), (2, 50, 61, 15, 32, 3.0),
                                  (1, 45, 45, 31, 64, 8.0), (2, 30, 33, 9, 10, 0.5), (1, 50, 52, 35, 8, 6.0)],
                         ids=lambda c: "C%d_H%d_W%d_T%d_B%d_sp%g" % c)
def test_gaussian_association(ctx, case):
    """Finite sigma_p against the oracle's direct weighted mean over the
    windows holding each pixel, through the block walk (window sides up to
    31) and the column walk; each walk's maps bitwise the same for every
    tile."""
    C, H, W, T, B, sp = case
    say(f"[sigma_p] C={C} H={H} W={W} T={T} B={B} sigma_p={sp}")
    _, bins, delta, e = problem(50 + T, C, H, W, T, B)
    cR = oracle.reference_cdf(bins, T, B).astype(np.int32)
    ref = oracle.score(bins, T, B, cR, delta, 1.0, want_w1=True, want_chan=True, sigma_p=sp)
    prm = q.Params.make(C=C, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE, sigma_p=sp)
    m = q.qfca_model_create(ctx, prm, None, None, e, delta, cR)
    bd = torch.from_numpy(bins).cuda()
    out = q.qfca_score_map(ctx, m, bd, amap=True, w1=True, achan=True)
    torch.cuda.synchronize()
    close(out.achan.cpu().numpy(), ref.Achan, "per-channel maps")
    close(out.amap.cpu().numpy(), ref.A, "channel mean")
    close(out.score.cpu().numpy(), ref.score, "score")
    close(out.w1.cpu().numpy(), ref.W1, "window W1")
    block = T <= 31  # the automatic tile runs the block walk
    try:
        if block:
            for (Ws, Hb) in [(T, 8), (2 * T, 5), (3 * T, 64)]:
                ctx.set_tile(Ws, Hb, 1, 1)
                o2 = q.qfca_score_map(ctx, m, bd, amap=True, w1=True, achan=True)
                torch.cuda.synchronize()
                for f in ("score", "amap", "w1", "achan"):
                    assert torch.equal(getattr(out, f), getattr(o2, f)), f"{f} differs with tile {(Ws, Hb)}"
        col = None
        for (Ws, Hb) in [(16, 8), (40, 13), (7, 100)]:
            ctx.set_tile(Ws, Hb, 1, 0)
            o2 = q.qfca_score_map(ctx, m, bd, amap=True, w1=True, achan=True)
            torch.cuda.synchronize()
            if col is None:
                col = o2
                close(o2.achan.cpu().numpy(), ref.Achan, "per-channel maps (column walk)")
                close(o2.score.cpu().numpy(), ref.score, "score (column walk)")
                if not block:
                    for f in ("score", "amap", "w1", "achan"):
                        assert torch.equal(getattr(out, f), getattr(o2, f)), f"{f} differs with tile {(Ws, Hb)}"
            else:
                for f in ("score", "amap", "w1", "achan"):
                    assert torch.equal(getattr(col, f), getattr(o2, f)), f"{f} differs with tile {(Ws, Hb)}"
    finally:
        ctx.set_tile(0)


def test_sigma_p_large_tends_to_box(ctx):
    """exp(-d^2 / (2 sigma_p^2)) -> 1: a very large sigma_p gives the plain
    mean of the default association."""
    C, H, W, T, B = 2, 48, 50, 9, 16
    _, bins, delta, e = problem(77, C, H, W, T, B)
    cR = oracle.reference_cdf(bins, T, B).astype(np.int32)
    bd = torch.from_numpy(bins).cuda()
    box = q.qfca_score_map(ctx, q.qfca_model_create(ctx, q.Params.make(C=C, k=0, B=B, T=T, preproc=0),
                                                    None, None, e, delta, cR), bd, amap=True)
    big = q.qfca_score_map(ctx, q.qfca_model_create(ctx, q.Params.make(C=C, k=0, B=B, T=T, preproc=0,
                                                                       sigma_p=1e6), None, None, e, delta, cR),
                           bd, amap=True)
    torch.cuda.synchronize()
    close(big.amap.cpu().numpy(), box.amap.cpu().numpy(), "sigma_p = 1e6 against the box")


@pytest.mark.parametrize("kind", ["quan_median", "quan_mean"])
@pytest.mark.parametrize("case", [(3, 40, 37, 5, 8), (2, 70, 64, 15, 32), (1, 50, 45, 9, 64)],
                         ids=lambda c: "C%d_H%d_W%d_T%d_B%d" % c)
def test_bin_wise_references(ctx, case, kind):
    """quan -> median / quan -> mean from the GPU's window-count table equal
    the oracle's bin-wise statistics of the full-window histograms, and the
    score with that general reference matches the oracle's."""
    C, H, W, T, B = case
    say(f"[reference {kind}] C={C} H={H} W={W} T={T} B={B}")
    _, bins, delta, e = problem(90 + T + B, C, H, W, T, B)
    refk = q.QFCA_REF_QUAN_MEDIAN if kind == "quan_median" else q.QFCA_REF_QUAN_MEAN
    prm = q.Params.make(C=C, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE, reference=refk)
    m = q.qfca_model_create(ctx, prm, None, None, e, delta, None)
    bd = torch.from_numpy(bins).cuda()
    q.qfca_fit_reference(ctx, m, bd)
    w = m.read("cRw")
    ow = oracle.reference_hist(bins, T, B, kind="median" if kind == "quan_median" else "mean")
    if kind == "quan_median":
        np.testing.assert_array_equal(w, ow)
    else:
        np.testing.assert_allclose(w, ow, rtol=1e-13, atol=0)
    out = q.qfca_score_map(ctx, m, bd, amap=True, w1=True, achan=True)
    torch.cuda.synchronize()
    ref = oracle.score(bins, T, B, w, delta, 1.0, want_w1=True, want_chan=True)
    close(out.achan.cpu().numpy(), ref.Achan, "per-channel maps")
    close(out.score.cpu().numpy(), ref.score, "score")
    close(out.w1.cpu().numpy(), ref.W1, "window W1")


def test_general_reference_weights(ctx):
    """Arbitrary real reference weights (any mass) set from the host, scored
    against the oracle; integer weights of mass T*T take the integer path and
    score bit for bit like a qfca_model_create reference."""
    C, H, W, T, B = 3, 45, 52, 7, 12
    _, bins, delta, e = problem(123, C, H, W, T, B)
    g = np.random.Generator(np.random.PCG64(124))
    w = np.cumsum(g.uniform(0.0, 3.0, (C, B)), axis=1)
    w[1, 3] = w[1, 2]  # an empty reference bin
    prm = q.Params.make(C=C, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE)
    m = q.qfca_model_create(ctx, prm, None, None, e, delta, None)
    q.qfca_model_set_reference(ctx, m, w)
    bd = torch.from_numpy(bins).cuda()
    out = q.qfca_score_map(ctx, m, bd, amap=True, achan=True)
    torch.cuda.synchronize()
    ref = oracle.score(bins, T, B, w, delta, 1.0, want_chan=True)
    close(out.achan.cpu().numpy(), ref.Achan, "per-channel maps")
    close(out.score.cpu().numpy(), ref.score, "score")
    cR = oracle.reference_cdf(bins, T, B).astype(np.int32)
    m1 = q.qfca_model_create(ctx, prm, None, None, e, delta, cR)
    m2 = q.qfca_model_create(ctx, prm, None, None, e, delta, None)
    q.qfca_model_set_reference(ctx, m2, cR.astype(np.float64))
    np.testing.assert_array_equal(m2.read("cR"), cR)
    a = q.qfca_score_map(ctx, m1, bd).score
    b = q.qfca_score_map(ctx, m2, bd).score
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_mean_quan_reference_from_the_fit(ctx):
    """mean -> quan: the rank-wise mean of the sorted full windows of the GPU's
    own residual, quantised with its own edges, equals the oracle's literal
    computation on that residual and those edges."""
    ts, p = qfca_synth.workload_small()
    X = ts[0].X
    prm = q.Params.make(C=p["C"], k=p["k"], B=p["B"], T=p["T"], reference=q.QFCA_REF_MEAN_QUAN)
    m = q.qfca_fit_pca(ctx, prm, torch.from_numpy(X).cuda())
    _, resid = q.qfca_quantize(ctx, m, torch.from_numpy(X).cuda(), resid=True)
    torch.cuda.synchronize()
    lit = oracle.reference_literal(resid.cpu().numpy().astype(np.float64), p["T"], p["B"], m.read("edges"),
                                   kind="mean")
    np.testing.assert_array_equal(m.read("cR"), lit)
    # and it differs from the median reference of the same image (a real choice)
    m0 = q.qfca_fit_pca(ctx, q.Params.make(C=p["C"], k=p["k"], B=p["B"], T=p["T"]), torch.from_numpy(X).cuda())
    assert not np.array_equal(m0.read("cR"), m.read("cR"))


def test_variants_export_import(ctx):
    C, H, W, T, B = 2, 40, 44, 7, 10
    _, bins, delta, e = problem(321, C, H, W, T, B)
    prm = q.Params.make(C=C, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE, sigma_p=2.5,
                        reference=q.QFCA_REF_QUAN_MEAN)
    m = q.qfca_model_create(ctx, prm, None, None, e, delta, None)
    bd = torch.from_numpy(bins).cuda()
    q.qfca_fit_reference(ctx, m, bd)
    blob = q.qfca_model_export(m)
    m2 = q.qfca_model_import(ctx, blob)
    assert m2.params.sigma_p == 2.5 and m2.params.reference == q.QFCA_REF_QUAN_MEAN
    np.testing.assert_array_equal(m2.read("cRw"), m.read("cRw"))
    a = q.qfca_score_map(ctx, m, bd).score
    b = q.qfca_score_map(ctx, m2, bd).score
    torch.cuda.synchronize()
    assert torch.equal(a, b)
