"""The batched path (one persistent quantise-histogram-score kernel under a
HIP graph) against the single-image path and the FP64 oracle."""
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


def close(g, o, rtol=1e-5, arel=1e-7):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    tol = rtol * np.abs(o) + arel * max(np.abs(o).max(), 1e-30)
    assert (np.abs(g - o) <= tol).all(), float((np.abs(g - o) - tol).max())


def make_jobs(ctx, shapes, C, k, B, T, prec, seed0):
    prm = q.Params.make(C=C, k=k, B=B, T=T, proj_prec=prec)
    jobs = []
    for i, (H, W) in enumerate(shapes):
        t = qfca_synth.make_texture(C, H, W, seed0 + i, anomalies=[("shift", 2, max(3, min(H, W) // 3))])
        X = torch.from_numpy(t.X).cuda()
        m = q.qfca_fit_pca(ctx, prm, X)
        jobs.append((m, X, torch.empty((H, W), device="cuda"), torch.empty((C, H, W), dtype=torch.uint8, device="cuda"),
                     torch.empty((H, W), device="cuda")))
    return jobs


CONFIGS = [
    # C, k, B, T, precision, shapes
    (64, 16, 16, 7, q.QFCA_PREC_FP32, [(40, 52), (64, 64), (23, 97), (130, 80), (9, 11)]),
    (256, 32, 32, 15, q.QFCA_PREC_BF16, [(96, 96), (64, 130), (150, 70)]),
    (256, 32, 32, 15, q.QFCA_PREC_FP32, [(80, 100), (48, 48)]),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"C{c[0]}_k{c[1]}_B{c[2]}_T{c[3]}_p{c[4]}")
def test_batch_equals_single_image_path(ctx, cfg):
    C, k, B, T, prec, shapes = cfg
    say(f"[batch] C={C} k={k} B={B} T={T} prec={prec} shapes={shapes}")
    jobs = make_jobs(ctx, shapes, C, k, B, T, prec, 700)
    q.qfca_score_batch(ctx, jobs)
    torch.cuda.synchronize()
    assert q.qfca_batch_error(ctx) == 0
    for (m, X, score, bins, amap) in jobs:
        b1, _ = q.qfca_quantize(ctx, m, X)
        o1 = q.qfca_score_map(ctx, m, b1, amap=True)
        torch.cuda.synchronize()
        assert torch.equal(bins, b1), "batch bins differ from qfca_quantize"
        # same block-walk arithmetic and an order-free channel sum: bitwise
        assert torch.equal(amap, o1.amap), "batch channel mean differs from qfca_score_map"
        assert torch.equal(score, o1.score), "batch score differs from qfca_score_map"


def test_batch_alone_equals_in_mix(ctx):
    C, k, B, T, prec, shapes = CONFIGS[0]
    say("[batch alone vs mix]")
    jobs = make_jobs(ctx, shapes, C, k, B, T, prec, 800)
    q.qfca_score_batch(ctx, jobs)
    torch.cuda.synchronize()
    mixed = [j[2].clone() for j in jobs]
    for i, j in enumerate(jobs):
        j[2].zero_()
        q.qfca_score_batch(ctx, [j])
        torch.cuda.synchronize()
        assert torch.equal(j[2], mixed[i]), f"image {i} differs alone vs in the batch"
    # a different order and repeated images in one batch
    order = [jobs[3], jobs[0], jobs[4], jobs[1], jobs[2]]
    q.qfca_score_batch(ctx, order)
    torch.cuda.synchronize()
    for i, j in enumerate(jobs):
        assert torch.equal(j[2], mixed[i])
    assert q.qfca_batch_error(ctx) == 0


def test_batch_against_oracle(ctx):
    """One image through the batch with the oracle's model: same tolerance as
    the single-image parity tests (bins compared inside the float32 edge band)."""
    ts, p = qfca_synth.workload_small()
    X = ts[0].X
    om, R, obins = oracle.fit(X, p["k"], p["B"], p["T"])
    prm = q.Params.make(C=p["C"], k=p["k"], B=p["B"], T=p["T"])
    m = q.qfca_model_create(ctx, prm, om.mu, om.V, om.edges, om.delta, om.cR)
    Xd = torch.from_numpy(X).cuda()
    H, W = X.shape[1:]
    score = torch.empty((H, W), device="cuda")
    bins = torch.empty(X.shape, dtype=torch.uint8, device="cuda")
    q.qfca_score_batch(ctx, [(m, Xd, score, bins)])
    torch.cuda.synchronize()
    g = bins.cpu().numpy()
    if (g == obins).all():
        ref = oracle.score(obins, p["T"], p["B"], om.cR, om.delta, 1.0)
        close(score.cpu().numpy(), ref.score)
    else:  # differing bins sit on float32 edge ties; score the GPU's own bins
        ref = oracle.score(g, p["T"], p["B"], om.cR, om.delta, 1.0)
        close(score.cpu().numpy(), ref.score)


def test_autotune_picks_a_valid_tile(ctx):
    C, k, B, T, prec, shapes = CONFIGS[0]
    jobs = make_jobs(ctx, shapes[:3], C, k, B, T, prec, 900)
    q.qfca_score_batch(ctx, jobs)
    torch.cuda.synchronize()
    before = [j[2].clone() for j in jobs]
    ws, hb, ms = q.qfca_autotune(ctx, jobs)
    say(f"[autotune] Ws={ws} Hb={hb} {ms:.3f} ms")
    assert ws % T == 0 and hb in (64, 128, 256) and ms > 0
    q.qfca_score_batch(ctx, jobs)
    torch.cuda.synchronize()
    for i, (m, X, score, bins, amap) in enumerate(jobs):
        o1 = q.qfca_score_map(ctx, m, bins, amap=True)
        torch.cuda.synchronize()
        # the tuned tile changes no bit, in the batch or the single-image path
        assert torch.equal(score, o1.score) and torch.equal(score, before[i])


@pytest.mark.parametrize("cfg", CONFIGS[:2], ids=lambda c: f"C{c[0]}_k{c[1]}_B{c[2]}_T{c[3]}_p{c[4]}")
def test_batch_channel_maps_against_oracle(ctx, cfg):
    """Per-channel maps of every image of a batch, every pixel and channel,
    against the oracle on the batch's own bins and the model."""
    C, k, B, T, prec, shapes = cfg
    say(f"[batch channel maps] C={C} k={k} B={B} T={T} prec={prec} shapes={shapes}")
    jobs = make_jobs(ctx, shapes, C, k, B, T, prec, 950)
    items = [j + (torch.empty((C,) + tuple(j[2].shape), device="cuda"),) for j in jobs]
    q.qfca_score_batch(ctx, items)
    torch.cuda.synchronize()
    assert q.qfca_batch_error(ctx) == 0
    for (m, X, score, bins, amap, achan) in items:
        ref = oracle.score(bins.cpu().numpy(), T, B, m.read("cR"), m.read("delta"), 1.0, want_chan=True)
        close(achan.cpu().numpy(), ref.Achan)
        close(amap.cpu().numpy(), ref.A)
        close(score.cpu().numpy(), ref.score)
