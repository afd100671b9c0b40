"""The largest configuration: a 1024x1024 feature map with C=512 channels, PCA
residual k=64 on BF16 MFMA, B=64 bins, T=31 windows, in one batch with
256x256 maps of the same channels.  Parity on sampled pixels: the channel
mean A(x) that the GPU computes from its own bins and model equals the
oracle's direct evaluation at those pixels (corners, edges, interior)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2510_15602_amd as q  # noqa: E402
import qfca_synth  # noqa: E402

C, K, B, T = 512, 64, 64, 31


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return q.Context(0)


def sample_pixels(H, W, rng, n_inner=4):
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, W // 2), (T // 2, W // 3),
           (H - 1 - T // 2, 2 * W // 3), (H // 3, 1)]
    pts += [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(n_inner)]
    ys = np.array([p[0] for p in pts], np.int32)
    xs = np.array([p[1] for p in pts], np.int32)
    return ys, xs


def test_large_batch_matches_oracle_on_sampled_pixels(ctx):
    prm = q.Params.make(C=C, k=K, B=B, T=T, proj_prec=q.QFCA_PREC_BF16)
    shapes = [(1024, 1024), (256, 256), (256, 256)]
    jobs = []
    for i, (H, W) in enumerate(shapes):
        if H == 1024:
            anoms = [("shift", 16, 96), ("scale", 16, 96), ("permute", 16, 96), ("shift", 16, 96),
                     ("scale", 16, 96)]
        else:
            anoms = [("shift", 8, 32)]
        say(f"[large] image {i}: {H}x{W} C={C}, fit (BF16 projection, k={K})")
        X, _, _ = qfca_synth.make_texture_torch(C, H, W, 500 + i, "cuda", anomalies=anoms)
        m = q.qfca_fit_pca(ctx, prm, X)
        jobs.append((m, X, torch.empty((H, W), device="cuda"),
                     torch.empty((C, H, W), dtype=torch.uint8, device="cuda"),
                     torch.empty((H, W), device="cuda")))
    torch.cuda.synchronize()
    say("[large] batch launch")
    q.qfca_score_batch(ctx, jobs)
    torch.cuda.synchronize()
    assert q.qfca_batch_error(ctx) == 0
    rng = np.random.Generator(np.random.PCG64(31))
    for i, (m, X, score, bins, amap) in enumerate(jobs[:2]):
        H, W = X.shape[1:]
        ys, xs = sample_pixels(H, W, rng)
        say(f"[large] image {i}: oracle A(x) at {ys.size} pixels")
        ref = oracle.amap_pixels(bins.cpu().numpy(), T, B, m.read("cR"), m.read("delta"), ys, xs)
        got = amap.cpu().numpy()[ys, xs].astype(np.float64)
        tol = 1e-5 * np.abs(ref) + 1e-7 * np.abs(ref).max()
        err = np.abs(got - ref)
        say(f"   max rel err {float((err / np.maximum(np.abs(ref), 1e-30)).max()):.2e}")
        assert (err <= tol).all(), (err - tol).max()
        assert np.isfinite(score.cpu().numpy()).all()


def test_large_single_image_path_equals_batch(ctx):
    """The standalone projection (512 channels) and score kernel (T=31, one
    channel per wavefront) on the large map agree with the batched kernel."""
    prm = q.Params.make(C=C, k=K, B=B, T=T, proj_prec=q.QFCA_PREC_BF16)
    X, _, _ = qfca_synth.make_texture_torch(C, 1024, 1024, 520, "cuda",
                                            anomalies=[("shift", 16, 96), ("permute", 16, 96)])
    m = q.qfca_fit_pca(ctx, prm, X)
    score = torch.empty((1024, 1024), device="cuda")
    bins = torch.empty((C, 1024, 1024), dtype=torch.uint8, device="cuda")
    amap = torch.empty((1024, 1024), device="cuda")
    say("[large single] batch of one")
    q.qfca_score_batch(ctx, [(m, X, score, bins, amap)])
    b1, _ = q.qfca_quantize(ctx, m, X)
    say("[large single] standalone score")
    o1 = q.qfca_score_map(ctx, m, b1, amap=True)
    torch.cuda.synchronize()
    assert torch.equal(b1, bins)
    a = o1.amap.cpu().numpy().astype(np.float64)
    g = amap.cpu().numpy().astype(np.float64)
    tol = 1e-5 * np.abs(a) + 1e-7 * np.abs(a).max()
    assert (np.abs(g - a) <= tol).all()
