"""The batched workloads at their full sizes, in the launch configuration the
benchmark uses (one qfca_score_batch over every image), checked on sampled
outputs the oracle computes one by one:

* 64 images, sides drawn from {128, 192, 256, 384, 512}, C = 256, PCA k = 32
  on BF16 MFMA, B = 32, T = 15;
* 8 maps of 1024 x 1024 and 32 of 256 x 256, C = 512, k = 64 on BF16 MFMA,
  B = 64, T = 31.

For sampled images: the batch's bins equal qfca_quantize's (same model), the
channel mean A(x) before the blur equals the oracle's direct evaluation at
sampled pixels (corners, borders, interior) from those bins and the model,
and the blurred score at an interior pixel equals the oracle's A on the 7 x 7
neighbourhood blurred with the sigma = 1 Gaussian (radius 3)."""
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


def sample_pixels(H, W, T, rng, n_inner=4):
    r = T // 2
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, W // 2), (r, W // 3),
           (H - 1 - r, 2 * W // 3), (H // 3, 1)]
    pts += [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(n_inner)]
    return np.array([p[0] for p in pts], np.int32), np.array([p[1] for p in pts], np.int32)


def check_image(ctx, m, X, score, bins, amap, T, B, rng, what):
    H, W = X.shape[1:]
    b1, _ = q.qfca_quantize(ctx, m, X)
    torch.cuda.synchronize()
    assert torch.equal(b1, bins), f"{what}: batch bins differ from qfca_quantize"
    hb = bins.cpu().numpy()
    cR, delta = m.read("cR"), m.read("delta")
    ys, xs = sample_pixels(H, W, T, rng)
    ref = oracle.amap_pixels(hb, T, B, cR, delta, ys, xs)
    got = amap.cpu().numpy()[ys, xs].astype(np.float64)
    tol = 1e-5 * np.abs(ref) + 1e-7 * max(np.abs(ref).max(), 1e-30)
    assert (np.abs(got - ref) <= tol).all(), f"{what}: A(x) worst {(np.abs(got - ref) - tol).max():.3e}"
    # blurred score at one interior pixel: the oracle's blur (radius 3 at
    # sigma = 1) of its A on the 7 x 7 neighbourhood, read at the centre
    for (y, x) in [(3 + (H - 7) // 3, 3 + (W - 7) // 4)]:
        yy, xx = np.meshgrid(np.arange(y - 3, y + 4), np.arange(x - 3, x + 4), indexing="ij")
        nb = oracle.amap_pixels(hb, T, B, cR, delta, yy.ravel().astype(np.int32),
                                xx.ravel().astype(np.int32)).reshape(7, 7)
        s_ref = float(oracle.blur(nb, 1.0)[3, 3])
        s_got = float(score[y, x].item())
        assert abs(s_got - s_ref) <= 1e-5 * abs(s_ref) + 1e-7 * max(np.abs(ref).max(), 1e-30), \
            f"{what}: score at ({y}, {x}) {s_got} vs {s_ref}"


def run_batch(ctx, prm, images, T, B, check, seed):
    jobs = []
    for i, X in enumerate(images):
        H, W = X.shape[1:]
        m = q.qfca_fit_pca(ctx, prm, X)
        jobs.append((m, X, torch.empty((H, W), device="cuda"),
                     torch.empty((X.shape[0], H, W), dtype=torch.uint8, device="cuda"),
                     torch.empty((H, W), device="cuda")))
    torch.cuda.synchronize()
    say(f"  batch of {len(jobs)} images, {sum(j[1].shape[1] * j[1].shape[2] for j in jobs)} pixels")
    q.qfca_score_batch(ctx, jobs)
    torch.cuda.synchronize()
    assert q.qfca_batch_error(ctx) == 0
    rng = np.random.Generator(np.random.PCG64(seed))
    for i in check:
        m, X, score, bins, amap = jobs[i]
        say(f"  image {i}: {X.shape[1]}x{X.shape[2]}")
        assert torch.isfinite(score).all()
        check_image(ctx, m, X, score, bins, amap, T, B, rng, f"image {i}")
    return jobs


def test_batch_64_uneven_images_full_size(ctx):
    say("[full batch] 64 images, C=256, k=32 BF16, B=32, T=15")
    imgs, p = qfca_synth.workload_batch_torch(n=64, device="cuda")
    prm = q.Params.make(C=p["C"], k=p["k"], B=p["B"], T=p["T"], q_lo=p["q_lo"], q_hi=p["q_hi"],
                        sigma_s=p["sigma_s"], proj_prec=q.QFCA_PREC_BF16)
    sides = [X.shape[1] for X, _, _ in imgs]
    check = sorted({sides.index(s) for s in set(sides)})  # one image of every side
    run_batch(ctx, prm, [X for X, _, _ in imgs], p["T"], p["B"], check, 64)


def test_batch_large_maps_full_size(ctx):
    C, k, B, T = 512, 64, 64, 31
    say(f"[full batch] 8 maps of 1024x1024 and 32 of 256x256, C={C}, k={k} BF16, B={B}, T={T}")
    prm = q.Params.make(C=C, k=k, B=B, T=T, proj_prec=q.QFCA_PREC_BF16)
    images = []
    for i in range(8):
        X, _, _ = qfca_synth.make_texture_torch(
            C, 1024, 1024, 600 + i, "cuda",
            anomalies=[("shift", 16, 96), ("scale", 16, 96), ("permute", 16, 96), ("shift", 16, 96),
                       ("scale", 16, 96)])
        images.append(X)
    for i in range(32):
        X, _, _ = qfca_synth.make_texture_torch(C, 256, 256, 700 + i, "cuda", anomalies=[("shift", 8, 32)])
        images.append(X)
    run_batch(ctx, prm, images, T, B, [0, 7, 8, 39], 31)
