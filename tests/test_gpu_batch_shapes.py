"""Every shape the persistent batch kernel is instantiated for (odd T from 3
to 31, each channel/component padding and precision) and the paper's own
operating point (C = 512, k = 10, B = 16, T = 9 and 13; Sec. 4.5.1, 4.5.2,
4.4) through qfca_score_batch and the server, against the single-image path
(bit for bit) and the FP64 oracle on the batch's own bins and model."""
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
    assert not bad.any(), f"{what}: {bad.sum()} outside tolerance, worst {(np.abs(g - o) - tol).max():.3e}"


# (C, k, B, precision): one per channel/component padding of the batch kernel
# (FP32 (64, 1), (256, 2), (512, 4); BF16 (256, 2), (512, 4)), C and k chosen
# below the padding so that padded channels and components are exercised
PADDINGS = [(50, 10, 16, q.QFCA_PREC_FP32), (200, 20, 32, q.QFCA_PREC_FP32), (300, 40, 64, q.QFCA_PREC_FP32),
            (160, 24, 32, q.QFCA_PREC_BF16), (512, 10, 16, q.QFCA_PREC_BF16)]
TS = list(range(3, 32, 2))


def run_and_check(ctx, C, k, B, T, prec, shapes, seed, with_chan=True):
    prm = q.Params.make(C=C, k=k, B=B, T=T, proj_prec=prec)
    items = []
    for i, (H, W) in enumerate(shapes):
        t = qfca_synth.make_texture(C, H, W, seed + i, anomalies=[("shift", 3, max(3, min(H, W) // 4))])
        X = torch.from_numpy(t.X).cuda()
        m = q.qfca_fit_pca(ctx, prm, X)
        f = dict(device="cuda")
        items.append((m, X, torch.empty((H, W), **f), torch.empty((C, H, W), dtype=torch.uint8, **f),
                      torch.empty((H, W), **f), torch.empty((C, H, W), **f) if with_chan else None))
    q.qfca_score_batch(ctx, [it if with_chan else it[:5] for it in items])
    torch.cuda.synchronize()
    assert q.qfca_batch_error(ctx) == 0
    for (m, X, score, bins, amap, achan) in items:
        b1, _ = q.qfca_quantize(ctx, m, X)
        o1 = q.qfca_score_map(ctx, m, b1, amap=True)
        torch.cuda.synchronize()
        assert torch.equal(bins, b1), "batch bins differ from qfca_quantize"
        assert torch.equal(amap, o1.amap) and torch.equal(score, o1.score), "batch differs from qfca_score_map"
        ref = oracle.score(bins.cpu().numpy(), T, B, m.read("cR"), m.read("delta"), 1.0, want_chan=with_chan)
        if with_chan:
            close(achan.cpu().numpy(), ref.Achan, "per-channel maps")
        close(amap.cpu().numpy(), ref.A, "channel mean")
        close(score.cpu().numpy(), ref.score, "score")
    return items


@pytest.mark.parametrize("T", TS)
@pytest.mark.parametrize("pad", PADDINGS, ids=lambda p: f"C{p[0]}_k{p[1]}_B{p[2]}_p{p[3]}")
def test_every_batch_instantiation(ctx, pad, T):
    C, k, B, prec = pad
    shapes = [(T + 6, T + 11), (2 * T + 3, T + 2)]
    say(f"[batch shape] T={T} C={C} k={k} B={B} prec={prec} shapes={shapes}")
    run_and_check(ctx, C, k, B, T, prec, shapes, 1000 + T)


@pytest.mark.parametrize("T", [9, 13])
@pytest.mark.parametrize("prec", [q.QFCA_PREC_FP32, q.QFCA_PREC_BF16], ids=["fp32", "bf16"])
def test_paper_operating_point_batch(ctx, prec, T):
    """C = 512 (WideResNet-50 layer 2), k = 10, B = 16, T = 9 and 13, three
    images of uneven size in one batch."""
    say(f"[paper point] C=512 k=10 B=16 T={T} prec={prec}")
    run_and_check(ctx, 512, 10, 16, T, prec, [(64, 64), (40, 90), (96, 72)], 2000 + T, with_chan=False)


@pytest.mark.parametrize("T", [9, 13])
def test_paper_operating_point_served(ctx, T):
    """The same point through the continuous-batching server: each served map
    equals the image's batch result alone and the oracle's."""
    C, k, B = 512, 10, 16
    prm = q.Params.make(C=C, k=k, B=B, T=T, proj_prec=q.QFCA_PREC_BF16)
    X0, _, _ = qfca_synth.make_texture_torch(C, 96, 96, 3000, "cuda", class_seed=3000)
    m = q.qfca_fit_pca(ctx, prm, X0)
    reqs = []
    for i, (H, W) in enumerate([(64, 64), (48, 80), (96, 96), (33, 57)]):
        X, _, _ = qfca_synth.make_texture_torch(C, H, W, 3100 + i, "cuda", anomalies=[("shift", 8, 12)],
                                                class_seed=3000)
        reqs.append((X, torch.full((H, W), float("nan"), device="cuda")))
    torch.cuda.synchronize()
    say(f"[paper point served] T={T}, {len(reqs)} requests")
    srv = q.Server(0, hbm_budget=1 << 30, max_inflight=2, max_batch=4)
    for X, s in reqs:
        srv.submit(m, X, s)
    srv.drain()
    done = srv.poll()
    srv.close()
    assert len(done) == len(reqs) and all(c["status"] == 0 for c in done)
    for X, s in reqs:
        alone = torch.empty_like(s)
        q.qfca_score_batch(ctx, [(m, X, alone)])
        bins, _ = q.qfca_quantize(ctx, m, X)
        torch.cuda.synchronize()
        assert torch.equal(s, alone)
        ref = oracle.score(bins.cpu().numpy(), T, B, m.read("cR"), m.read("delta"), 1.0)
        close(s.cpu().numpy(), ref.score, "served score")
