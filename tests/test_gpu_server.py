"""The continuous-batching server (qfca_server_*): every request's score map is
bitwise the one the image gets alone, under memory pressure and with
launches overlapping on the device."""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2510_15602_amd as q  # noqa: E402
import qfca_synth  # noqa: E402

C, K, B, T = 256, 32, 32, 15


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return q.Context(0)


@pytest.fixture(scope="module")
def models(ctx):
    """Three texture classes, each fitted on an anomaly-free exemplar (BF16 projection)."""
    prm = q.Params.make(C=C, k=K, B=B, T=T, proj_prec=q.QFCA_PREC_BF16)
    out = []
    for cls in range(3):
        X, _, _ = qfca_synth.make_texture_torch(C, 96, 96, 400 + cls, "cuda", class_seed=400 + cls)
        out.append(q.qfca_fit_pca(ctx, prm, X))
    torch.cuda.synchronize()
    return out


def requests(n, seed, sides=(40, 64, 96, 128)):
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for i in range(n):
        cls = int(rng.integers(0, 3))
        H, W = int(rng.choice(sides)), int(rng.choice(sides))
        X, _, _ = qfca_synth.make_texture_torch(C, H, W, 5000 + seed * 100 + i, "cuda",
                                                anomalies=[("shift", 4, 12)], class_seed=400 + cls)
        reqs.append((cls, X, torch.full((H, W), float("nan"), device="cuda")))
    torch.cuda.synchronize()
    return reqs


def alone(ctx, models, reqs):
    outs = []
    for cls, X, _ in reqs:
        s = torch.empty(X.shape[1:], device="cuda")
        q.qfca_score_batch(ctx, [(models[cls], X, s)])
        outs.append(s)
    torch.cuda.synchronize()
    return outs


def serve(srv, models, reqs, gap_s=0.0):
    tickets = {}
    for i, (cls, X, s) in enumerate(reqs):
        tickets[srv.submit(models[cls], X, s)] = i
        if gap_s:
            time.sleep(gap_s)
    srv.drain()
    done = srv.poll()
    assert sorted(c["ticket"] for c in done) == sorted(tickets)
    assert all(c["status"] == 0 for c in done)
    torch.cuda.synchronize()
    return done


def test_server_results_equal_alone(ctx, models):
    say("[server] 24 requests, 2 slots, staggered arrivals")
    reqs = requests(24, 1)
    ref = alone(ctx, models, reqs)
    srv = q.Server(0, hbm_budget=2 << 30, max_inflight=2, max_batch=8)
    done = serve(srv, models, reqs, gap_s=0.002)
    st = srv.stats()
    say(f"  stats {st}")
    lat = sorted(c["t_done"] - c["t_submit"] for c in done)
    say(f"  latency p50 {1e3 * lat[len(lat) // 2]:.2f} ms, max {1e3 * lat[-1]:.2f} ms")
    for i, (_, _, s) in enumerate(reqs):
        assert torch.equal(s, ref[i]), f"request {i} differs from its result alone"
    assert st["completed"] == st["submitted"] == 24 and st["failed"] == 0
    srv.close()
    # served maps against the FP64 oracle on the request's bins (those of
    # qfca_quantize with the class model, which the batch reproduces bit for bit)
    for i in range(0, 24, 5):
        cls, X, s = reqs[i]
        m = models[cls]
        bins, _ = q.qfca_quantize(ctx, m, X)
        torch.cuda.synchronize()
        ref_o = oracle.score(bins.cpu().numpy(), T, B, m.read("cR"), m.read("delta"), 1.0)
        g = s.cpu().numpy().astype(np.float64)
        tol = 1e-5 * np.abs(ref_o.score) + 1e-7 * np.abs(ref_o.score).max()
        assert (np.abs(g - ref_o.score) <= tol).all(), f"request {i}: served score against the oracle"


def test_server_memory_budget_defers_and_completes(ctx, models):
    reqs = requests(12, 2, sides=(128,))
    need = q_bytes(128, 128)
    budget = 2 * need + 1000  # two requests at a time
    say(f"[server] budget {budget} bytes ({need} per request)")
    ref = alone(ctx, models, reqs)
    srv = q.Server(0, hbm_budget=budget, max_inflight=3, max_batch=8)
    serve(srv, models, reqs)
    st = srv.stats()
    say(f"  stats {st}")
    assert st["deferred_memory"] >= 1
    assert st["arena_peak"] <= st["arena_bytes"] and st["arena_peak"] <= 2 * need
    assert st["max_batch_seen"] <= 2
    for i, (_, _, s) in enumerate(reqs):
        assert torch.equal(s, ref[i])
    srv.close()


def test_server_launches_overlap(ctx, models):
    """A launch issued on one slot while the other slot's launch runs is on
    the device at the same time (its interval meets the other's).  The first
    launch of each slot does one-time set-up (staging buffers, graph
    capture) that waits for the device, so a warm-up burst comes first."""
    reqs = requests(16, 3, sides=(128,))
    ref = alone(ctx, models, reqs)
    srv = q.Server(0, hbm_budget=4 << 30, max_inflight=2, max_batch=4)
    serve(srv, models, reqs)  # warm-up: both slots set up
    st0 = srv.stats()
    for _, _, s in reqs:
        s.fill_(float("nan"))
    serve(srv, models, reqs)
    st = srv.stats()
    say(f"[server overlap] {st}")
    assert st0["max_inflight_seen"] == 2
    assert st["overlapped"] - st0["overlapped"] >= 2
    assert st["device_busy_s"] <= st["device_span_s"] + 1e-9
    for i, (_, _, s) in enumerate(reqs):
        assert torch.equal(s, ref[i])
    srv.close()


def test_server_rejects_bad_requests(ctx, models):
    srv = q.Server(0, hbm_budget=1 << 20, max_inflight=1, max_batch=4)
    X = torch.zeros((C, 128, 128), device="cuda")
    s = torch.empty((128, 128), device="cuda")
    with pytest.raises(q.QfcaError) as e:
        srv.submit(models[0], X, s)  # 128x128 needs ~4.3 MB
    assert e.value.status == 3
    with pytest.raises(ValueError):
        srv.submit(models[0], X, torch.empty((64, 64), device="cuda"))
    assert srv.stats()["submitted"] == 0
    srv.close()
    with pytest.raises(q.QfcaError):
        q.Server(0, hbm_budget=1 << 20, max_inflight=0)


def q_bytes(H, W):
    def a(x):
        return (x + 255) // 256 * 256
    N = H * W
    return a(C * N) + a(8 * N)
