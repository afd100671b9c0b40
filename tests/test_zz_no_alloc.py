"""qfca_score_map_noalloc (no device allocation, fixed library scratch)
against qfca_score_map: bit for bit, on two calls in a row, the second with
a smaller map, and the size limit refused before any launch."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import paper_2510_15602_amd as q  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return q.Context(0)


def problem(seed, C, H, W, T, B):
    g = np.random.Generator(np.random.PCG64(seed))
    R = g.standard_normal((C, H, W))
    _, _, delta, e = oracle.edges(R, B)
    bins = oracle.quantize(R, B, e)
    cR = oracle.reference_cdf(bins, T, B).astype(np.int32)
    return bins, delta, e, cR


def maps(H, W, C, with_all):
    f = dict(device="cuda", dtype=torch.float32)
    out = q.ScoreMaps(torch.full((H, W), float("nan"), **f))
    if with_all:
        out.amap = torch.full((H, W), float("nan"), **f)
        out.w1 = torch.full((H, W), float("nan"), **f)
        out.achan = torch.full((C, H, W), float("nan"), **f)
    return out


@pytest.mark.parametrize("with_all", [False, True], ids=["score", "all_maps"])
def test_noalloc_equals_score_map(ctx, with_all):
    C, T, B = 6, 15, 32
    # the second call is smaller: the scratch keeps the first call's sums,
    # which the call must clear
    for (H, W, seed) in [(300, 257, 1), (97, 130, 2)]:
        say(f"[no-alloc] C={C} H={H} W={W} T={T} B={B} all_maps={with_all}")
        bins, delta, e, cR = problem(seed, C, H, W, T, B)
        prm = q.Params.make(C=C, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE)
        m = q.qfca_model_create(ctx, prm, None, None, e, delta, cR)
        bd = torch.from_numpy(bins).cuda()
        ref = q.qfca_score_map(ctx, m, bd, amap=with_all, w1=with_all, achan=with_all)
        got = q.qfca_score_map_noalloc(ctx, m, bd, maps(H, W, C, with_all))
        torch.cuda.synchronize()
        for f in ("score", "amap", "w1", "achan"):
            a, b = getattr(ref, f), getattr(got, f)
            assert (a is None) == (b is None)
            if a is not None:
                assert torch.equal(a, b), f"{f} differs from qfca_score_map ({H}x{W})"


def test_noalloc_refuses_maps_above_its_limit(ctx):
    C, T, B = 1, 3, 4
    H, W = 2049, 2048  # one row more than 2048 x 2048
    bins = torch.zeros((C, H, W), dtype=torch.uint8, device="cuda")
    cR = np.array([[9, 9, 9, 9]], np.int32)
    prm = q.Params.make(C=C, k=0, B=B, T=T, preproc=q.QFCA_PRE_NONE)
    m = q.qfca_model_create(ctx, prm, None, None, np.array([[0.5, 1.0, 1.5]], np.float32),
                            np.array([0.5]), cR)
    with pytest.raises(q.QfcaError) as err:
        q.qfca_score_map_noalloc(ctx, m, bins, maps(H, W, C, False))
    assert err.value.status == 7
