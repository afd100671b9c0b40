"""Model serialisation: a fitted model exported to host bytes and imported
again quantises and scores bit for bit like the original, and malformed
buffers are refused."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2510_15602_amd as q  # noqa: E402
import qfca_synth  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return q.Context(0)


@pytest.mark.parametrize("prec", [q.QFCA_PREC_FP32, q.QFCA_PREC_BF16], ids=["fp32", "bf16"])
def test_export_import_round_trip(ctx, prec):
    C, H, W = 256, 96, 80
    say(f"[model io] C={C} {H}x{W} prec={prec}")
    X, _, _ = qfca_synth.make_texture_torch(C, H, W, 77, "cuda", anomalies=[("shift", 6, 20)])
    prm = q.Params.make(C=C, k=32, B=32, T=15, proj_prec=prec)
    m = q.qfca_fit_pca(ctx, prm, X)
    blob = q.qfca_model_export(m)
    m2 = q.qfca_model_import(ctx, blob)
    for f in ("mu", "V", "edges", "delta", "cR", "evals", "lo", "hi"):
        np.testing.assert_array_equal(m.read(f), m2.read(f), err_msg=f)
    assert q.qfca_model_export(m2) == blob
    b1, _ = q.qfca_quantize(ctx, m, X)
    b2, _ = q.qfca_quantize(ctx, m2, X)
    s1 = q.qfca_score_map(ctx, m, b1, amap=True)
    s2 = q.qfca_score_map(ctx, m2, b2, amap=True)
    torch.cuda.synchronize()
    assert torch.equal(b1, b2)
    assert torch.equal(s1.score, s2.score) and torch.equal(s1.amap, s2.amap)


def test_import_refuses_malformed_buffers(ctx):
    C, H, W = 8, 20, 20
    X = torch.from_numpy(np.random.Generator(np.random.PCG64(5)).standard_normal((C, H, W)).astype(np.float32)).cuda()
    m = q.qfca_fit_pca(ctx, q.Params.make(C=C, k=2, B=8, T=5), X)
    blob = q.qfca_model_export(m)
    for bad in (blob[:-1], blob + b"\0", b"XXXXXXXX" + blob[8:]):
        with pytest.raises(q.QfcaError) as err:
            q.qfca_model_import(ctx, bad)
        assert err.value.status == 1
    wrong_version = blob[:8] + (99).to_bytes(4, "little") + blob[12:]
    with pytest.raises(q.QfcaError) as err:
        q.qfca_model_import(ctx, wrong_version)
    assert err.value.status == 7
    bad_T = bytearray(blob)
    bad_T[16 + 12:16 + 16] = (4).to_bytes(4, "little")  # an even window
    with pytest.raises(q.QfcaError) as err:
        q.qfca_model_import(ctx, bytes(bad_T))
    assert err.value.status == 7
