"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/qfca.h declares, and the host eigensolver agrees with LAPACK."""
import os
import re

import numpy as np
import pytest

import paper_2510_15602_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "qfca.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qfca_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(q.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = q.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert L.qfca_version() >= 100
    assert L.qfca_status_str(2) == b"invalid shape"


def test_params_struct_layout():
    import ctypes
    assert ctypes.sizeof(q.Params) == 44


@pytest.mark.parametrize("n", [1, 2, 5, 33, 128])
def test_host_eigensolver_matches_eigh(n):
    g = np.random.Generator(np.random.PCG64(n))
    M = g.standard_normal((n, 2 * n + 3))
    A = M @ M.T / M.shape[1]
    ev, V = q.host_sym_eig(A)
    w, U = np.linalg.eigh(A)
    np.testing.assert_allclose(ev, w[::-1], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(A @ V, V * ev, atol=1e-11)
    assert np.all(np.diff(ev) <= 0)


def test_host_eigensolver_degenerate_spectrum():
    A = np.diag([3.0, 3.0, 1.0, 1.0, 1.0]) + 0.0
    ev, V = q.host_sym_eig(A)
    np.testing.assert_allclose(ev, [3, 3, 1, 1, 1], atol=1e-14)
    np.testing.assert_allclose(V.T @ V, np.eye(5), atol=1e-14)


def test_oracle_library_builds_and_is_separate():
    import oracle
    assert os.path.exists(oracle.build(force=False))
    # the product package never imports the oracle
    src = open(os.path.join(ROOT, "paper_2510_15602_amd", "__init__.py")).read()
    assert "import oracle" not in src


def test_model_serialisation_rejects_bad_arguments_without_a_gpu():
    """Argument checks of qfca_model_export / qfca_model_import run before
    any device call."""
    import ctypes
    L = q.lib()
    n = ctypes.c_size_t(0)
    assert L.qfca_model_export(None, None, ctypes.byref(n)) == 1
    h = ctypes.c_void_p()
    blob = ctypes.create_string_buffer(b"QFCAMDL\0" + bytes(64))
    assert L.qfca_model_import(None, blob, 72, ctypes.byref(h)) == 1
    assert not h.value


def _spectra():
    g = np.random.Generator(np.random.PCG64(17))
    n = 96
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    M = g.standard_normal((n, 3 * n))
    R = g.standard_normal((n, 10))
    return {
        "wishart": (M @ M.T / M.shape[1], 24),
        "rank 10 < k": (R @ R.T, 24),
        "equal leading eigenvalues": ((Q * np.r_[[5.0] * 4, [3.0] * 6, np.linspace(2, 0.1, n - 10)]) @ Q.T, 24),
        "cluster across k": ((Q * np.r_[[5.0] * 30, np.linspace(2, 0.1, n - 30)]) @ Q.T, 24),
        "near-null tail": ((Q * np.r_[np.linspace(5, 4, 8), [1e-9] * (n - 8)]) @ Q.T, 24),
        "zero matrix": (np.zeros((6, 6)), 3),
    }


@pytest.mark.parametrize("name", list(_spectra()))
def test_host_top_k_eigensolver_against_eigh(name):
    """The fit's eigensolver: all eigenvalues, and k orthonormal vectors that
    are eigenvectors (A v = lambda v) of the k largest, on spectra with equal
    eigenvalues, clusters across k and rank below k."""
    A, k = _spectra()[name]
    ev, V = q.host_sym_eig_top(A, k)
    w = np.linalg.eigvalsh(A)[::-1]
    sc = max(np.abs(w).max(), 1.0)
    np.testing.assert_allclose(ev, w, atol=1e-12 * sc)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(A @ V, V * ev[:k], atol=1e-11 * sc)
    # the sign convention of the full solver: largest-magnitude entry positive
    assert np.all(V[np.abs(V).argmax(axis=0), np.arange(k)] > 0)


def test_host_full_eigensolver_rank_deficient():
    """A covariance of rank below its size (fewer pixels than channels): the
    cluster of zero eigenvalues must deflate (QL tested against the matrix
    norm as well as the neighbouring diagonal)."""
    g = np.random.Generator(np.random.PCG64(3))
    R = g.standard_normal((128, 12))
    A = R @ R.T
    ev, V = q.host_sym_eig(A)
    w = np.linalg.eigvalsh(A)[::-1]
    np.testing.assert_allclose(ev, w, atol=1e-12 * w[0])
    np.testing.assert_allclose(V.T @ V, np.eye(128), atol=1e-12)
    np.testing.assert_allclose(A @ V, V * ev, atol=1e-11 * w[0])
