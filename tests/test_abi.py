"""The C ABI library loads, exports every declared symbol, and its host-side
logic (no GPU needed) agrees with independent references."""
import ctypes

import numpy as np
import pytest

from oracle import poly as PO
from paper_2109_01232_amd import binding as B


def test_library_exports_every_declared_function():
    lib = B.lib()
    names = B.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.gmresir_abi_version() == 4


def test_status_strings_and_errors():
    for st in (0, 1, 2, 3, -1, -2, -3, -4, -5):
        assert len(B.status_string(st)) >= 2 and B.status_string(st) != "unknown status"
    assert B.status_string(12345) == "unknown status"
    res = B.Result()
    p = B.make_params()
    # NULL matrix: rejected before any GPU call
    st = B.lib().gmresir_solve(None, None, None, ctypes.byref(p), None, None, 0, ctypes.byref(res), None, 0, None)
    assert st == B.ERR_INVALID_ARG
    assert "NULL" in B.last_error()
    assert B.lib().gmresir_workspace_bytes(None, ctypes.byref(p)) == 0


def test_storage_bytes():
    L = B.lib()
    assert L.gmresir_matrix_storage_bytes(0, 0) == 0
    assert L.gmresir_matrix_storage_bytes(10, -1) == 0
    assert L.gmresir_matrix_storage_bytes(10, 1 << 31) == 0
    n, nnz = 1_000_000, 4_996_000
    s = L.gmresir_matrix_storage_bytes(n, nnz)
    assert s >= 4 * nnz + 4 * (n // 512)
    assert s % 256 == 0


def random_hessenberg(n, seed):
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((n, n)), -1)
    return H


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (11, 4), (41, 5), (101, 6)])
def test_hessenberg_eigenvalues_match_lapack(n, seed):
    H = random_hessenberg(n, seed)
    ours = B.gmresir_host_hessenberg_eigvals(H)
    ref = np.linalg.eigvals(H)
    # match each eigenvalue to its nearest reference
    for z in ours:
        d = np.min(np.abs(ref - z))
        assert d <= 1e-9 * max(1.0, np.abs(ref).max()), (z, d)
    assert np.allclose(np.sort_complex(ours), np.sort_complex(ref), atol=1e-9 * max(1, np.abs(ref).max()))
    # conjugate pairs come out adjacent and exact
    i = 0
    while i < n:
        if ours[i].imag != 0:
            assert ours[i + 1] == np.conj(ours[i])
            i += 2
        else:
            i += 1


def test_hessenberg_special_matrices():
    # rotation block: eigenvalues +-i; a Jordan-like shift; diagonal
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    z = B.gmresir_host_hessenberg_eigvals(R)
    assert np.allclose(sorted(z.imag), [-1, 1]) and np.allclose(z.real, 0)
    D = np.diag([3.0, -1.0, 2.0, 7.0])
    assert np.allclose(sorted(B.gmresir_host_hessenberg_eigvals(D).real), [-1, 2, 3, 7])
    C = np.zeros((6, 6))  # companion-like cyclic shift: 6th roots of unity
    for i in range(1, 6):
        C[i, i - 1] = 1.0
    C[0, 5] = 1.0
    z = B.gmresir_host_hessenberg_eigvals(C)
    assert np.allclose(np.abs(z), 1.0, atol=1e-10)


@pytest.mark.parametrize("k,seed", [(2, 0), (5, 1), (11, 2), (21, 3), (41, 4)])
def test_harmonic_ritz_leja_matches_oracle(k, seed):
    """Library (own QR + Leja) vs oracle (LAPACK eigvals + its own Leja)."""
    from oracle import linalg as L
    from paper_2109_01232_amd import problems as P

    A = P.conv_diff(2, 12, 30.0, (1.0, 0.3))
    M = L.csr_matrix(A, np.float64)
    cyc = L.gmres_cycle(lambda v: L.spmv(M, v), PO.start_vector(A.n, seed), k, np.float64)
    assert cyc.k == k
    ours = B.gmresir_host_harmonic_ritz_leja(cyc.Hbar)
    ref = PO.leja_order(PO.harmonic_ritz(cyc.Hbar))
    scale = np.abs(ref).max()
    assert np.allclose(np.sort_complex(ours), np.sort_complex(ref), atol=1e-9 * scale)
    assert abs(ours[0]) == pytest.approx(np.abs(ref).max(), rel=1e-12)
    # same Leja order unless two candidates tie to rounding
    assert np.allclose(ours, ref, atol=1e-8 * scale)


def test_leja_property_of_library_order():
    rng = np.random.default_rng(9)
    H = np.triu(rng.standard_normal((16, 15)), -1)
    H[np.arange(1, 16), np.arange(15)] = np.abs(H[np.arange(1, 16), np.arange(15)]) + 0.1
    out = B.gmresir_host_harmonic_ritz_leja(H)
    assert len(out) == 15
    for i in range(1, len(out)):
        if out[i].imag < 0:
            assert out[i] == np.conj(out[i - 1])
            continue
        chosen = out[:i]
        score = lambda t: np.sum(np.log(np.abs(t - chosen)))
        assert score(out[i]) >= max(score(t) for t in out[i:] if t.imag >= 0) - 1e-9
