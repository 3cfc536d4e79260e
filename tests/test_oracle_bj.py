"""Pins of the oracle's block-Jacobi preconditioner (right preconditioning
inside GMRES-IR; blocks of consecutive rows, inverses in fp64 rounded to fp32).

Block size 1 is Jacobi (division by the diagonal); every block inverse
times its block is the identity; one block covering the whole matrix makes
M^{-1} the fp32-rounded inverse of A, so every inner cycle reaches fp32
accuracy in a step or two; on the convection-diffusion parity system the
preconditioner cuts the iteration count."""
import numpy as np
import pytest

from oracle import linalg as L
from paper_2109_01232_amd import problems as P


def test_block_size_one_is_jacobi():
    A = P.conv_diff(3, 9, 10.0, (1, 1, 1), (1, 1, 1e-2))  # diagonal 4.02: 1/d is rounded in fp32
    inv = L.block_jacobi_inverses(A, 1)
    d = A.scipy().diagonal()
    v = np.random.default_rng(0).standard_normal(A.n)
    y = L.block_jacobi_apply(inv, v, np.float64)
    assert np.array_equal(y, (1.0 / d).astype(np.float32).astype(np.float64) * v)


@pytest.mark.parametrize("bs", [7, 16, 42, 64])
def test_inverses_invert_the_diagonal_blocks(bs):
    s = P.parity_system()
    S = s.A.scipy().tocsr()
    inv = L.block_jacobi_inverses(s.A, bs)
    assert len(inv) == -(-s.A.n // bs)
    r0 = 0
    for Bi in inv:
        k = Bi.shape[0]
        blk = S[r0:r0 + k, r0:r0 + k].toarray()
        assert np.abs(Bi @ blk - np.eye(k)).max() <= 1e-12
        r0 += k
    assert r0 == s.A.n


def test_one_block_is_the_inverse():
    rng = np.random.default_rng(4)
    n = 40
    Ad = rng.standard_normal((n, n)) / np.sqrt(n) + 3.0 * np.eye(n)
    import scipy.sparse as sp

    S = sp.csr_matrix(Ad)
    A = P.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))
    b = rng.standard_normal(n)
    res = L.gmres_ir(A, b, m=20, rtol=1e-12, inner="fp32", bj_block=n, check_mode=1)
    assert res.status == L.OK
    assert np.linalg.norm(res.x - np.linalg.solve(Ad, b)) / np.linalg.norm(res.x) <= 1e-10
    # A M^{-1} = I + O(u_fp32): each inner cycle stops after at most two steps
    assert res.iters <= 2 * res.refinements


def test_block_jacobi_reduces_iterations():
    s = P.parity_system()
    plain = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", check_mode=1)
    bj = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", bj_block=32, check_mode=1)
    assert plain.status == bj.status == L.OK
    assert bj.rel_resid <= 1e-10
    assert bj.iters < plain.iters
