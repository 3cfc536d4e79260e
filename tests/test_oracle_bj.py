"""Pins of the oracle's block-Jacobi preconditioner (right preconditioning,
blocks of consecutive rows, inverses computed and applied in the inner
precision: Section "Preconditioning", case (b), computes and applies the fp32
preconditioner of GMRES-IR entirely in fp32).

Block size 1 is Jacobi: in fp32 the inverse is the correctly rounded fp32
quotient 1 / fl32(a_ii) (one IEEE division), which differs from the fp64
quotient rounded to fp32 on some rows of a matrix with a varied diagonal;
every block inverse times its block is the identity to the precision's
accuracy; one block covering the whole matrix makes M^{-1} the inverse of A
to fp32 accuracy, so every inner cycle stops in a step or two; on the
convection-diffusion parity system the preconditioner cuts the iteration
count."""
import numpy as np
import pytest

from oracle import linalg as L
from paper_2109_01232_amd import problems as P


def varied_diagonal_system(n=2000, seed=0):
    """A tridiagonal matrix whose diagonal entries are random (so that 1 / d
    rounds differently in fp32 and fp64 on some rows)."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    d = rng.uniform(3.0, 7.0, n)
    S = sp.diags([np.full(n - 1, -1.0), d, np.full(n - 1, -1.3)], [-1, 0, 1], format="csr")
    S.sort_indices()
    return P.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)), d


def test_block_size_one_is_jacobi_fp32():
    A, d = varied_diagonal_system()
    inv = L.block_jacobi_inverses(A, 1, np.float32)
    assert all(Bi.dtype == np.float32 for Bi in inv)
    v = np.random.default_rng(0).standard_normal(A.n).astype(np.float32)
    y = L.block_jacobi_apply(inv, v, np.float32)
    d32 = d.astype(np.float32)
    want = (np.float32(1.0) / d32) * v  # fp32 division and product, each correctly rounded
    assert np.array_equal(y, want)
    # the fp32 computation is not the fp64 one rounded afterwards on every row
    assert np.any((np.float32(1.0) / d32) != (1.0 / d).astype(np.float32))


def test_block_size_one_is_jacobi_fp64():
    A, d = varied_diagonal_system()
    inv = L.block_jacobi_inverses(A, 1, np.float64)
    v = np.random.default_rng(1).standard_normal(A.n)
    assert np.array_equal(L.block_jacobi_apply(inv, v, np.float64), (1.0 / d) * v)


@pytest.mark.parametrize("bs", [7, 16, 42, 64])
@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 2e-6)])
def test_inverses_invert_the_diagonal_blocks(bs, dtype, tol):
    s = P.parity_system()
    S = s.A.scipy().tocsr()
    inv = L.block_jacobi_inverses(s.A, bs, dtype)
    assert len(inv) == -(-s.A.n // bs)
    r0 = 0
    for Bi in inv:
        k = Bi.shape[0]
        assert Bi.dtype == dtype
        blk = S[r0:r0 + k, r0:r0 + k].toarray()
        assert np.abs(Bi.astype(np.float64) @ blk - np.eye(k)).max() <= tol
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
