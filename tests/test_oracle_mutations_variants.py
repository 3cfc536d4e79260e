"""Planted mistakes in the oracle's GMRES-FD, block-Jacobi and fp32-polynomial
modes must be caught by their pins (same method as the core mutation test:
copy the module source, apply one mistake, run the pins on the mutant)."""
import numpy as np
import pytest

import oracle.linalg as L_orig
from oracle import poly as PO
from paper_2109_01232_amd import problems as P

from test_oracle_mutations import mutant


def _tiny_dense(n=40, seed=4):
    rng = np.random.default_rng(seed)
    Ad = rng.standard_normal((n, n)) / np.sqrt(n) + 3.0 * np.eye(n)
    import scipy.sparse as sp

    S = sp.csr_matrix(Ad)
    return P.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)), Ad, \
        rng.standard_normal(n)


def variant_pins(L):
    failed = []
    s = P.parity_system()
    # GMRES-FD
    try:
        fd = L.gmres_fd(s.A, s.b, 0, m=50, rtol=1e-10)
        ref = L.gmres(s.A, s.b, m=50, rtol=1e-10)
        if not (fd.iters == ref.iters and np.array_equal(fd.x, ref.x)):
            failed.append("fd switch 0")
        rng = np.random.default_rng(7)
        b = np.zeros(s.A.n)
        b[rng.choice(s.A.n, 16, replace=False)] = rng.choice([-1.0, 1.0], 16)
        fd = L.gmres_fd(s.A, b, 100, m=50, rtol=1e-10, max_iters=100)
        x32, _ = L.gmres_single(s.A, b, m=50, rtol=0.0, max_iters=100)
        if not (fd.iters == 100 and np.array_equal(fd.x, x32.astype(np.float64))):
            failed.append("fd single phase")
        fd = L.gmres_fd(s.A, s.b, 100, m=50, rtol=1e-10, check_mode=1)
        if not (fd.status == 0 and fd.rel_resid <= 1e-10 and fd.outer[2] == fd.outer[1]
                and fd.iters == len(fd.hist) and fd.iters > 100):
            failed.append("fd double phase")
    except Exception:
        failed.append("fd (exception)")
    # block Jacobi
    try:
        from test_oracle_bj import varied_diagonal_system

        Aj, d = varied_diagonal_system()
        inv = L.block_jacobi_inverses(Aj, 1, np.float32)
        v = np.random.default_rng(0).standard_normal(Aj.n).astype(np.float32)
        if not np.array_equal(L.block_jacobi_apply(inv, v, np.float32),
                              (np.float32(1.0) / d.astype(np.float32)) * v):
            failed.append("bj jacobi fp32")
        S = s.A.scipy().tocsr()
        inv = L.block_jacobi_inverses(s.A, 16, np.float64)
        v = np.random.default_rng(1).standard_normal(s.A.n)
        y = L.block_jacobi_apply(inv, v, np.float64)
        blk = S[16:32, 16:32].toarray()
        if not (len(inv) == 256 and np.abs(blk @ y[16:32] - v[16:32]).max() <= 1e-12 * np.abs(v[16:32]).max()):
            failed.append("bj blocks")
        A, Ad, b = _tiny_dense()
        r = L.gmres_ir(A, b, m=20, rtol=1e-12, inner="fp32", bj_block=A.n, check_mode=1)
        if not (r.status == 0 and r.iters <= 2 * r.refinements):
            failed.append("bj one block")
    except Exception:
        failed.append("bj (exception)")
    # fp32 polynomial in fp64 GMRES
    try:
        A = P.stencil_matrix("laplace3d_7", 12)
        b = A.scipy() @ np.random.default_rng(0).uniform(-1, 1, A.n)
        roots = PO.poly_roots(A, 40, seed=12345)
        mix = L.gmres_ir(A, b, m=50, rtol=1e-10, inner="fp64", poly_roots=roots, poly_prec="fp32", check_mode=1)
        if not (mix.hist[mix.cycle_starts[1] - 1] <= 1e-10 and mix.outer[1] >= 1e-8 and mix.status == 0):
            failed.append("poly32 gap")
    except Exception:
        failed.append("poly32 (exception)")
    return failed


def test_unmodified_oracle_passes():
    assert variant_pins(L_orig) == []


MUTATIONS = [
    ("fd: double phase from zero", "double = gmres(A, b, x0=x,", "double = gmres(A, b, x0=None,"),
    ("fd: iterations of the single phase not counted", "total.iters += double.iters",
     "total.iters = double.iters"),
    ("fd: single phase in fp64", 'single = gmres_ir(A, b, m=m, rtol=rtol, inner="fp32"',
     'single = gmres_ir(A, b, m=m, rtol=rtol, inner="fp64"'),
    ("bj: fp32 inverses computed in fp64 and rounded", "S = csr_matrix(A, dtype)\n    out = []",
     "S = csr_matrix(A, np.float64)\n    out = []"),
    ("bj: transposed inverse", "y[r0:r0 + k] = Bi.astype(dtype, copy=False) @ v[r0:r0 + k]",
     "y[r0:r0 + k] = Bi.T.astype(dtype) @ v[r0:r0 + k]"),
    # (An inner solve given fp64 inverses rounded to fp32 instead of fp32 ones is
    # not listed: the two preconditioners differ only at fp32 rounding level, so
    # the solves differ at that level too; the fp32 computation itself is pinned
    # bitwise at the function level by "bj jacobi fp32".)
    ("bj: overlapping blocks", "r1 = min(A.n, r0 + bs)", "r1 = min(A.n, r0 + bs + 1)"),
    ("poly32: polynomial left in fp64", 'if poly_prec == "fp32" and wp == np.float64:', "if False:"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_variant_mutation_is_caught(name, old, new):
    m = mutant(L_orig, old, new)
    assert variant_pins(m) != [], name
