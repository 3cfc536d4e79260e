"""Pins of the GMRES-FD oracle (Section "Mixed Precision GMRES-FD").

GMRES-FD runs GMRES(m) in single precision up to a switch point, then GMRES(m)
in double precision from the single-precision solution.  Pinned by: the
switch at 0 reduces to plain fp64 GMRES(m); the single phase equals an
independently written fp32 GMRES(m) (``gmres_single``, restarted from its own
fp32 residual) bit for bit when ||b|| is a power of two, since the oracle's
scaling by 1 / ||b|| is then exact; dense LU on a tiny system; convergence to
the tolerance with the iteration counts of both phases adding up.
"""
import numpy as np
import pytest

from oracle import linalg as L
from paper_2109_01232_amd import problems as P


def test_switch_zero_is_fp64_gmres():
    s = P.parity_system()
    fd = L.gmres_fd(s.A, s.b, 0, m=50, rtol=1e-10)
    ref = L.gmres(s.A, s.b, m=50, rtol=1e-10)
    assert fd.status == ref.status == L.OK
    assert fd.iters == ref.iters
    assert np.array_equal(fd.x, ref.x)


@pytest.mark.parametrize("switch", [50, 100])
def test_single_phase_equals_independent_fp32_gmres(switch):
    """b with 16 entries of +-1 has ||b|| = 4 exactly: the scaled fp32 solve
    is the unscaled one times 1/4, exactly, at every step."""
    s = P.parity_system()
    rng = np.random.default_rng(7)
    b = np.zeros(s.A.n)
    idx = rng.choice(s.A.n, 16, replace=False)
    b[idx] = rng.choice([-1.0, 1.0], 16)
    assert float(np.linalg.norm(b)) == 4.0
    fd = L.gmres_fd(s.A, b, switch, m=50, rtol=1e-10, max_iters=switch)
    assert fd.status == L.NOT_CONVERGED and fd.iters == switch
    x32, outer = L.gmres_single(s.A, b, m=50, rtol=0.0, max_iters=switch)
    assert np.array_equal(fd.x, x32.astype(np.float64))
    assert fd.outer[-1] == pytest.approx(outer[-1], rel=1e-12)


def test_tiny_system_matches_dense_lu():
    rng = np.random.default_rng(3)
    n = 30
    Ad = rng.standard_normal((n, n)) / np.sqrt(n) + 2.0 * np.eye(n)
    import scipy.sparse as sp

    S = sp.csr_matrix(Ad)
    A = P.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))
    b = rng.standard_normal(n)
    fd = L.gmres_fd(A, b, n, m=n, rtol=1e-12, check_mode=1)
    assert fd.status == L.OK
    xlu = np.linalg.solve(Ad, b)
    assert np.linalg.norm(fd.x - xlu) / np.linalg.norm(xlu) <= 1e-10
    # outer: the start, then the residual at the switch -- the full-length
    # single phase stops at fp32 accuracy, not below
    assert fd.outer[0] == 1.0
    assert 1e-9 < fd.outer[1] < 1e-4


def test_converges_and_counts_both_phases():
    s = P.parity_system()
    fd = L.gmres_fd(s.A, s.b, 100, m=50, rtol=1e-10, check_mode=1)
    assert fd.status == L.OK
    assert fd.rel_resid <= 1e-10
    assert fd.iters == len(fd.hist)
    assert fd.iters > 100
    # the double phase starts from the single phase's iterate
    single = fd.xs[0]
    r = s.b - L.spmv(L.csr_matrix(s.A, np.float64), single)
    assert fd.outer[1] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(s.b), rel=1e-12)
    assert fd.outer[2] == fd.outer[1]
    assert np.linalg.norm(fd.x - s.u) / np.linalg.norm(s.u) < 1e-6


def test_switch_beyond_budget_stops_in_single_phase():
    s = P.parity_system()
    fd = L.gmres_fd(s.A, s.b, 100, m=50, rtol=1e-10, max_iters=60)
    assert fd.status == L.NOT_CONVERGED
    assert fd.iters == 60
