"""Pins of the chooser features on matrices whose features are known in closed form."""
import numpy as np
import pytest

from oracle import features as F
from paper_2109_01232_amd import problems as P


def diag_csr(d):
    n = len(d)
    return P.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.asarray(d, float))


def test_scaled_identity():
    A = diag_csr(np.full(100, 3.0))
    f = F.features(A, np.ones(100))
    assert f[0] == pytest.approx(2.0)
    assert f[1] == 1 and f[2] == 1
    assert f[3] == 1 and f[4] == 1 and f[5] == 1
    assert f[6] == pytest.approx(1.0)
    assert f[7] == pytest.approx(np.log10(3.0))
    assert f[8] == 0 and f[9] == 0
    # one Arnoldi step: exact breakdown, residual 0 (floored), Ritz value 3
    assert f[10] == pytest.approx(-30) and f[11] == pytest.approx(-30)
    assert f[12] == pytest.approx(0.0, abs=1e-6) and f[13] == 0
    assert f[14] == pytest.approx(1.0) and f[15] == pytest.approx(0.0, abs=1e-6)


def test_laplacian_row_stats():
    n = 20
    A = P.conv_diff(2, n, 0.0, (1.0, 1.0))
    f = F.features(A, np.ones(A.n))
    N = n * n
    # interior rows have d = S = 4 -> fraction 1/2; boundary rows have fewer neighbours
    n_int = (n - 2) ** 2
    n_edge = 4 * (n - 2)
    n_corner = 4
    frac = (n_int * 0.5 + n_edge * 4 / 7 + n_corner * 4 / 6) / N
    assert f[3] == pytest.approx(frac)
    assert f[4] == pytest.approx(0.5)
    assert f[5] == 1.0
    rowsum = (n_edge * 1 + n_corner * 2) / N
    assert f[6] == pytest.approx(rowsum / 4.0)
    assert f[8] == 0.0
    # |U_i - L_i| / S_i: 0 in the interior, 1/3 on edges, 1 on two corners, 0 on the other two
    assert f[9] == pytest.approx((n_edge / 3.0 + 2.0) / N)
    assert f[2] == 5 and f[1] == pytest.approx(A.nnz / N)
    # symmetric positive definite: real Ritz values inside (0, 8)
    assert f[13] == pytest.approx(0.0, abs=1e-6)
    assert f[14] > 0


def test_convection_raises_asymmetry_feature():
    a = F.row_features(P.conv_diff(2, 20, 0.0, (1.0, 1.0)))
    b = F.row_features(P.conv_diff(2, 20, 150.0, (1.0, 1.0)))
    assert b[9] > a[9] + 0.1
