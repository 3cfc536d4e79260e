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


# ----------------------------------------------------------------------------
# Arnoldi features (10-15) on a matrix with seven known eigenvalues
# ----------------------------------------------------------------------------
#
# A = 5 I + 4 P with P the cyclic shift of 7 elements, in 16 identical
# diagonal blocks (N = 112), and b = the first unit vector of every block
# (||b|| = 4).  The eigenvalues are 5 + 4 w^k with w^k the seventh roots of
# unity.  Every Arnoldi step is exact in fp32 (values are multiples of 1/4):
# v_j is the j-th unit vector of every block, H is 5 on the diagonal and 4 on
# the subdiagonal, and step 7 breaks down exactly (A v_7 = 5 v_7 + 4 v_1).
# So the Ritz values of the 7 x 7 Hessenberg matrix are the seven
# eigenvalues, features 12-15 have closed forms, the implicit residual after
# step 7 is exactly 0 (feature 11 at its floor), and the residual after j < 7
# steps is that of the bidiagonal least-squares problem, whose residual is
# along the null vector z of H^T, z_i = (-5/4)^i: rho_j = 1 / sqrt(sum_{i<=j} (25/16)^i).

BLOCK, COPIES = 7, 16
CENTRE, RADIUS = 5.0, 4.0


def cyclic_system():
    import scipy.sparse as sp

    Pm = np.roll(np.eye(BLOCK), 1, axis=0)  # P e_i = e_{i+1}, P e_7 = e_1
    blk = CENTRE * np.eye(BLOCK) + RADIUS * Pm
    S = sp.block_diag([blk] * COPIES, format="csr")
    S.eliminate_zeros()
    S.sort_indices()
    A = P.CSR(S.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))
    rhs = np.zeros(A.n)
    rhs[::BLOCK] = 1.0
    return A, S.toarray(), rhs


def rho_closed(j):
    return 1.0 / np.sqrt(sum((25.0 / 16.0) ** i for i in range(j + 1)))


def brute_krylov_residual(Ad, b, j):
    """min ||b - A z|| / ||b|| over z in span{b, A b, ..., A^{j-1} b} (fp64 QR least squares)."""
    K = [b / np.linalg.norm(b)]
    for _ in range(j - 1):
        v = Ad @ K[-1]
        K.append(v / np.linalg.norm(v))
    Q, _ = np.linalg.qr(Ad @ np.column_stack(K))
    return np.linalg.norm(b - Q @ (Q.T @ b)) / np.linalg.norm(b)


def test_cyclic_closed_forms_agree_with_brute_force():
    A, Ad, b = cyclic_system()
    for j in range(1, BLOCK):
        assert brute_krylov_residual(Ad, b, j) == pytest.approx(rho_closed(j), rel=1e-12)
    assert brute_krylov_residual(Ad, b, BLOCK) <= 1e-12
    lam = np.linalg.eigvals(Ad)
    ks = np.arange(BLOCK)
    want = CENTRE + RADIUS * np.exp(2j * np.pi * ks / BLOCK)
    for w in want:
        assert np.abs(lam - w).min() <= 1e-12


def arnoldi_feature_pins(Fmod):
    """Names of the failed pins of features 10-15 for an oracle.features-like module."""
    failed = []
    A, Ad, b = cyclic_system()
    try:
        f = Fmod.features(A, b)
    except Exception:
        return ["features (exception)"]
    th = 2 * np.pi * np.arange(BLOCK) / BLOCK
    lam = CENTRE + RADIUS * np.exp(1j * th)
    amax, amin = np.abs(lam).max(), np.abs(lam).min()  # 9 and |5 + 4 exp(6 pi i / 7)|
    D = CENTRE
    if abs(f[10] - np.log10(rho_closed(5))) > 1e-4:
        failed.append("f10 = log10 rho_5")
    if f[11] != -30.0:
        failed.append("f11 = log10 rho_7 = floor (exact breakdown)")
    if abs(f[12] - np.log10(amax / amin)) > 1e-5:
        failed.append("f12 modulus spread")
    if abs(f[13] - np.abs(lam.imag).max() / amax) > 1e-5:
        failed.append("f13 imaginary part")
    if abs(f[14] - lam.real.min() / amax) > 1e-5:
        failed.append("f14 leftmost real part")
    if abs(f[15] - np.log10(amax / D)) > 1e-5:
        failed.append("f15 modulus over diagonal")
    return failed


def test_arnoldi_features_seven_eigenvalues():
    assert arnoldi_feature_pins(F) == []


def test_arnoldi_breaks_down_at_seven_steps():
    from oracle import linalg as L

    A, Ad, b = cyclic_system()
    M = L.csr_matrix(A, np.float32)
    cyc = L.gmres_cycle(lambda z: L.spmv(M, z), b.astype(np.float32), 10, np.float32)
    assert cyc.k == BLOCK and cyc.breakdown
    for j in range(1, BLOCK):
        assert cyc.hist[j - 1] == pytest.approx(rho_closed(j), rel=1e-6)
    assert cyc.hist[BLOCK - 1] == 0.0


def test_row_features_cyclic_system():
    A, Ad, b = cyclic_system()
    f = F.features(A, b)
    assert f[1] == 2 and f[2] == 2
    assert f[3] == pytest.approx(5 / 9) and f[4] == pytest.approx(5 / 9) and f[5] == 1.0
    assert f[6] == pytest.approx(9 / 5)
    assert f[7] == pytest.approx(np.log10(np.sqrt(41.0)))
    assert f[8] == 0.0
    assert f[9] == pytest.approx(1.0)  # one off-diagonal per row: |U - L| / S = 1


FEATURE_MUTATIONS = [
    ("f10 and f11 swapped", "f[0] = _log10(hist[min(5, k) - 1])\n    f[1] = _log10(hist[k - 1])",
     "f[0] = _log10(hist[k - 1])\n    f[1] = _log10(hist[min(5, k) - 1])"),
    ("f10 one step late", "f[0] = _log10(hist[min(5, k) - 1])", "f[0] = _log10(hist[min(5, k)])"),
    ("f10 one step early", "f[0] = _log10(hist[min(5, k) - 1])", "f[0] = _log10(hist[min(5, k) - 2])"),
    ("f11 one step early", "f[1] = _log10(hist[k - 1])", "f[1] = _log10(hist[k - 2])"),
    ("f12 min and max swapped", "f[2] = _log10(amax / max(amin, TINY))", "f[2] = _log10(amin / max(amax, TINY))"),
    ("f13 real part instead of imaginary", "f[3] = np.abs(theta.imag).max()", "f[3] = np.abs(theta.real).max()"),
    ("f14 rightmost instead of leftmost", "f[4] = theta.real.min()", "f[4] = theta.real.max()"),
    ("f15 smallest modulus", "f[5] = _log10(amax / max(D, TINY))", "f[5] = _log10(amin / max(D, TINY))"),
    ("Ritz values of a shifted block of Hbar",
     "theta = np.linalg.eigvals(cyc.Hbar[:k, :k].astype(np.float64))",
     "theta = np.linalg.eigvals(cyc.Hbar[1:k + 1, :k].astype(np.float64))"),
]


@pytest.mark.parametrize("name,old,new", FEATURE_MUTATIONS, ids=[m[0] for m in FEATURE_MUTATIONS])
def test_feature_mutation_is_caught(name, old, new):
    from test_oracle_mutations import mutant

    m = mutant(F, old, new)
    assert arnoldi_feature_pins(m) != [], name
