"""Pins of the oracle's one-reduction CGS2 cycle (``gmres_cycle_lowsync``:
CGS2 with the second pass and the normalisation delayed by one iteration,
the DCGS2 Arnoldi of Bielich et al., Parallel Computing 2022).

In exact arithmetic it produces the same basis and Hessenberg matrix as the
two-pass CGS2 of Section "GMRES", so it is held to what pins any GMRES
cycle: the Arnoldi relation and the orthogonality of the basis (fp64, 1e-12),
the minimal residual over the Krylov space by brute force (QR least squares),
dense LU on tiny systems, termination in at most N steps, non-increasing
residuals; in fp32 its loss of orthogonality stays at the level of fp32 CGS2;
GMRES-IR with it converges to the same solution."""
import numpy as np
import pytest

import oracle.linalg as L_orig
from paper_2109_01232_amd import problems as P

from test_oracle_mutations import dense_system, mutant


def lowsync_pins(L):
    failed = []
    # brute force: |g_{j+1}| = min ||r - A z|| over K_j
    try:
        A, Ad, b = dense_system(30, 7, shift=1.0)
        M = L.csr_matrix(A, np.float64)
        cyc = L.gmres_cycle_lowsync(lambda v: L.spmv(M, v), b, 8, np.float64)
        gamma = np.linalg.norm(b)
        basis, v = [], b / gamma
        for j in range(1, 9):
            basis.append(v)
            Q, _ = np.linalg.qr(Ad @ np.column_stack(basis))
            brute = np.linalg.norm(b - Q @ (Q.T @ b)) / gamma
            if abs(cyc.hist[j - 1] - brute) > 1e-10 * brute + 1e-14:
                failed.append(f"brute force step {j}")
                break
            v = Ad @ v
            v = v / np.linalg.norm(v)
    except Exception:
        failed.append("brute force (exception)")
    # dense LU and termination
    try:
        A, Ad, b = dense_system()
        r = L.gmres(A, b, m=A.n, rtol=1e-12, check_mode=1, ortho="dcgs2")
        x = np.linalg.solve(Ad, b)
        if not (r.status == 0 and np.linalg.norm(r.x - x) / np.linalg.norm(x) <= 1e-10 and r.iters <= A.n):
            failed.append("dense LU")
    except Exception:
        failed.append("dense LU (exception)")
    # Arnoldi relation, orthogonality, monotone residuals (parity system, fp64)
    s = P.parity_system()
    M = L.csr_matrix(s.A, np.float64)
    try:
        cyc = L.gmres_cycle_lowsync(lambda v: L.spmv(M, v), s.b, 40, np.float64)
        V = cyc.V[:, : cyc.k + 1]
        AV = np.column_stack([L.spmv(M, V[:, j]) for j in range(cyc.k)])
        if cyc.k != 40 or np.linalg.norm(AV - V @ cyc.Hbar) / np.linalg.norm(cyc.Hbar) > 1e-12:
            failed.append("Arnoldi relation")
        if np.linalg.norm(np.eye(cyc.k + 1) - V.T @ V) > 1e-12:
            failed.append("orthogonality")
        if np.any(np.diff(cyc.hist) > 1e-15):
            failed.append("monotone residual")
        x = cyc.V[:, : cyc.k] @ cyc.y
        if abs(np.linalg.norm(s.b - L.spmv(M, x)) / np.linalg.norm(s.b) - cyc.hist[-1]) > 1e-8 * cyc.hist[-1]:
            failed.append("explicit = implicit residual")
    except Exception:
        failed.append("cycle (exception)")
    # exact breakdown: n = 12 < m
    try:
        A = P.conv_diff(2, 3, 5.0, (1.0, 0.0))
        b = np.arange(1.0, A.n + 1)
        cyc = L.gmres_cycle_lowsync(lambda v: L.spmv(L.csr_matrix(A, np.float64), v), b, 30, np.float64)
        if not (cyc.breakdown and cyc.k <= A.n and cyc.hist[-1] <= 1e-12):
            failed.append("termination in <= N steps")
    except Exception:
        failed.append("breakdown (exception)")
    # GMRES-IR with fp32 inner cycles: same solution as with two-pass CGS2
    try:
        ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-12, inner="fp32", check_mode=1)
        low = L.gmres_ir(s.A, s.b, m=50, rtol=1e-12, inner="fp32", check_mode=1, ortho="dcgs2")
        if not (low.status == 0 and low.rel_resid <= 1e-12
                and np.linalg.norm(low.x - ref.x) / np.linalg.norm(ref.x) <= 1e-9):
            failed.append("IR solution")
    except Exception:
        failed.append("IR (exception)")
    return failed


def test_unmodified_lowsync_passes():
    assert lowsync_pins(L_orig) == []


def test_fp32_orthogonality_like_cgs2():
    s = P.parity_system()
    M32 = L_orig.csr_matrix(s.A, np.float32)
    r = s.b.astype(np.float32)
    low = L_orig.gmres_cycle_lowsync(lambda v: L_orig.spmv(M32, v), r, 50, np.float32)
    two = L_orig.gmres_cycle(lambda v: L_orig.spmv(M32, v), r, 50, np.float32)

    def loss(c):
        V = c.V[:, : c.k + 1].astype(np.float64)
        return np.linalg.norm(np.eye(c.k + 1) - V.T @ V)

    assert low.k == two.k == 50
    assert loss(low) <= max(4 * loss(two), 1e-5)
    # the fp32 histories of the two orderings agree to fp32 accuracy
    assert np.max(np.abs(np.array(low.hist) - np.array(two.hist))) <= 1e-5


def test_same_cycle_as_cgs2_in_fp64():
    s = P.parity_system()
    M = L_orig.csr_matrix(s.A, np.float64)
    a = L_orig.gmres_cycle(lambda v: L_orig.spmv(M, v), s.b, 50, np.float64)
    b = L_orig.gmres_cycle_lowsync(lambda v: L_orig.spmv(M, v), s.b, 50, np.float64)
    assert a.k == b.k
    assert np.max(np.abs(a.Hbar - b.Hbar)) <= 1e-12 * np.abs(a.Hbar).max()
    assert np.max(np.abs(np.array(a.hist) - np.array(b.hist))) <= 1e-13


def test_stop_and_restart_semantics():
    s = P.parity_system()
    r1 = L_orig.gmres(s.A, s.b, m=50, rtol=1e-10, check_mode=1)
    r2 = L_orig.gmres(s.A, s.b, m=50, rtol=1e-10, check_mode=1, ortho="dcgs2")
    assert r1.iters == r2.iters and r2.status == 0 and r2.rel_resid <= 1e-10
    r0 = L_orig.gmres(s.A, s.b, m=50, rtol=1e-10, check_mode=0, ortho="dcgs2")
    assert r0.iters % 50 == 0
    with pytest.raises(ValueError):
        L_orig.gmres_ir(s.A, s.b, inner="fp32", basis="bf16", ortho="dcgs2")


LOWSYNC_MUTATIONS = [
    ("second pass omitted", "V[:, j] = (u - Q @ a) / rho", "V[:, j] = u / rho"),
    ("Arnoldi-relation correction omitted", "u = p / rho - V[:, : j + 1] @ (t / rho + h1)",
     "u = p / rho - V[:, : j + 1] @ h1"),
    ("SpMV output not scaled by 1/rho", "u = p / rho - V[:, : j + 1] @ (t / rho + h1)",
     "u = p - V[:, : j + 1] @ (t / rho + h1)"),
    ("new coefficient not scaled twice", "h1[j] = ((gam - np.dot(a, c)) / rho - t[j]) / rho",
     "h1[j] = ((gam - np.dot(a, c)) / rho - t[j])"),
    ("rotation sign (delayed column)", "tt = cs[i] * R[i, jj] + sn[i] * R[i + 1, jj]",
     "tt = cs[i] * R[i, jj] - sn[i] * R[i + 1, jj]"),
    # (Not listed: mistakes in terms that carry the second-pass coefficients a --
    # dropping a from the Hessenberg column, rho from alpha alone, the a^T c term
    # of h1_j, a shifted or wrong-iteration t = H a.  After one Gram-Schmidt pass
    # a = Q^T u_j is zero in exact arithmetic and O(u) in floating point, so each
    # of these changes results only at rounding level and no pin can separate
    # it; what the second pass buys is the orthogonality of V, which "second pass
    # omitted" covers.  The same holds for two-pass CGS2's h2, see the core
    # mutation tests.)
]


@pytest.mark.parametrize("name,old,new", LOWSYNC_MUTATIONS, ids=[m[0] for m in LOWSYNC_MUTATIONS])
def test_lowsync_mutation_is_caught(name, old, new):
    m = mutant(L_orig, old, new)
    assert lowsync_pins(m) != [], name
