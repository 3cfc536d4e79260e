"""Pins of the GMRES / GMRES-IR oracle against mathematics and the paper.

None of these retypes the oracle's formulas: each checks a property that a
correct GMRES(m) with CGS2 and Givens least squares must have (dense LU
agreement, the Arnoldi relation, orthogonality, minimal residual by brute
force, finite termination), a special case that reduces to another algorithm
(GMRES-IR with an fp64 inner solve is restarted GMRES(m)), or a behaviour the
paper reports (IR counts are multiples of m; fp32-only GMRES stalls).
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import linalg as L
from paper_2109_01232_amd import problems as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense_csr(Ad):
    import scipy.sparse as sp

    S = sp.csr_matrix(Ad)
    S.sort_indices()
    return P.CSR(Ad.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


def random_system(n, seed, shift=None):
    rng = np.random.default_rng(seed)
    Ad = rng.standard_normal((n, n)) / np.sqrt(n)
    Ad += (shift if shift is not None else 2.0) * np.eye(n)
    return dense_csr(Ad), Ad, rng.standard_normal(n)


@pytest.mark.parametrize("n,seed", [(8, 0), (20, 1), (40, 2), (64, 3)])
def test_matches_dense_lu_and_terminates_in_n_steps(n, seed):
    A, Ad, b = random_system(n, seed)
    res = L.gmres(A, b, m=n, rtol=1e-12, check_mode=1)
    assert res.status == L.OK
    assert res.iters <= n
    xlu = np.linalg.solve(Ad, b)
    assert np.linalg.norm(res.x - xlu) / np.linalg.norm(xlu) <= 1e-10
    # a nonsymmetric, poorly conditioned one: still exact within n steps
    A2, Ad2, b2 = random_system(n, seed + 100, shift=0.3)
    res2 = L.gmres(A2, b2, m=n, rtol=1e-13, check_mode=1)
    x2 = np.linalg.solve(Ad2, b2)
    assert res2.iters <= n
    assert np.linalg.norm(Ad2 @ res2.x - b2) / np.linalg.norm(b2) <= 1e-12
    assert np.linalg.norm(res2.x - x2) / np.linalg.norm(x2) <= 1e-8


def test_arnoldi_relation_and_orthogonality():
    """A V_k = V_{k+1} Hbar_k to 1e-12 and ||I - V^T V|| <= 1e-12 with fp64 CGS2."""
    s = P.parity_system()
    M = L.csr_matrix(s.A, np.float64)
    cyc = L.gmres_cycle(lambda v: L.spmv(M, v), s.b, 50, np.float64)
    k = cyc.k
    assert k == 50
    V = cyc.V[:, : k + 1]
    AV = np.column_stack([L.spmv(M, V[:, j]) for j in range(k)])
    rel = np.linalg.norm(AV - V @ cyc.Hbar) / np.linalg.norm(cyc.Hbar)
    assert rel <= 1e-12
    assert np.linalg.norm(np.eye(k + 1) - V.T @ V) <= 1e-12
    # Hbar is upper Hessenberg with a positive subdiagonal
    assert np.all(np.tril(cyc.Hbar, -2) == 0)
    assert np.all(np.diag(cyc.Hbar, -1) > 0)


def test_minimal_residual_brute_force():
    """|g_{j+1}| equals min ||r - A z|| over the Krylov space K_j(A, r) (QR least squares)."""
    A, Ad, b = random_system(30, 7, shift=1.0)
    M = L.csr_matrix(A, np.float64)
    cyc = L.gmres_cycle(lambda v: L.spmv(M, v), b, 8, np.float64)
    gamma = np.linalg.norm(b)
    basis = []
    v = b / gamma
    for j in range(1, 9):
        basis.append(v)
        K = np.column_stack(basis)  # span{b, Ab, ..., A^{j-1} b}, columns scaled
        Q, _ = np.linalg.qr(Ad @ K)
        resid = b - Q @ (Q.T @ b)
        brute = np.linalg.norm(resid) / gamma
        assert abs(cyc.hist[j - 1] - brute) <= 1e-10 * max(brute, 1e-300) + 1e-14
        v = Ad @ v
        v = v / np.linalg.norm(v)


def test_residuals_nonincreasing_within_cycle():
    s = P.parity_system()
    M = L.csr_matrix(s.A, np.float64)
    cyc = L.gmres_cycle(lambda v: L.spmv(M, v), s.b, 40, np.float64)
    h = np.array(cyc.hist)
    assert np.all(np.diff(h) <= 1e-15)
    # explicit residual of every intermediate iterate x_j = V_j y_j, also non-increasing
    from oracle.linalg import back_substitute

    prev = np.inf
    beta = np.linalg.norm(s.b)
    for j in range(1, cyc.k + 1, 3):
        sub = L.gmres_cycle(lambda v: L.spmv(M, v), s.b, j, np.float64)
        x = sub.V[:, :j] @ sub.y
        rel = np.linalg.norm(s.b - L.spmv(M, x)) / beta
        assert rel <= prev * (1 + 1e-12) + 1e-14
        assert rel == pytest.approx(sub.hist[-1], rel=1e-8, abs=1e-13)
        prev = rel


def test_ir_with_fp64_inner_is_restarted_gmres():
    """Algorithm 2 with an fp64 inner GMRES(m) and one cycle per refinement is GMRES(m)."""
    s = P.parity_system()
    ref = L.gmres(s.A, s.b, m=30, rtol=1e-10, check_mode=0)
    ir = L.gmres_ir(s.A, s.b, m=30, rtol=1e-10, inner="fp64", check_mode=0)
    assert ref.status == ir.status == L.OK
    assert ref.iters == ir.iters and ref.refinements == ir.refinements
    assert np.linalg.norm(ref.x - ir.x) / np.linalg.norm(ref.x) <= 1e-12
    # same cycle histories; rounding noise in r_i grows as ||r_i|| / ||b|| shrinks
    a, b = np.array(ref.hist), np.array(ir.hist)
    assert np.allclose(a[:90], b[:90], rtol=1e-12)
    assert np.allclose(a, b, rtol=1e-5)


def test_paper_mode_iteration_counts_are_multiples_of_m():
    with open(os.path.join(GOLD, "paper_ir_iterations.json")) as f:
        g = json.load(f)
    # the reading (checks only at restarts) is what the paper's printed counts show
    assert all(c["ir_iters"] % c["m"] == 0 for c in g["cases"])
    assert any(c["double_iters"] % c["m"] != 0 for c in g["cases"])
    s = P.parity_system()
    for m in (25, 50):
        ir = L.gmres_ir(s.A, s.b, m=m, rtol=1e-10, inner="fp32", check_mode=0)
        assert ir.status == L.OK and ir.iters % m == 0
        cm1 = L.gmres_ir(s.A, s.b, m=m, rtol=1e-10, inner="fp32", check_mode=1)
        assert cm1.status == L.OK and cm1.iters <= ir.iters and cm1.rel_resid <= 1e-10
        assert ir.iters - cm1.iters <= m - 1


def test_fp32_only_stalls_and_ir_reaches_fp64_accuracy():
    """fp32 GMRES floors near 1e-6 (Section 'Convergence and Kernel Speedup'); IR reaches 1e-10."""
    s = P.parity_system()
    _, outer = L.gmres_single(s.A, s.b, m=50, max_iters=3000)
    floor = min(outer)
    assert 1e-8 <= floor <= 1e-4
    ir = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32")
    assert ir.status == L.OK and ir.rel_resid <= 1e-10
    ref = L.gmres(s.A, s.b, m=50, rtol=1e-10)
    # the IR curve follows the fp64 one: same number of restarts within one cycle
    assert abs(ir.refinements - ref.refinements) <= 1
    assert np.linalg.norm(ir.x - s.u) / np.linalg.norm(s.u) <= 1e-6


def test_bf16_basis_converges():
    s = P.parity_system()
    r = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", basis="bf16")
    assert r.status == L.OK and r.rel_resid <= 1e-10


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    vals = [rng.standard_normal(2000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 2000)]
    # exact ties at the rounding point (bit pattern ...8000) in both parities
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x00018000, 0x7F7F8000], dtype=np.uint32).view(np.float32)
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-40, -3e-39, 3.4e38, 1.0, -1.0],
                       dtype=np.float32)
    x = np.concatenate(vals + [ties, special])
    ours = L.to_bf16_bits(x)
    theirs = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    nan = np.isnan(x)
    assert np.array_equal(ours[~nan], theirs[~nan])
    assert np.all(np.isnan(L.round_bf16(x[nan])))


def test_failure_modes():
    s = P.parity_system()
    b = s.b.copy()
    b[5] = np.nan
    assert L.gmres_ir(s.A, b, m=20).status == L.ERR_NUMERIC
    r = L.gmres_ir(s.A, s.b, m=20, max_iters=40)
    assert r.status == L.NOT_CONVERGED and r.iters == 40
    assert r.rel_resid < 1.0
    r = L.gmres_ir(s.A, s.b, m=50, rtol=1e-20, max_iters=4000)
    assert r.status == L.STAGNATED and r.rel_resid <= 1e-12
    z = L.gmres_ir(s.A, np.zeros(s.A.n), m=10)
    assert z.status == L.OK and not np.any(z.x)


def test_resume_equals_single_call():
    """A restart's whole state is x (Algorithm 1's restart), so stopping and resuming is exact."""
    s = P.parity_system()
    full = L.gmres(s.A, s.b, m=30, rtol=1e-10, check_mode=0)
    part = L.gmres(s.A, s.b, m=30, rtol=1e-10, check_mode=0, max_iters=90)
    assert part.status == L.NOT_CONVERGED and part.iters == 90
    rest = L.gmres(s.A, s.b, x0=part.x, m=30, rtol=1e-10, check_mode=0)
    assert part.iters + rest.iters == full.iters
    assert np.array_equal(rest.x, full.x)


def test_inner_cap_restarts_in_inner_precision():
    s = P.parity_system()
    one = L.gmres_ir(s.A, s.b, m=25, rtol=1e-10, inner="fp32", cap=25)
    two = L.gmres_ir(s.A, s.b, m=25, rtol=1e-10, inner="fp32", cap=75)
    assert one.status == two.status == L.OK
    assert two.refinements < one.refinements
    assert len(two.cycle_starts) > two.refinements  # several inner cycles per refinement
