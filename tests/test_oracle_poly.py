"""Pins of the polynomial-preconditioner oracle.

Harmonic Ritz values are the roots of the GMRES residual polynomial, so the
GMRES residual after d+1 steps must equal pi(A) r0 (checked densely); the
product-form apply must equal the dense monomial evaluation of p(A); and
``I - A p(A) = pi(A)`` must hold.  The counter-based start vector is pinned
to SplitMix64's published first output.
"""
import json
import os

import numpy as np
import pytest

from oracle import linalg as L
from oracle import poly as PO
from paper_2109_01232_amd import problems as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def small(n=10, Pe=40.0):
    A = P.conv_diff(2, n, Pe, (1.0, 0.5))
    return A, A.scipy().toarray()


def test_splitmix64_published_value():
    with open(os.path.join(GOLD, "splitmix64.json")) as f:
        g = json.load(f)
    assert PO.splitmix64(g["state"]) == int(g["first_output_hex"], 16)
    v = PO.start_vector(64, 987654321)
    ref = [2.0 * ((PO.splitmix64(987654321 ^ i) >> 11) * 2.0 ** -53) - 1.0 for i in range(64)]
    assert np.array_equal(v, np.array(ref))
    assert np.all(np.abs(v) < 1.0)


@pytest.mark.parametrize("d", [1, 3, 6, 9])
def test_harmonic_ritz_values_are_gmres_residual_roots(d):
    A, Ad = small()
    r0 = PO.start_vector(A.n, 5)
    M = L.csr_matrix(A, np.float64)
    cyc = L.gmres_cycle(lambda v: L.spmv(M, v), r0, d + 1, np.float64)
    theta = PO.harmonic_ritz(cyc.Hbar)
    x = cyc.V[:, : cyc.k] @ cyc.y
    r_gmres = r0 - Ad @ x
    r_poly = (PO.residual_poly_dense(Ad, theta) @ r0)
    assert np.abs(r_poly.imag).max() <= 1e-10 * np.linalg.norm(r0)
    assert np.linalg.norm(r_gmres - r_poly.real) <= 1e-8 * np.linalg.norm(r0)


@pytest.mark.parametrize("d", [0, 1, 2, 5, 10])
def test_product_form_equals_dense_polynomial(d):
    A, Ad = small(8)
    roots = PO.poly_roots(A, d, seed=1, dtype=np.float64)
    assert len(roots) == d + 1
    v = np.random.default_rng(d).standard_normal(A.n)
    M = L.csr_matrix(A, np.float64)
    y = PO.apply_product_form(M, roots, v, np.float64)
    pd = PO.p_dense(Ad, roots)
    assert np.linalg.norm(y - pd @ v) <= 1e-10 * np.linalg.norm(pd @ v)
    # I - A p(A) = pi(A)
    pi = PO.residual_poly_dense(Ad, roots)
    assert np.linalg.norm(np.eye(A.n) - Ad @ pd - pi.real) <= 1e-9 * np.linalg.norm(pi.real) + 1e-12
    if d == 0:
        assert np.allclose(y, v / roots[0].real)


def test_leja_order_properties():
    rng = np.random.default_rng(3)
    re = rng.uniform(0.1, 5, 6)
    im = rng.uniform(0.1, 2, 3)
    theta = np.concatenate([re, im + 1j * im, im - 1j * im])
    rng.shuffle(theta)
    out = PO.leja_order(theta)
    assert sorted(map(complex, out), key=lambda z: (z.real, z.imag)) == sorted(
        map(complex, theta), key=lambda z: (z.real, z.imag))
    assert abs(out[0]) == np.abs(theta).max()
    i = 0
    while i < len(out):
        if out[i].imag != 0:
            assert out[i].imag > 0 and out[i + 1] == np.conj(out[i])
            i += 2
        else:
            i += 1
    # each next real root maximises the product of distances to the chosen ones
    for k in range(1, len(out)):
        if out[k].imag < 0:
            continue
        chosen = out[:k]
        score = lambda t: np.sum(np.log(np.abs(t - chosen)))
        rest = [t for t in out[k:] if t.imag >= 0]
        assert score(out[k]) >= max(score(t) for t in rest) - 1e-12


def test_right_preconditioned_ir_converges_with_true_residual():
    """A p(A) y = b then x = p(A) y: residuals are those of A (Section 'Preconditioning')."""
    A = P.conv_diff(3, 12, 10.0, (1, 1, 1), (1, 1, 1e-2))
    u = np.random.default_rng(0).uniform(-1, 1, A.n)
    b = A.scipy() @ u
    plain = L.gmres_ir(A, b, m=30, rtol=1e-10, inner="fp32")
    roots = PO.poly_roots(A, 10, seed=2, dtype=np.float32)
    pre = L.gmres_ir(A, b, m=30, rtol=1e-10, inner="fp32", poly_roots=roots)
    assert plain.status == pre.status == L.OK
    assert pre.rel_resid <= 1e-10
    assert pre.iters < plain.iters
    assert np.linalg.norm(b - A.scipy() @ pre.x) / np.linalg.norm(b) == pytest.approx(pre.rel_resid)


# ---------------------------------------------------------------------------
# fp32 polynomial inside fp64 GMRES (Section "Preconditioning", an fp32 M
# applied to fp64 vectors)
# ---------------------------------------------------------------------------

def _laplace3d(n):
    A = P.stencil_matrix("laplace3d_7", n)
    u = np.random.default_rng(0).uniform(-1, 1, A.n)
    return A, A.scipy() @ u


@pytest.mark.parametrize("d", [10, 40])
def test_fp32_polynomial_in_fp64_gmres(d):
    """The paper reports that with the polynomial applied in fp32 and all
    else in fp64 the implicit (Givens) residual parts from the explicit one:
    here the first cycle's implicit residual meets 1e-10 while the explicit
    residual of its iterate stays above 1e-8; with the polynomial in fp64 the
    two agree.  Restarts from the explicit residual still reach 1e-10."""
    A, b = _laplace3d(12)
    roots = PO.poly_roots(A, d, seed=12345)
    r64 = L.gmres_ir(A, b, m=50, rtol=1e-10, inner="fp64", poly_roots=roots, check_mode=1)
    assert r64.status == L.OK and r64.refinements == 1 and r64.outer[1] <= 1e-10
    mix = L.gmres_ir(A, b, m=50, rtol=1e-10, inner="fp64", poly_roots=roots, poly_prec="fp32", check_mode=1)
    first_implicit = mix.hist[mix.cycle_starts[1] - 1]
    assert first_implicit <= 1e-10
    assert mix.outer[1] >= 1e-8
    assert mix.status == L.OK and mix.rel_resid <= 1e-10 and mix.refinements >= 2


def test_fp32_polynomial_apply_is_fp32_accurate():
    A, _ = _laplace3d(10)
    roots = PO.poly_roots(A, 10, seed=1)
    v = np.random.default_rng(2).standard_normal(A.n)
    M64 = L.csr_matrix(A, np.float64)
    M32 = L.csr_matrix(A, np.float32)
    y64 = PO.apply_product_form(M64, roots, v, np.float64)
    y32 = PO.apply_product_form(M32, roots, v.astype(np.float32), np.float32).astype(np.float64)
    err = np.linalg.norm(y32 - y64) / np.linalg.norm(y64)
    assert 1e-9 < err < 1e-4
