"""GPU parity of fp64 GMRES(m) with an fp32 polynomial preconditioner
(Section "Preconditioning": an fp32 M applied to fp64 vectors), through the
C ABI, against the oracle's same mode.  Roots come from the oracle and are
passed to both sides.  Bars, at a parity tolerance rtol = 1e-12: final fp64
relative residual <= 1e-12 on both sides; solutions within 1e-8 relative; the
first cycle's implicit history within 1e-5 (the fp32 polynomial is evaluated
as fused product-form steps on the GPU, step by step in the oracle: rounding
differs at the fp32 level; measured history gaps 1.2e-8 (d = 10) and 1.6e-7
(d = 40), solution gaps 3e-12 and 3e-16).  And the paper's observation on both
sides, at rtol = 1e-10: the first cycle's implicit residual meets the target
while the explicit residual of its iterate stays above 1e-8, so restarts are
needed."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import linalg as L
from oracle import poly as PO
from paper_2109_01232_amd import binding as B
from paper_2109_01232_amd import problems as P

from gpu_common import dev_tensor, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


def _laplace3d(n):
    A = P.stencil_matrix("laplace3d_7", n)
    u = np.random.default_rng(0).uniform(-1, 1, A.n)
    return A, A.scipy() @ u, u


@pytest.mark.parametrize("d", [10, 40])
def test_fp32_poly_in_fp64_gmres_matches_oracle(d):
    A, bnp, u = _laplace3d(12)
    roots = PO.poly_roots(A, d, seed=12345)
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bnp)
    say("fp64 gmres + fp32 poly", d)
    x, dres, h = B.solve(M, b, restart=50, inner="fp64", rtol=1e-12, check_mode=1, poly_degree=d,
                         poly_prec="fp32", poly_roots=roots, hist_cap=10000)
    ref = L.gmres_ir(A, bnp, m=50, rtol=1e-12, inner="fp64", poly_roots=roots, poly_prec="fp32", check_mode=1)
    xs = x.cpu().numpy()
    assert dres["status"] == B.OK and ref.status == L.OK
    true = np.linalg.norm(bnp - A.scipy() @ xs) / np.linalg.norm(bnp)
    assert true <= 1e-12 and ref.rel_resid <= 1e-12
    assert rel(xs, ref.x) <= 1e-8
    assert dres["iters"] == ref.iters
    assert dres["refinements"] >= 2
    say("fp64 gmres + fp32 poly at 1e-10", d)
    x, dres, h = B.solve(M, b, restart=50, inner="fp64", rtol=1e-10, check_mode=1, poly_degree=d,
                         poly_prec="fp32", poly_roots=roots, hist_cap=10000)
    ref = L.gmres_ir(A, bnp, m=50, rtol=1e-10, inner="fp64", poly_roots=roots, poly_prec="fp32", check_mode=1)
    # first cycle: ends where the implicit residual first meets the target
    k1 = int(np.argmax(h <= 1e-10)) + 1
    assert h[k1 - 1] <= 1e-10
    href = np.array(ref.hist[: ref.cycle_starts[1]])
    n1 = min(k1, len(href))
    assert np.max(np.abs(h[:n1] - href[:n1])) <= 1e-5
    # the same first cycle alone: its explicit residual stays far above the target
    say("fp64 gmres + fp32 poly, first cycle", d, k1)
    x1, d1, _ = B.solve(M, b, restart=50, inner="fp64", rtol=1e-10, check_mode=1, poly_degree=d,
                        poly_prec="fp32", poly_roots=roots, max_iters=k1)
    assert d1["status"] == B.NOT_CONVERGED and d1["iters"] == k1
    assert d1["rel_resid_true"] >= 1e-8 and ref.outer[1] >= 1e-8
    # with the polynomial in fp64 the first cycle's explicit residual meets the target
    say("fp64 gmres + fp64 poly", d)
    x2, d2, _ = B.solve(M, b, restart=50, inner="fp64", rtol=1e-10, check_mode=1, poly_degree=d,
                        poly_roots=roots)
    assert d2["status"] == B.OK and d2["refinements"] == 1
    M.close()


def test_poly_prec_argument():
    A, bnp, _ = _laplace3d(8)
    M = B.Matrix.from_csr(A)
    say("poly_prec argument")
    assert B.gmresir_workspace_bytes(M, B.make_params(inner="fp64", poly_degree=5, poly_prec="bf16")) == 0
    # with an fp32 inner solve the polynomial is fp32 already: same bits as the default
    roots = PO.poly_roots(A, 5, seed=3)
    b = dev_tensor(bnp)
    xa, da, ha = B.solve(M, b, restart=30, inner="fp32", rtol=1e-10, poly_degree=5, poly_roots=roots, hist_cap=500)
    xb, db, hb = B.solve(M, b, restart=30, inner="fp32", rtol=1e-10, poly_degree=5, poly_prec="fp32",
                         poly_roots=roots, hist_cap=500)
    assert torch.equal(xa, xb) and np.array_equal(ha, hb)
    M.close()


def test_fp32_poly_full_size_converges():
    """3D anisotropic 150^3 system, fp64 GMRES(100) with an fp32 polynomial
    of degree 20 built on the GPU: reaches 1e-10 (checked on the host)."""
    s = P.aniso3d_system(0)
    M = B.Matrix.from_csr(s.A)
    b = dev_tensor(s.b)
    say("aniso3d 150^3 fp64 + fp32 poly 20")
    roots = B.gmresir_poly_setup(M, 20, seed=12345)
    x, d, _ = B.solve(M, b, restart=100, inner="fp64", rtol=1e-10, check_mode=1, poly_degree=20,
                      poly_prec="fp32", poly_roots=roots)
    xs = x.cpu().numpy()
    assert d["status"] == B.OK
    assert np.linalg.norm(s.b - s.A.scipy() @ xs) / np.linalg.norm(s.b) <= 1e-10
    M.close()
