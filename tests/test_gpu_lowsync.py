"""GPU parity of the one-reduction CGS2 cycle (ortho = 1: the second
Gram-Schmidt pass and the normalisation delayed by one iteration) through
the C ABI, against the oracle's same mode (``ortho="dcgs2"``) and against the
two-pass CGS2 path.

Bars, as for two-pass CGS2: fp64 cycle histories within 1e-10 of the
oracle's (same algorithm, rounding-level differences), fp32 cycle histories
within 1e-5, solutions within 1e-8 relative at a parity tolerance
rtol = 1e-12, final fp64 residuals <= rtol; iteration counts equal in fp64 and
within one restart cycle in fp32.  Systems of at least 65,536 rows take the
fused sliced SpMV + reduction kernel; smaller ones the plain SpMV and a
separate reduction kernel; both are covered, with ragged row counts, every
column-count class (m = 1 .. 128), and the polynomial and block-Jacobi
preconditioners."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import linalg as L
from oracle import poly as PO
from paper_2109_01232_amd import binding as B
from paper_2109_01232_amd import problems as P

from gpu_common import dev_tensor, rel, say

pytestmark = pytest.mark.gpu

HIST_TOL_FP32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


def _system(side, pe=30.0, seed=0, wind=(1.0, -0.5)):
    A = P.conv_diff(2, side, pe, wind)
    u = np.random.default_rng(seed).uniform(-1, 1, A.n)
    return A, A.scipy() @ u


def _first(ref):
    return ref.cycle_starts[1] if len(ref.cycle_starts) > 1 else len(ref.hist)


@pytest.mark.parametrize("side", [37, 64, 259])  # 1369 and 4096 rows (separate reduction), 67081 (fused)
def test_fp64_matches_oracle(side):
    A, bb = _system(side)
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    say("lowsync fp64 gmres(50)", side)
    x, d, h = B.solve(M, b, restart=50, inner="fp64", rtol=1e-12, check_mode=1, ortho="dcgs2", hist_cap=200000,
                      max_iters=20000)
    ref = L.gmres(A, bb, m=50, rtol=1e-12, check_mode=1, ortho="dcgs2", max_iters=20000)
    assert d["status"] == B.OK and ref.status == L.OK
    assert d["iters"] == ref.iters
    assert d["rel_resid_true"] <= 1e-12
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    k = min(150, len(ref.hist))
    assert np.max(np.abs(h[:k] - np.array(ref.hist[:k]))) <= 1e-10
    # the same cycles as two-pass CGS2 to rounding
    x2, d2, h2 = B.solve(M, b, restart=50, inner="fp64", rtol=1e-12, check_mode=1, hist_cap=200000,
                         max_iters=20000)
    assert np.max(np.abs(h[:k] - h2[:k])) <= 1e-10
    M.close()


@pytest.mark.parametrize("side", [37, 64, 259])
def test_gmres_ir_fp32_matches_oracle(side):
    A, bb = _system(side)
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    say("lowsync IR fp32", side)
    x, d, h = B.solve(M, b, restart=50, inner="fp32", rtol=1e-12, check_mode=1, ortho="dcgs2", hist_cap=200000,
                      max_iters=20000)
    ref = L.gmres_ir(A, bb, m=50, rtol=1e-12, inner="fp32", check_mode=1, ortho="dcgs2", max_iters=20000)
    assert d["status"] == B.OK and ref.status == L.OK
    assert d["rel_resid_true"] <= 1e-12
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    assert abs(d["iters"] - ref.iters) <= 50
    k1 = _first(ref)
    assert np.max(np.abs(h[:k1] - np.array(ref.hist[:k1]))) <= HIST_TOL_FP32
    M.close()


@pytest.mark.parametrize("m", [1, 7, 16, 17, 33, 64, 65, 100, 128])
@pytest.mark.parametrize("side", [37, 259])
def test_restart_classes_first_cycle(m, side):
    """Every column-count class of the fused and separate reduction kernels:
    the first cycle against the oracle's (paper mode, full cycles)."""
    A, bb = _system(side, pe=20.0, seed=m)
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    for inner in ("fp64", "fp32"):
        say("lowsync first cycle", side, m, inner)
        x, d, h = B.solve(M, b, restart=m, inner=inner, rtol=1e-10, check_mode=0, ortho="dcgs2", max_iters=m,
                          hist_cap=m)
        if inner == "fp64":
            ref = L.gmres(A, bb, m=m, rtol=1e-10, check_mode=0, ortho="dcgs2", max_iters=m)
            tol = 1e-10
        else:
            ref = L.gmres_ir(A, bb, m=m, rtol=1e-10, inner="fp32", check_mode=0, ortho="dcgs2", max_iters=m)
            tol = HIST_TOL_FP32
        k = min(m, len(ref.hist))
        assert d["iters"] == ref.iters
        assert np.max(np.abs(h[:k] - np.array(ref.hist[:k]))) <= tol, (m, inner)
    M.close()


def test_paper_mode_and_breakdown():
    A, bb = _system(64, pe=10.0, wind=(1.0, 1.0))
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    say("lowsync check_mode 0")
    x, d, _ = B.solve(M, b, restart=50, inner="fp32", rtol=1e-10, check_mode=0, ortho="dcgs2")
    assert d["status"] == B.OK and d["iters"] % 50 == 0 and d["rel_resid_true"] <= 1e-10
    M.close()
    # n = 12 < m: exact termination by breakdown
    A = P.conv_diff(2, 3, 5.0, (1.0, 0.0))
    M = B.Matrix.from_csr(A)
    bb = np.arange(1.0, A.n + 1)
    for inner in ("fp64", "fp32"):
        say("lowsync breakdown", inner)
        x, d, _ = B.solve(M, dev_tensor(bb), restart=30, inner=inner, rtol=1e-10, ortho="dcgs2")
        assert d["status"] == B.OK and d["rel_resid_true"] <= 1e-10 and d["iters"] <= 2 * A.n
        assert rel(x.cpu().numpy(), np.linalg.solve(A.scipy().toarray(), bb)) <= 1e-8
    M.close()


@pytest.mark.parametrize("side", [14, 42])  # 3D: 2744 rows (separate reduction), 74088 rows (fused)
def test_polynomial_preconditioned(side):
    A = P.conv_diff(3, side, 10.0, (1, 1, 1), (1, 1, 1e-2))
    bb = A.scipy() @ np.random.default_rng(0).uniform(-1, 1, A.n)
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    roots = PO.poly_roots(A, 10, start=PO.start_vector(A.n, 3), dtype=np.float32)
    say("lowsync poly d=10", side)
    x, d, h = B.solve(M, b, restart=30, inner="fp32", rtol=1e-12, poly_degree=10, poly_roots=roots, ortho="dcgs2",
                      hist_cap=5000)
    ref = L.gmres_ir(A, bb, m=30, rtol=1e-12, inner="fp32", poly_roots=roots, check_mode=1, ortho="dcgs2")
    assert d["status"] == B.OK and ref.status == L.OK and d["rel_resid_true"] <= 1e-12
    assert abs(d["iters"] - ref.iters) <= 30
    k1 = _first(ref)
    assert np.max(np.abs(h[:k1] - np.array(ref.hist[:k1]))) <= HIST_TOL_FP32
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    M.close()


@pytest.mark.parametrize("side", [64, 259])
def test_block_jacobi(side):
    A, bb = _system(side)
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    say("lowsync block Jacobi 8", side)
    x, d, h = B.solve(M, b, restart=50, inner="fp32", rtol=1e-12, bj_block=8, ortho="dcgs2", hist_cap=100000)
    ref = L.gmres_ir(A, bb, m=50, rtol=1e-12, inner="fp32", bj_block=8, check_mode=1, ortho="dcgs2")
    assert d["status"] == B.OK and ref.status == L.OK and d["rel_resid_true"] <= 1e-12
    k1 = _first(ref)
    assert np.max(np.abs(h[:k1] - np.array(ref.hist[:k1]))) <= HIST_TOL_FP32
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    M.close()


def test_fp32_polynomial_in_fp64():
    A = P.stencil_matrix("laplace3d_7", 12)
    bnp = A.scipy() @ np.random.default_rng(0).uniform(-1, 1, A.n)
    roots = PO.poly_roots(A, 10, seed=12345)
    M = B.Matrix.from_csr(A)
    say("lowsync fp64 + fp32 poly")
    x, d, h = B.solve(M, dev_tensor(bnp), restart=50, inner="fp64", rtol=1e-12, poly_degree=10, poly_prec="fp32",
                      poly_roots=roots, ortho="dcgs2", hist_cap=10000)
    ref = L.gmres_ir(A, bnp, m=50, rtol=1e-12, inner="fp64", poly_roots=roots, poly_prec="fp32", check_mode=1,
                     ortho="dcgs2")
    assert d["status"] == B.OK and ref.status == L.OK
    assert d["iters"] == ref.iters
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    k1 = _first(ref)
    assert np.max(np.abs(h[:k1] - np.array(ref.hist[:k1]))) <= 1e-5
    M.close()


def test_graph_replay_and_determinism():
    A, bb = _system(64)
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    for kw in (dict(restart=50, inner="fp32"), dict(restart=30, inner="fp64"), dict(restart=20, inner="fp32",
                                                                                   inner_cap=60)):
        say("lowsync graph vs direct", kw)
        xg, dg, hg = B.solve(M, b, rtol=1e-10, hist_cap=20000, ortho="dcgs2", **kw)
        xg2, _, _ = B.solve(M, b, rtol=1e-10, ortho="dcgs2", **kw)
        xd, dd, hd = B.solve(M, b, rtol=1e-10, hist_cap=20000, profile=1, ortho="dcgs2", **kw)
        assert dg["status"] == B.OK and dg["refinements"] >= 2
        assert torch.equal(xg, xd) and torch.equal(xg, xg2)
        assert np.array_equal(hg, hd)
    M.close()


def test_arguments():
    A, bb = _system(20)
    M = B.Matrix.from_csr(A)
    say("lowsync arguments")
    assert B.gmresir_workspace_bytes(M, B.make_params(basis="bf16", ortho="dcgs2")) == 0
    assert B.gmresir_workspace_bytes(M, B.make_params(restart=129, ortho="dcgs2")) == 0
    assert B.gmresir_workspace_bytes(M, B.make_params(ortho=2)) == 0
    assert B.gmresir_workspace_bytes(M, B.make_params(restart=128, ortho="dcgs2")) > 0
    M.close()
