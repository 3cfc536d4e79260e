"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (GMRES-IR, fp32 inner GMRES(50) or GMRES(100), fp64
refinement, implicit early exit, default workspace).

At these sizes the oracle cannot run whole solves in test time, so the
comparisons are on outputs it computes one at a time:

* SpMV: every row, bitwise (both sides sum each row in column order);
* the first inner cycle (identical input ``round(b / ||b||)``): the
  cycle-normalised implicit residual history, 1e-5 for fp32 bases and the
  relative bf16 bar of ``gpu_common.bf16_hist_ok`` for bf16-stored bases, as
  for the small systems -- on the 150^3 system also with a degree-10
  polynomial built from the oracle's roots (GMRES(100)), and with the
  one-reduction CGS2 on both 3D systems;
* later cycles: the GPU restarts from the oracle's own fp64 iterates and runs
  one cycle, compared with the oracle's next cycle;
* the polynomial preconditioner: the product form with the oracle's roots,
  element by element against the oracle's fp32 product form, and the
  GPU-built Hessenberg matrix for the same start vector;
* whole solves: properties that hold at any size -- the fp64 relative
  residual ``||b - A x|| / ||b||`` recomputed here with scipy is <= 1e-10 and
  matches the one the library reports.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import linalg as L
from oracle import poly as PO
from paper_2109_01232_amd import binding as B
from paper_2109_01232_amd import problems as P

from gpu_common import bf16_hist_ok, dev_tensor, rel, say

pytestmark = pytest.mark.gpu

HIST_TOL_FP32 = 1e-5
U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def ws():
    return B.Workspace()


@pytest.fixture(scope="module")
def cd2d():
    say("build convdiff2d 1000x1000")
    s = P.convdiff2d_system(0)
    return s, B.Matrix.from_csr(s.A)


@pytest.fixture(scope="module")
def vc27():
    say("build varcoef27 128^3")
    s = P.varcoef27_system(0)
    return s, B.Matrix.from_csr(s.A)


@pytest.fixture(scope="module")
def an3d():
    say("build aniso3d 150^3")
    s = P.aniso3d_system(0)
    return s, B.Matrix.from_csr(s.A)


def _spmv_bitwise(s, M):
    x = np.random.default_rng(7).uniform(-1, 1, s.A.n)
    for prec, dt in (("fp64", np.float64), ("fp32", np.float32)):
        xd = dev_tensor(x.astype(dt))
        yd = torch.empty_like(xd)
        B.gmresir_spmv(M, xd, yd, prec)
        torch.cuda.synchronize()
        ref = L.spmv(L.csr_matrix(s.A, dt), x.astype(dt))
        y = yd.cpu().numpy()
        assert np.array_equal(y, ref), (prec, int(np.sum(y != ref)), float(np.abs(y - ref).max()))


def _true_resid(s, xd):
    xs = xd.cpu().numpy()
    return float(np.linalg.norm(s.b - s.A.scipy() @ xs) / np.linalg.norm(s.b)), xs


def test_convdiff2d_spmv(cd2d):
    say("spmv convdiff2d 1000x1000")
    _spmv_bitwise(*cd2d)


def test_convdiff2d_first_cycle_and_solve(cd2d, ws):
    s, M = cd2d
    b = dev_tensor(s.b)
    say("ir fp32 m=50 convdiff2d 1000x1000")
    x, d, h = B.solve(M, b, ws=ws, restart=50, inner="fp32", rtol=1e-10, check_mode=1, hist_cap=1 << 16)
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", check_mode=0, max_iters=50)
    assert ref.iters == 50
    assert np.max(np.abs(h[:50] - np.array(ref.hist[:50]))) <= HIST_TOL_FP32
    assert d["status"] == B.OK
    true, xs = _true_resid(s, x)
    assert true <= 1e-10 and d["rel_resid_true"] == pytest.approx(true, rel=1e-6)
    # the manufactured solution (the error measured in the benchmark runs is ~1e-7)
    assert rel(xs, s.u) <= 1e-6


def test_convdiff2d_cycle_replay(cd2d, ws):
    """Later cycles on identical input: both sides restart from the oracle's
    fp64 iterate x_i and run one fp32 cycle.  (Against the oracle's fp64
    cycle the fp32 history drifts by ~1e-5 at N = 1e6 -- that gap is the
    precision change, not a defect -- so the comparison is fp32 with fp32.)"""
    s, M = cd2d
    say("oracle fp64 IR, 2 cycles, convdiff2d 1000x1000")
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-14, inner="fp64", check_mode=0, max_iters=100, keep_iterates=True)
    b = dev_tensor(s.b)
    for i in (0, 1):
        say("replay cycle", i + 1)
        one = L.gmres_ir(s.A, s.b, x0=ref.xs[i], m=50, rtol=1e-14, inner="fp32", check_mode=0, max_iters=50)
        x, d, h = B.solve(M, b, ws=ws, x0=dev_tensor(ref.xs[i]), restart=50, inner="fp32", rtol=1e-14,
                          check_mode=0, max_iters=50, hist_cap=50)
        assert d["iters"] == 50 and one.iters == 50
        assert np.max(np.abs(h - np.array(one.hist))) <= HIST_TOL_FP32, i


def test_convdiff2d_bf16_first_cycle_and_solve(cd2d, ws):
    """bf16-stored basis on the 1000x1000 system: the refinement stagnates
    between 1e-7 and 1e-6 on both sides (the oracle's GMRES-IR(50) with a bf16
    basis stops with STAGNATED at 1.0e-7 after 50 refinements): with
    cond(A) ~ 1e3-1e4 the bf16 unit roundoff 2^-9 no longer gives the inner
    solve the accuracy iterative refinement needs.  Checked: the first cycle
    agrees with the oracle, and the solve ends OK or STAGNATED with the
    stagnation level of the oracle."""
    s, M = cd2d
    b = dev_tensor(s.b)
    say("ir bf16 basis m=50 convdiff2d 1000x1000")
    x, d, h = B.solve(M, b, ws=ws, restart=50, inner="fp32", basis="bf16", rtol=1e-10, check_mode=1,
                      hist_cap=1 << 16)
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", basis="bf16", check_mode=0, max_iters=50)
    ok, info = bf16_hist_ok(h[:50], ref.hist[:50])
    assert ok, info
    assert d["status"] in (B.OK, B.STAGNATED)
    true, _ = _true_resid(s, x)
    assert true <= 1e-6 and d["rel_resid_true"] == pytest.approx(true, rel=1e-6)


def test_varcoef27_spmv(vc27):
    say("spmv varcoef27 128^3")
    _spmv_bitwise(*vc27)


@pytest.mark.parametrize("basis", ["fp32", "bf16"])
def test_varcoef27_first_cycle_and_solve(vc27, ws, basis):
    s, M = vc27
    b = dev_tensor(s.b)
    say("ir", basis, "basis m=50 varcoef27 128^3")
    x, d, h = B.solve(M, b, ws=ws, restart=50, inner="fp32", basis=basis, rtol=1e-10, check_mode=1,
                      hist_cap=1 << 16)
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", basis=basis, check_mode=0, max_iters=50)
    if basis == "bf16":
        ok, info = bf16_hist_ok(h[:50], ref.hist[:50])
        assert ok, info
    else:
        assert np.max(np.abs(h[:50] - np.array(ref.hist[:50]))) <= HIST_TOL_FP32
    assert d["status"] == B.OK
    true, _ = _true_resid(s, x)
    assert true <= 1e-10 and d["rel_resid_true"] == pytest.approx(true, rel=1e-6)


def test_varcoef27_fp64_gmres_first_cycle_and_solve(vc27, ws):
    """The fp64 GMRES(50) the headline compares against: first cycle against
    the oracle's fp64 cycle (fp64 on both sides: 1e-10), then the whole
    solve's fp64 residual."""
    s, M = vc27
    b = dev_tensor(s.b)
    say("fp64 gmres m=50 varcoef27 128^3")
    x, d, h = B.solve(M, b, ws=ws, restart=50, inner="fp64", rtol=1e-10, check_mode=1, hist_cap=1 << 16)
    ref = L.gmres(s.A, s.b, m=50, rtol=1e-10, check_mode=0, max_iters=50)
    assert np.max(np.abs(h[:50] - np.array(ref.hist[:50]))) <= 1e-10
    assert d["status"] == B.OK
    true, _ = _true_resid(s, x)
    assert true <= 1e-10 and d["rel_resid_true"] == pytest.approx(true, rel=1e-6)


def test_varcoef27_one_reduction_first_cycle_and_solve(vc27, ws):
    """The one-reduction CGS2 variant the benchmark times beside the
    headline: first cycle against the oracle's one-reduction fp32 cycle, then
    the whole solve's fp64 residual."""
    s, M = vc27
    b = dev_tensor(s.b)
    say("ir one-reduction m=50 varcoef27 128^3")
    x, d, h = B.solve(M, b, ws=ws, restart=50, inner="fp32", ortho="dcgs2", rtol=1e-10, check_mode=1,
                      hist_cap=1 << 16)
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", ortho="dcgs2", check_mode=0, max_iters=50)
    assert np.max(np.abs(h[:50] - np.array(ref.hist[:50]))) <= HIST_TOL_FP32
    assert d["status"] == B.OK
    true, _ = _true_resid(s, x)
    assert true <= 1e-10 and d["rel_resid_true"] == pytest.approx(true, rel=1e-6)


def test_aniso3d_one_reduction_first_cycle(an3d, ws):
    """One-reduction CGS2 at the 150^3 configuration (fp32 GMRES(100), every
    column class up to 100): first cycle on identical input against the
    oracle's one-reduction fp32 cycle."""
    s, M = an3d
    b = dev_tensor(s.b)
    say("ir one-reduction m=100 first cycle aniso3d 150^3")
    x, d, h = B.solve(M, b, ws=ws, restart=100, inner="fp32", ortho="dcgs2", rtol=1e-10, check_mode=0,
                      max_iters=100, hist_cap=100)
    ref = L.gmres_ir(s.A, s.b, m=100, rtol=1e-10, inner="fp32", ortho="dcgs2", check_mode=0, max_iters=100)
    assert d["iters"] == ref.iters == 100
    assert np.max(np.abs(h - np.array(ref.hist))) <= HIST_TOL_FP32


def test_aniso3d_spmv(an3d):
    say("spmv aniso3d 150^3")
    _spmv_bitwise(*an3d)


def test_aniso3d_poly_apply_and_setup(an3d, ws):
    s, M = an3d
    d = 20
    start = PO.start_vector(s.A.n, 5)
    say("oracle poly roots d=20 aniso3d 150^3")
    ref_cyc = L.gmres_cycle(lambda z: L.spmv(L.csr_matrix(s.A, np.float32), z), start.astype(np.float32), d + 1,
                            np.float32)
    roots = PO.poly_roots(s.A, d, start=start, dtype=np.float32)
    v = np.random.default_rng(3).standard_normal(s.A.n).astype(np.float32)
    vd = dev_tensor(v)
    yd = torch.empty_like(vd)
    say("poly apply d=20 aniso3d 150^3")
    B.gmresir_poly_apply(M, roots, vd, yd, ws=ws)
    torch.cuda.synchronize()
    ref32 = PO.apply_product_form(L.csr_matrix(s.A, np.float32), roots, v, np.float32)
    ref64 = PO.apply_product_form(L.csr_matrix(s.A, np.float64), roots, v.astype(np.float64), np.float64)
    got = yd.cpu().numpy()
    scale = np.abs(ref32).max()
    gap = np.abs(got - ref32).max() / scale
    # two fp32 evaluations, each within the fp32 rounding error e of the exact
    # (fp64) value, differ by at most 2 e: at this size e = 1.24e-5 element-wise
    # (the oracle's own), measured gap 1.5e-5
    e_or = np.abs(ref32 - ref64).max() / scale
    assert gap <= max(8 * d * U32, 2.5 * e_or), (gap, e_or)
    assert np.abs(got - ref64).max() / scale <= max(8 * d * U32, 2.5 * e_or)
    say("poly setup d=20 aniso3d 150^3, given start")
    groots, hbar = B.gmresir_poly_setup(M, d, start=dev_tensor(start), ws=ws, with_hbar=True)
    assert rel(hbar, ref_cyc.Hbar) <= 1e-4
    # the root sets: each GPU root lies near an oracle root and vice versa
    # (harmonic Ritz values of close eigenvalue clusters are ill-conditioned,
    # so this is a loose bound; the apply check above is the tight one)
    scale = np.abs(roots).max()
    dist = np.abs(groots[:, None] - roots[None, :])
    assert dist.min(axis=1).max() <= 1e-2 * scale and dist.min(axis=0).max() <= 1e-2 * scale


@pytest.mark.parametrize("deg", [10, 40])
def test_aniso3d_poly_solve(an3d, ws, deg):
    s, M = an3d
    b = dev_tensor(s.b)
    say("poly setup + ir m=100 aniso3d 150^3 d", deg)
    roots = B.gmresir_poly_setup(M, deg, seed=12345, ws=ws)
    x, d, _ = B.solve(M, b, ws=ws, restart=100, inner="fp32", rtol=1e-10, check_mode=1, poly_degree=deg,
                      poly_roots=roots)
    assert d["status"] == B.OK
    true, _ = _true_resid(s, x)
    assert true <= 1e-10 and d["rel_resid_true"] == pytest.approx(true, rel=1e-6)


@pytest.mark.parametrize("deg", [0, 10])
def test_aniso3d_first_cycle(an3d, ws, deg):
    """The benchmark configuration of the 150^3 system, fp32 GMRES(100) (with
    a degree-10 polynomial from the oracle's roots), first cycle on identical
    input against the oracle's fp32 cycle (measured gaps 2.1e-7 and 1.3e-8)."""
    s, M = an3d
    b = dev_tensor(s.b)
    roots = None
    if deg:
        say("oracle poly roots d=10 aniso3d 150^3")
        roots = PO.poly_roots(s.A, deg, start=PO.start_vector(s.A.n, 12345), dtype=np.float32)
    say("ir m=100 first cycle aniso3d 150^3 d", deg)
    x, d, h = B.solve(M, b, ws=ws, restart=100, inner="fp32", rtol=1e-10, check_mode=0, max_iters=100,
                      poly_degree=deg, poly_roots=roots, hist_cap=100)
    ref = L.gmres_ir(s.A, s.b, m=100, rtol=1e-10, inner="fp32", check_mode=0, max_iters=100, poly_roots=roots)
    assert d["iters"] == ref.iters == 100
    assert np.max(np.abs(h - np.array(ref.hist))) <= HIST_TOL_FP32
