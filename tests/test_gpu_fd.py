"""GPU parity of GMRES-FD (Section "Mixed Precision GMRES-FD") through the C ABI.

Bars as in the other parity tests: final fp64 relative residual <= rtol on
both sides, solutions within 1e-8 relative, the first fp32 cycle's implicit
residual history within 1e-5 of the oracle's (same input b / ||b||), and the
explicit residual at the switch within 1e-5 of the oracle's (the fp32 phases
differ only by rounding order).  Switch 0 is the library's own fp64 GMRES(m),
bit for bit.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import linalg as L
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


@pytest.fixture(scope="module")
def conv64():
    s = P.parity_system()
    return s, B.Matrix.from_csr(s.A)


def test_switch_zero_is_fp64_gmres(conv64):
    s, M = conv64
    say("fd switch 0 vs fp64 solve")
    b = dev_tensor(s.b)
    x0, d0, h0 = B.solve(M, b, restart=50, inner="fp64", rtol=1e-10, check_mode=1, hist_cap=5000)
    x1, d1, h1 = B.solve_fd(M, b, 0, restart=50, rtol=1e-10, check_mode=1, hist_cap=5000)
    assert d0["status"] == d1["status"] == B.OK
    assert d0["iters"] == d1["iters"]
    assert torch.equal(x0, x1)
    assert np.array_equal(h0, h1)


def test_fd_matches_oracle(conv64):
    s, M = conv64
    say("fd switch 100 conv64 vs oracle")
    b = dev_tensor(s.b)
    x, d, h = B.solve_fd(M, b, 100, restart=50, rtol=1e-12, check_mode=0, hist_cap=100000)
    ref = L.gmres_fd(s.A, s.b, 100, m=50, rtol=1e-12, check_mode=0)
    xs = x.cpu().numpy()
    assert d["status"] == B.OK and ref.status == L.OK
    true = np.linalg.norm(s.b - s.A.scipy() @ xs) / np.linalg.norm(s.b)
    assert true <= 1e-12 and ref.rel_resid <= 1e-12
    assert d["rel_resid_true"] == pytest.approx(true, rel=1e-6)
    assert rel(xs, ref.x) <= 1e-8
    assert rel(xs, s.u) <= 1e-6
    assert len(h) == d["iters"] and d["iters"] > 100
    # the fp64 phase checks at restarts (check_mode 0): whole cycles after the switch
    assert (d["iters"] - 100) % 50 == 0
    assert abs(d["iters"] - ref.iters) <= 50
    assert np.max(np.abs(h[:50] - np.array(ref.hist[:50]))) <= 1e-5


@pytest.mark.parametrize("switch", [50, 120])
def test_iterate_at_switch(conv64, switch):
    """max_iters = switch stops after the fp32 phase: its explicit residual
    agrees with the oracle's, and the phase equals one refinement of the
    fp32 GMRES-IR path with inner_cap = switch (same kernels, same bits)."""
    s, M = conv64
    say("fd iterate at switch", switch)
    b = dev_tensor(s.b)
    x, d, h = B.solve_fd(M, b, switch, restart=50, rtol=1e-10, max_iters=switch, hist_cap=1000)
    ref = L.gmres_fd(s.A, s.b, switch, m=50, rtol=1e-10, max_iters=switch)
    assert d["status"] == B.NOT_CONVERGED and ref.status == L.NOT_CONVERGED
    assert d["iters"] == switch == ref.iters
    assert abs(d["rel_resid_true"] - ref.outer[1]) <= 1e-5
    assert np.max(np.abs(h[:50] - np.array(ref.hist[:50]))) <= 1e-5
    x2, d2, h2 = B.solve(M, b, restart=50, inner="fp32", rtol=1e-10, inner_cap=switch, max_iters=switch,
                         check_mode=0, hist_cap=1000)
    assert d2["iters"] == switch
    assert torch.equal(x, x2)
    assert np.array_equal(h, h2)


def test_bf16_basis_phase(conv64):
    s, M = conv64
    say("fd bf16 basis conv64")
    b = dev_tensor(s.b)
    x, d, _ = B.solve_fd(M, b, 100, restart=50, basis="bf16", rtol=1e-10, check_mode=1)
    xs = x.cpu().numpy()
    assert d["status"] == B.OK
    assert np.linalg.norm(s.b - s.A.scipy() @ xs) / np.linalg.norm(s.b) <= 1e-10


def test_argument_errors(conv64):
    s, M = conv64
    say("fd argument errors")
    lib = B.lib()
    for kw, sw in ((dict(inner_cap=100), 50), (dict(poly_degree=5), 50), ({}, -1)):
        p = B.make_params(inner="fp32", **kw)
        assert lib.gmresir_fd_workspace_bytes(M.handle, ctypes.byref(p), sw) == 0
    p = B.make_params(inner="fp64")
    assert lib.gmresir_fd_workspace_bytes(M.handle, ctypes.byref(p), 50) == 0
    p = B.make_params(inner="fp32")
    need = B.gmresir_fd_workspace_bytes(M, p, 100)
    assert need >= max(B.gmresir_workspace_bytes(M, B.make_params(inner="fp64")),
                       B.gmresir_workspace_bytes(M, B.make_params(inner="fp32", inner_cap=100)))
    b = dev_tensor(s.b)
    x = torch.zeros_like(b)
    ws = B._empty_bytes(need - 256, "cuda")
    res = B.Result()
    st = lib.gmresir_solve_fd(M.handle, B._ptr(b), B._ptr(x), ctypes.byref(p), 100, B._ptr(ws), ws.numel(),
                              ctypes.byref(res), None, 0, B._stream())
    assert st == B.ERR_WORKSPACE
    assert torch.count_nonzero(x) == 0
    # b = 0 gives x = 0
    z = torch.zeros_like(b)
    x.fill_(1.0)
    _, d, _ = B.gmresir_solve_fd(M, z, x, p, 100)
    assert d["status"] == B.OK and torch.count_nonzero(x) == 0


def test_fd_headline_size_converges():
    """2D convection-diffusion 1000 x 1000 (seed 0): switch after 500 fp32
    iterations, then fp64 GMRES(50) to 1e-10 (checked on the host)."""
    s = P.convdiff2d_system(0)
    M = B.Matrix.from_csr(s.A)
    say("fd 1000^2 switch 500")
    b = dev_tensor(s.b)
    x, d, _ = B.solve_fd(M, b, 500, restart=50, rtol=1e-10, check_mode=1)
    xs = x.cpu().numpy()
    assert d["status"] == B.OK and d["iters"] > 500
    true = np.linalg.norm(s.b - s.A.scipy() @ xs) / np.linalg.norm(s.b)
    assert true <= 1e-10
    assert d["rel_resid_true"] == pytest.approx(true, rel=1e-3)
    M.close()
