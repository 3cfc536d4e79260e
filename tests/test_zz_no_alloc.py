"""gmresir_solve_noalloc (workspace from the library's static device array)
against gmresir_solve with a caller workspace, through the C ABI.

Both run the same kernels on the same workspace layout (the workspace is
carved at the same offsets from a 256-byte aligned base; gmresir_solve
replays small systems' cycles as a HIP graph, which gives the same bits as
the direct launches the allocation-free call makes), so the bar is bitwise
equality of the solution, the iteration counts and the history.  Each case
makes two calls in a row, the second on a smaller system, since every call
on a GPU shares the one array and must not depend on what the last call left
in it.  The results are also held to the oracle at the parity bars."""
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


@pytest.mark.parametrize("inner,basis", [("fp32", "fp32"), ("fp64", "fp64"), ("fp32", "bf16")])
def test_noalloc_matches_workspace_solve(inner, basis):
    systems = [P.parity_system(), P.convdiff2d_system(3, n=40)]  # 4096 rows, then 1600
    for s in systems:
        M = B.Matrix.from_csr(s.A)
        b = dev_tensor(s.b)
        p = B.make_params(restart=50, inner=inner, basis=basis, rtol=1e-10, check_mode=1)
        assert B.gmresir_workspace_bytes(M, p) <= B.NOALLOC_MAX_BYTES
        say("noalloc", inner, basis, s.A.n)
        x_ws = torch.zeros_like(b)
        st_ws, d_ws, h_ws = B.gmresir_solve(M, b, x_ws, p, hist_cap=100000)
        x_na = torch.zeros_like(b)
        st_na, d_na, h_na = B.gmresir_solve_noalloc(M, b, x_na, p, hist_cap=100000)
        torch.cuda.synchronize()
        assert st_na == st_ws
        assert d_na["iters"] == d_ws["iters"] and d_na["refinements"] == d_ws["refinements"]
        assert torch.equal(x_na, x_ws)
        assert np.array_equal(h_na, h_ws)
        if basis != "bf16":
            ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner=inner, check_mode=1)
            assert st_na == B.OK and ref.status == L.OK
            assert d_na["rel_resid_true"] <= 1e-10
            xs = x_na.cpu().numpy()
            assert np.linalg.norm(s.b - s.A.scipy() @ xs) / np.linalg.norm(s.b) <= 1e-10
        M.close()


def test_noalloc_rejects_oversized_solve():
    s = P.convdiff2d_system(0, n=600)  # 360,000 rows: the fp32 basis of GMRES(50) alone is 73 MB
    M = B.Matrix.from_csr(s.A)
    b = dev_tensor(s.b)
    p = B.make_params(restart=50, inner="fp32", rtol=1e-10)
    assert B.gmresir_workspace_bytes(M, p) > B.NOALLOC_MAX_BYTES
    x = torch.full_like(b, 0.5)
    say("noalloc oversized")
    with pytest.raises(B.GmresirError) as e:
        B.gmresir_solve_noalloc(M, b, x, p)
    assert e.value.status == B.ERR_WORKSPACE
    assert "scratch" in B.last_error()
    assert torch.all(x == 0.5)
    with pytest.raises(B.GmresirError) as e:
        B.gmresir_solve_noalloc(M, b, x, B.make_params(restart=50, inner="fp32", profile=1))
    assert e.value.status == B.ERR_INVALID_ARG
    M.close()
