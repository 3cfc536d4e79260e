"""GPU SpMV parity over the constant-coefficient stencil families of the SpMV
study (2D 5/9/9/13-point, 3D 7/19/27-point): bitwise against the oracle's
SpMV in fp64 and fp32 (both sum each row in column order from identically
rounded products), on grids whose rows span several tiles and slices and end
in a ragged slice."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import linalg as L
from paper_2109_01232_amd import binding as B
from paper_2109_01232_amd import problems as P

from gpu_common import dev_tensor, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", sorted(P.STENCILS))
def test_spmv_family_bitwise(name):
    dim = P.STENCILS[name][0]
    n = 301 if dim == 2 else 45  # 90601 / 91125 rows: ragged last 64-row slice
    A = P.stencil_matrix(name, n)
    say("spmv family", name, A.n, A.nnz)
    M = B.Matrix.from_csr(A)
    x = np.random.default_rng(5).uniform(-1, 1, A.n)
    for prec, dt in (("fp64", np.float64), ("fp32", np.float32)):
        xd = dev_tensor(x.astype(dt))
        yd = torch.empty_like(xd)
        B.gmresir_spmv(M, xd, yd, prec)
        torch.cuda.synchronize()
        ref = L.spmv(L.csr_matrix(A, dt), x.astype(dt))
        assert np.array_equal(yd.cpu().numpy(), ref), prec
    M.close()
