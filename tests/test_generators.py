"""Input generators: sparsity structure pinned to the sizes the paper prints."""
import json
import os

import numpy as np
import pytest

from paper_2109_01232_amd import problems as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("case", _load("paper_stencil_sizes.json")["cases"], ids=lambda c: c["name"])
def test_stencil_counts_match_paper(case):
    """Eliminated-Dirichlet stencils reproduce the paper's N / nnz exactly."""
    n = case["n"]
    if case["dim"] == 2:
        assert n * n == case["N"]
        assert P.stencil_nnz_2d5(n) == case["nnz"]
    else:
        assert n ** 3 == case["N"]
        assert P.stencil_nnz_3d7(n) == case["nnz"]


@pytest.mark.slow
def test_generator_builds_paper_sizes():
    """The generator itself (not only the closed form) hits the printed counts."""
    A = P.conv_diff(2, 1500, 10.0, (1.0, 1.0))
    assert (A.n, A.nnz) == (2250000, 11244000)
    A = P.conv_diff(3, 150, 10.0, (1.0, 1.0, 1.0), (1.0, 1.0, 1e-2))
    assert (A.n, A.nnz) == (3375000, 23490000)


@pytest.mark.parametrize("n", [3, 4, 7, 13])
def test_small_stencils_structure(n):
    A2 = P.conv_diff(2, n, 10.0, (1.0, 1.0))
    assert A2.nnz == P.stencil_nnz_2d5(n)
    A3 = P.conv_diff(3, n, 10.0, (1.0, 1.0, 1.0))
    assert A3.nnz == P.stencil_nnz_3d7(n)
    A27 = P.varcoef27(n, 5)
    assert A27.nnz == P.stencil_nnz_27(n)
    for A in (A2, A3, A27):
        rp = A.rowptr
        assert rp[0] == 0 and np.all(np.diff(rp) > 0)
        for i in range(A.n):
            cols = A.colidx[rp[i]:rp[i + 1]]
            assert np.all(np.diff(cols) > 0), "columns ascending within a row"
            assert i in cols, "diagonal present"


def test_convdiff_stencil_values():
    """Interior row of the 2D operator: centre 2(k1+k2), neighbours -k_d -/+ Pe w_d h / 2."""
    n, Pe, w, k = 9, 30.0, (0.6, -0.8), (1.0, 0.25)
    A = P.conv_diff(2, n, Pe, w, k).scipy().toarray()
    h = 1.0 / (n + 1)
    i = 4 + n * 4
    assert A[i, i] == pytest.approx(2 * (k[0] + k[1]))
    assert A[i, i - 1] == pytest.approx(-k[0] - Pe * w[0] * h / 2)
    assert A[i, i + 1] == pytest.approx(-k[0] + Pe * w[0] * h / 2)
    assert A[i, i - n] == pytest.approx(-k[1] - Pe * w[1] * h / 2)
    assert A[i, i + n] == pytest.approx(-k[1] + Pe * w[1] * h / 2)
    # Pe = 0 gives the symmetric (scaled) Laplacian
    L = P.conv_diff(2, n, 0.0, (1.0, 1.0)).scipy()
    assert abs(L - L.T).max() == 0.0


def test_varcoef27_is_m_matrix_with_row_sum():
    A = P.varcoef27(6, 11)
    S = A.scipy()
    rs = S @ np.ones(A.n)
    assert np.max(np.abs(rs - 0.05)) <= 1e-13
    D = S.diagonal()
    off = S - __import__("scipy.sparse", fromlist=["diags"]).diags(D)
    assert off.max() < 0 or off.nnz == 0 or off.data.max() < 0
    assert np.all(D > np.asarray(abs(off).sum(axis=1)).ravel())
    assert abs(S - S.T).max() > 0.1, "nonsymmetric"
    # entries within the documented range: -(1 +- 0.3) +- 0.5
    assert off.data.min() >= -1.8 - 1e-12 and off.data.max() <= -0.2 + 1e-12


def test_varcoef27_shift_and_chooser_families():
    # the row-sum shift is a parameter; the off-diagonal draws do not depend on it
    A1, A2 = P.varcoef27(5, 3, shift=0.3), P.varcoef27(5, 3)
    assert np.max(np.abs(A1.scipy() @ np.ones(A1.n) - 0.3)) <= 1e-13
    off = A1.colidx != np.repeat(np.arange(A1.n), np.diff(A1.rowptr))
    assert np.array_equal(A1.vals[off], A2.vals[off])
    # the chooser population: about a quarter 27-point systems, the rest convection-diffusion
    fams = [P.chooser_system(s, n_max=2e4).meta["family"] for s in range(400)]
    k = fams.count("varcoef27")
    assert 70 <= k <= 130 and fams.count("convdiff") == 400 - k
    s27 = next(P.chooser_system(s, n_max=2e4) for s in range(400) if fams[s] == "varcoef27")
    assert 1e-2 <= s27.meta["shift"] <= 1.0 and s27.A.nnz > 20 * s27.A.n


def test_seeded_reproducible():
    a = P.convdiff2d_system(3, n=30)
    b = P.convdiff2d_system(3, n=30)
    c = P.convdiff2d_system(4, n=30)
    assert np.array_equal(a.b, b.b) and a.meta["Pe"] == b.meta["Pe"]
    assert not np.array_equal(a.b, c.b)
    assert 1.0 <= a.meta["Pe"] <= 100.0
    s1, s2 = P.chooser_system(7, n_max=5e4), P.chooser_system(7, n_max=5e4)
    assert np.array_equal(s1.A.vals, s2.A.vals) and np.array_equal(s1.b, s2.b)


def test_rhs_is_A_u():
    s = P.parity_system()
    assert np.allclose(s.A.scipy() @ np.ones(s.A.n), s.b)
    # b = A * ones is nonzero only next to the boundary (interior rows sum to 0 when Pe terms cancel)
    assert s.A.n == 4096 and s.A.nnz == 20224


# ---------------------------------------------------------------------------
# constant-coefficient stencil families of the SpMV study
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", sorted(P.STENCILS))
@pytest.mark.parametrize("n", [7, 16])
def test_stencil_family_nnz_and_layout(name, n):
    A = P.stencil_matrix(name, n)
    assert A.nnz == P.stencil_nnz(name, n)
    dim, pat = P.STENCILS[name]
    assert A.n == n ** dim
    counts = np.diff(A.rowptr)
    assert counts.max() == len(pat)  # interior rows hold the whole stencil
    for r in range(A.n):
        c = A.colidx[A.rowptr[r]:A.rowptr[r + 1]]
        assert np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < A.n


def _tri(n, lo, mid, hi):
    import scipy.sparse as sp

    return sp.diags([np.full(n - 1, lo), np.full(n, mid), np.full(n - 1, hi)], [-1, 0, 1])


@pytest.mark.parametrize("n", [5, 11])
def test_stencil_families_equal_kronecker_forms(n):
    import scipy.sparse as sp

    I = sp.identity(n)
    T = _tri(n, -1.0, 2.0, -1.0)
    J = _tri(n, 1.0, 1.0, 1.0)
    T4 = sp.diags([np.full(n - 2, 1.0), np.full(n - 1, -16.0), np.full(n, 30.0), np.full(n - 1, -16.0),
                   np.full(n - 2, 1.0)], [-2, -1, 0, 1, 2])
    forms = {
        "laplace2d_5": sp.kron(I, T) + sp.kron(T, I),
        "fourth2d_9": sp.kron(I, T4) + sp.kron(T4, I),
        "box2d_9": 9.0 * sp.identity(n * n) - sp.kron(J, J),
        "laplace3d_7": sp.kron(I, sp.kron(I, T)) + sp.kron(I, sp.kron(T, I)) + sp.kron(T, sp.kron(I, I)),
        "box3d_27": 27.0 * sp.identity(n ** 3) - sp.kron(J, sp.kron(J, J)),
    }
    for name, K in forms.items():
        A = P.stencil_matrix(name, n).scipy()
        assert abs(A - K).max() == 0.0, name
