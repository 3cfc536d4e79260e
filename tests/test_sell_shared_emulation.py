"""CPU restatement of the shared-offset sliced SpMV layout (no GPU).

Builds, as the library's matrix set-up does, each 64-row slice's sorted union
of column offsets c - r, the slot values (0 for an absent neighbour) and the
choice rule (strictly increasing columns in every row, slots at most 1.25x
the per-row copy's), then sums every row over all of its slice's slots in
slot order with the gather index clamped to [0, n), in fp32 and fp64, and
checks the sums bitwise against the CSR row sums in column order -- the
claim the kernel's comment makes (an absent slot adds 0 * x = +-0 to a sum
that started at +0).  x includes exact zeros and negative zeros."""
import numpy as np
import pytest

from paper_2109_01232_amd import problems as P

SELL_C = 64
GROWTH = 1.25


def shared_layout(A):
    """(ok, offsets per slice, slot values per slice) as the set-up builds them."""
    rp, ci = A.rowptr, A.colidx
    ns = -(-A.n // SELL_C)
    offs, slots_shared, slots_row = [], 0, 0
    for sl in range(ns):
        rows = range(sl * SELL_C, min(A.n, (sl + 1) * SELL_C))
        U = set()
        kmax = 0
        for r in rows:
            d = ci[rp[r]:rp[r + 1]] - r
            if len(d) > 1 and np.any(np.diff(d) <= 0):
                return False, None
            U.update(d.tolist())
            kmax = max(kmax, len(d))
        offs.append(np.array(sorted(U), dtype=np.int64))
        slots_shared += len(U)
        slots_row += kmax
    return slots_shared <= GROWTH * slots_row, offs


def spmv_shared(A, offs, x, dt):
    rp, ci = A.rowptr, A.colidx
    v = A.vals.astype(dt)
    y = np.zeros(A.n, dt)
    for sl, U in enumerate(offs):
        for r in range(sl * SELL_C, min(A.n, (sl + 1) * SELL_C)):
            entries = dict(zip((ci[rp[r]:rp[r + 1]] - r).tolist(), v[rp[r]:rp[r + 1]]))
            s = dt(0)
            for o in U.tolist():
                c = min(max(r + o, 0), A.n - 1)
                s = dt(s + dt(dt(entries.get(o, 0.0)) * x[c]))
            y[r] = s
    return y


def spmv_csr(A, x, dt):
    rp, ci = A.rowptr, A.colidx
    v = A.vals.astype(dt)
    y = np.zeros(A.n, dt)
    for r in range(A.n):
        s = dt(0)
        for p in range(rp[r], rp[r + 1]):
            s = dt(s + dt(v[p] * x[ci[p]]))
        y[r] = s
    return y


def holed(A0, seed):
    import scipy.sparse as sp
    S = A0.scipy().tocoo()
    rng = np.random.default_rng(seed)
    keep = (S.row == S.col) | (rng.uniform(size=S.nnz) > 0.05)
    r, c, v = S.row[keep], S.col[keep], S.data[keep].copy()
    v[rng.choice(len(v), 10, replace=False)] = 0.0
    keep = ~np.isin(r, [3, A0.n - 1])
    H = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(A0.n, A0.n))
    H.sort_indices()
    return P.CSR(A0.n, H.indptr.astype(np.int32), H.indices.astype(np.int32), H.data)


CASES = {
    "laplace2d_5": lambda: P.stencil_matrix("laplace2d_5", 13),
    "box3d_27": lambda: P.stencil_matrix("box3d_27", 7),
    "varcoef27": lambda: P.varcoef27(6, 3),
    "convdiff_ragged": lambda: P.conv_diff(2, 11, 25.0, (1.0, -0.5)),
    "holed_laplace3d": lambda: holed(P.stencil_matrix("laplace3d_7", 7), 1),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_shared_layout_sums_are_csr_sums(case):
    A = CASES[case]()
    ok, offs = shared_layout(A)
    assert ok
    x = np.random.default_rng(7).uniform(-1, 1, A.n)
    x[::5] = 0.0
    x[2::7] = -0.0
    for dt in (np.float32, np.float64):
        xs = x.astype(dt)
        y3, yc = spmv_shared(A, offs, xs, dt), spmv_csr(A, xs, dt)
        assert np.array_equal(y3.view(np.uint8), yc.view(np.uint8)), (case, dt)


def test_shared_layout_rejections():
    A = P.stencil_matrix("laplace2d_5", 12)
    # a row stored in decreasing column order
    cols = A.colidx.copy()
    lo, hi = A.rowptr[20], A.rowptr[21]
    cols[lo:hi] = cols[lo:hi][::-1]
    assert not shared_layout(P.CSR(A.n, A.rowptr, cols, A.vals))[0]
    # a repeated column
    cols = A.colidx.copy()
    cols[lo + 1] = cols[lo]
    assert not shared_layout(P.CSR(A.n, A.rowptr, cols, A.vals))[0]
    # rows of a slice that each couple to their own far column: the union grows past 1.25x
    import scipy.sparse as sp
    S = A.scipy() + sp.csr_matrix((np.full(A.n, -1e-3), (np.arange(A.n), (np.arange(A.n) * 37 + 11) % A.n)),
                                  shape=(A.n, A.n))
    S = S.tocsr()
    S.sort_indices()
    assert not shared_layout(P.CSR(A.n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data))[0]
