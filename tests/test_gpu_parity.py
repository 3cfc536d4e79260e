"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: bitwise for the fp32/fp64 SpMV on stencil rows (both sum each row in
column order from identically rounded products); final fp64 relative
residual <= rtol for both sides; solution agreement 1e-8 relative, compared
at a parity tolerance rtol = 1e-12 (the parity system has condition number
~1e3, so two solutions with residual 1e-12 agree to ~1e-9; measured GPU-oracle
gaps 1e-16..7e-12); cycle-normalised implicit residual histories within 1e-5
for fp32 cycles (measured gaps up to 2e-7); for bf16-stored bases a relative
bar on every step, |d rho_j| <= BF16_REL rho_j + BF16_FLOOR (see
``bf16_hist_ok``); the fp32 polynomial apply element by element against the
oracle's fp32 product form, max |dy| <= max(8 d u32, 2.5 e) max |y| with e the
oracle's own element-wise fp32 error against the fp64 evaluation (two fp32
evaluations of d product-form steps each within e of the exact value;
measured 1.7e-7 at d = 1 .. 6.1e-6 at d = 40).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import linalg as L
from oracle import poly as PO
from paper_2109_01232_amd import binding as B
from paper_2109_01232_amd import problems as P

from gpu_common import bf16_hist_ok, cycle_slices, dev_tensor, rel, say

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
def conv64():
    s = P.parity_system()
    return s, B.Matrix.from_csr(s.A)


def ragged_matrix_with_long_row(n=1500, seed=0):
    """Random CSR with empty rows and one row longer than a tile (6144 nnz)."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        if i % 97 == 5:
            rows.append(np.array([], dtype=np.int64))
        elif i == 700:
            rows.append(np.sort(rng.choice(n, min(n, 1400), replace=False)))
        else:
            k = rng.integers(1, 12)
            rows.append(np.sort(rng.choice(n, k, replace=False)))
    # make the long row longer than a tile by repeating the matrix width
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i, r in enumerate(rows):
        cols.append(r)
        vals.append(rng.standard_normal(len(r)))
        rowptr[i + 1] = rowptr[i] + len(r)
    return P.CSR(n, rowptr.astype(np.int32), np.concatenate(cols).astype(np.int32), np.concatenate(vals))


def long_row_matrix(n=8000, seed=1):
    rng = np.random.default_rng(seed)
    rowptr = [0]
    cols, vals = [], []
    for i in range(n):
        k = 7000 if i == 3 else (0 if i % 50 == 7 else rng.integers(2, 9))
        c = np.sort(rng.choice(n, k, replace=False))
        cols.append(c)
        vals.append(rng.standard_normal(k))
        rowptr.append(rowptr[-1] + k)
    return P.CSR(n, np.array(rowptr, dtype=np.int32), np.concatenate(cols).astype(np.int32), np.concatenate(vals))


def far_column_matrix(side=264, seed=2, far=True):
    """2D convection-diffusion on side^2 >= 65473 rows (enough slices for the
    sliced SpMV + projection kernel) plus one coupling per seventh row, each
    at its own distance (so the rows of a slice do not share their column
    offsets): far=True about n/2 away, too far for 16-bit offsets, so the
    sliced copy keeps 32-bit columns; far=False 100..3000 columns away, so it
    keeps 16-bit offsets.  Still diagonally dominant."""
    import scipy.sparse as sp
    A0 = P.conv_diff(2, side, 20.0, (1.0, 0.3))
    n = A0.n
    rng = np.random.default_rng(seed)
    r = np.arange(0, n, 7)
    if far:
        c = (r + n // 2 + rng.integers(-1000, 1000, len(r))) % n
    else:
        d = rng.choice([-1, 1], len(r)) * rng.integers(100, 3000, len(r))
        c = np.where((r + d < 0) | (r + d >= n), r - d, r + d)
    S = A0.scipy() + sp.csr_matrix((-1e-3 * rng.uniform(0.5, 1.0, len(r)), (r, c)), shape=(n, n))
    S = S.tocsr()
    S.sort_indices()
    return P.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data), S


# ---------------------------------------------------------------------------
# SpMV
# ---------------------------------------------------------------------------

# layout the library picks: 3 = sliced copy with one column-offset list per
# slice (stencils), 2 = with 16-bit column offsets per entry, 1 = with 32-bit
# columns, 0 = CSR row tiles only (a row longer than 512)
SPMV_LAYOUT = {"conv64": 3, "ragged2d": 3, "aniso3d": 3, "varcoef27": 3, "irregular": 0, "longrow": 0, "farcols": 1,
               "nearcols": 2}


@pytest.mark.parametrize("case", ["conv64", "ragged2d", "aniso3d", "varcoef27", "irregular", "longrow", "farcols",
                                  "nearcols"])
def test_spmv_parity(case):
    say("spmv", case)
    if case == "conv64":
        A = P.parity_system().A
    elif case == "ragged2d":
        A = P.conv_diff(2, 37, 25.0, (1.0, -0.5))
    elif case == "aniso3d":
        A = P.conv_diff(3, 23, 10.0, (1, 1, 1), (1, 1, 1e-2))
    elif case == "varcoef27":
        A = P.varcoef27(17, 3)
    elif case == "irregular":
        A = ragged_matrix_with_long_row()
    elif case == "farcols":
        A, _ = far_column_matrix()
    elif case == "nearcols":
        A, _ = far_column_matrix(far=False)
    else:
        A = long_row_matrix()
    M = B.Matrix.from_csr(A)
    assert M.layout == SPMV_LAYOUT[case]
    x = np.random.default_rng(1).uniform(-1, 1, A.n)
    for prec, dt in (("fp64", np.float64), ("fp32", np.float32)):
        xd = dev_tensor(x.astype(dt))
        yd = torch.empty_like(xd)
        B.gmresir_spmv(M, xd, yd, prec)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        ref = L.spmv(L.csr_matrix(A, dt), x.astype(dt))
        if case == "longrow":
            # the long row is a block-wide reduction: tolerance for it, bitwise elsewhere
            mask = np.ones(A.n, bool)
            mask[3] = False
            assert np.array_equal(y[mask], ref[mask])
            lo, hi = A.rowptr[3], A.rowptr[4]
            scale = np.abs(A.vals[lo:hi] * x[A.colidx[lo:hi]]).sum()
            eps = np.finfo(dt).eps
            assert abs(float(y[3]) - float(ref[3])) <= 8 * eps * scale
        else:
            assert np.array_equal(y, ref), (prec, np.abs(y - ref).max())


def holed_stencil_matrix(side=20, seed=5):
    """The 7-point Laplacian on side^3 with about 3 % of its off-diagonal
    entries removed at random, a few explicit zeros kept as entries, and three
    empty rows (one of them the last row): the rows of a slice then hold
    different subsets of the slice's offsets, so the shared-offset layout
    stores zeros in the middle of rows, and a slice has a row with no entry."""
    A0 = P.stencil_matrix("laplace3d_7", side)
    S = A0.scipy().tocoo()
    rng = np.random.default_rng(seed)
    keep = (S.row == S.col) | (rng.uniform(size=S.nnz) > 0.03)
    r, c, v = S.row[keep], S.col[keep], S.data[keep].copy()
    v[rng.choice(len(v), 20, replace=False)] = 0.0  # explicit zeros
    empty = np.array([5, 777, A0.n - 1])
    keep = ~np.isin(r, empty)
    import scipy.sparse as sp
    H = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(A0.n, A0.n))
    H.sort_indices()
    return P.CSR(A0.n, H.indptr.astype(np.int32), H.indices.astype(np.int32), H.data)


def coupled_stencil_matrix(extra_offsets, side=40):
    """5-point convection-diffusion on side^2 plus, in every 64-row slice,
    couplings of its rows to columns r + o for the offsets o in
    extra_offsets, taken in turn row by row (so a slice's offset union grows
    by len(extra_offsets) while no row gets more than one extra entry)."""
    import scipy.sparse as sp
    A0 = P.conv_diff(2, side, 20.0, (1.0, 0.3))
    n = A0.n
    r = np.arange(n)
    o = np.array(extra_offsets)[r % len(extra_offsets)]
    keep = (r + o >= 0) & (r + o < n)
    S = A0.scipy() + sp.csr_matrix((np.full(keep.sum(), -1e-3), (r[keep], (r + o)[keep])), shape=(n, n))
    S = S.tocsr()
    S.sort_indices()
    return P.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)


@pytest.mark.parametrize("case,layout", [("two_extra", 3), ("three_extra", 2), ("unsorted_row", 2),
                                         ("repeated_column", 2)])
def test_spmv_layout_choice(case, layout):
    """The shared-offset layout is taken only while a slice's offset union
    stays within 1.25x the slots of the per-row copy and every row's columns
    strictly increase: 5 + 2 offsets over rows of at most 6 entries (7/6) keep
    it, 5 + 3 (8/6) do not; a row stored in decreasing column order, or with a
    column repeated, keeps the per-entry copy (summed in stored order).  The
    SpMV is bitwise the CSR sums in stored order either way."""
    if case == "two_extra":
        A = coupled_stencil_matrix([3, 5])
    elif case == "three_extra":
        A = coupled_stencil_matrix([3, 5, 7])
    else:
        A = coupled_stencil_matrix([3, 5])
        lo, hi = A.rowptr[100], A.rowptr[101]
        cols, vals = A.colidx.copy(), A.vals.copy()
        if case == "unsorted_row":
            cols[lo:hi], vals[lo:hi] = cols[lo:hi][::-1].copy(), vals[lo:hi][::-1].copy()
        else:
            cols[lo + 1] = cols[lo]  # the row's second entry repeats its first column
        A = P.CSR(A.n, A.rowptr, cols, vals)
    M = B.Matrix.from_csr(A)
    say("spmv layout choice", case, M.layout)
    assert M.layout == layout
    x = np.random.default_rng(4).uniform(-1, 1, A.n)
    for prec, dt in (("fp64", np.float64), ("fp32", np.float32)):
        xd = dev_tensor(x.astype(dt))
        yd = torch.empty_like(xd)
        B.gmresir_spmv(M, xd, yd, prec)
        torch.cuda.synchronize()
        ref = L.spmv(L.csr_matrix(A, dt), x.astype(dt))
        assert np.array_equal(yd.cpu().numpy(), ref), (case, prec)
    M.close()


def test_spmv_shared_layout_with_holes():
    """Shared-offset layout on rows that miss some of their slice's offsets,
    explicit zeros and empty rows: bitwise the CSR row sums, both precisions
    (including x with exact zeros and negative zeros)."""
    A = holed_stencil_matrix()
    assert A.nnz < P.stencil_nnz("laplace3d_7", 20)
    M = B.Matrix.from_csr(A)
    assert M.layout == 3
    say("spmv shared layout with holes")
    x = np.random.default_rng(2).uniform(-1, 1, A.n)
    x[::11] = 0.0
    x[3::13] = -0.0
    for prec, dt in (("fp64", np.float64), ("fp32", np.float32)):
        xd = dev_tensor(x.astype(dt))
        yd = torch.empty_like(xd)
        B.gmresir_spmv(M, xd, yd, prec)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        ref = L.spmv(L.csr_matrix(A, dt), x.astype(dt))
        assert np.array_equal(y, ref), (prec, np.abs(y - ref).max())
        assert np.all(y[[5, 777, A.n - 1]] == 0)
    M.close()


# ---------------------------------------------------------------------------
# full solves on the parity system (64x64 convection-diffusion)
# ---------------------------------------------------------------------------

def test_fp64_gmres_matches_oracle(conv64):
    s, M = conv64
    say("fp64 gmres(50) conv64")
    b = dev_tensor(s.b)
    x, d, h = B.solve(M, b, restart=50, inner="fp64", rtol=1e-10, check_mode=0, hist_cap=100000)
    ref = L.gmres(s.A, s.b, m=50, rtol=1e-10, check_mode=0)
    xs = x.cpu().numpy()
    assert d["status"] == B.OK and ref.status == L.OK
    assert d["iters"] == ref.iters and d["refinements"] == ref.refinements
    true = np.linalg.norm(s.b - s.A.scipy() @ xs) / np.linalg.norm(s.b)
    assert true <= 1e-10 and d["rel_resid_true"] == pytest.approx(true, rel=1e-6)
    assert rel(xs, ref.x) <= 1e-8
    assert rel(xs, s.u) <= 1e-6
    # fp64 on both sides: the first cycles agree to rounding; later cycles
    # start from residuals that carry the iterates' rounding noise
    href = np.array(ref.hist)
    assert np.max(np.abs(h[:150] - href[:150])) <= 1e-10
    assert np.max(np.abs(h - href)) <= 1e-5


def test_gmres_ir_fp32_matches_oracle(conv64):
    s, M = conv64
    say("ir fp32 conv64")
    b = dev_tensor(s.b)
    x, d, h = B.solve(M, b, restart=50, inner="fp32", rtol=1e-12, check_mode=0, hist_cap=100000)
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-12, inner="fp32", check_mode=0)
    xs = x.cpu().numpy()
    assert d["status"] == B.OK
    assert d["rel_resid_true"] <= 1e-12 and ref.rel_resid <= 1e-12
    assert rel(xs, ref.x) <= 1e-8
    assert d["iters"] % 50 == 0  # paper mode: convergence checked at restarts only
    # same number of restarts up to one (rounding), first cycle identical input
    assert abs(d["refinements"] - ref.refinements) <= 1
    assert np.max(np.abs(h[:50] - np.array(ref.hist[:50]))) <= HIST_TOL_FP32


def test_ir_cycle_histories_from_oracle_iterates(conv64):
    """Per-cycle parity on the same input r_i: the GPU restarts from the
    oracle's own iterate x_i and runs one fp32 cycle; its history is compared
    with the fp64 oracle's cycle i+1 (the gate oracle runs the inner solve in
    fp64)."""
    s, M = conv64
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-12, inner="fp64", check_mode=0, keep_iterates=True)
    cycles = cycle_slices(ref.hist, ref.cycle_starts)
    b = dev_tensor(s.b)
    for i in (0, 2, 4, 6):
        say("ir cycle replay", i)
        x0 = dev_tensor(ref.xs[i])
        x, d, h = B.solve(M, b, x0=x0, restart=50, inner="fp32", rtol=1e-14, check_mode=0, max_iters=50,
                          hist_cap=50)
        assert d["iters"] == 50
        assert np.max(np.abs(h - cycles[i + 1])) <= HIST_TOL_FP32, i


def test_check_mode_implicit_exit(conv64):
    s, M = conv64
    say("check_mode 1")
    b = dev_tensor(s.b)
    x0, d0, _ = B.solve(M, b, restart=50, inner="fp32", rtol=1e-10, check_mode=0)
    x1, d1, _ = B.solve(M, b, restart=50, inner="fp32", rtol=1e-10, check_mode=1)
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", check_mode=1)
    assert d1["status"] == B.OK and d1["rel_resid_true"] <= 1e-10
    assert d1["iters"] <= d0["iters"] and d0["iters"] - d1["iters"] <= 49
    assert abs(d1["iters"] - ref.iters) <= 10


def test_bf16_basis(conv64):
    s, M = conv64
    say("bf16 basis conv64")
    b = dev_tensor(s.b)
    x, d, h = B.solve(M, b, restart=50, inner="fp32", basis="bf16", rtol=1e-10, check_mode=0, hist_cap=100000)
    ref = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32", basis="bf16", check_mode=0)
    assert d["status"] == B.OK and d["rel_resid_true"] <= 1e-10
    ok, info = bf16_hist_ok(h[:50], ref.hist[:50])
    assert ok, info
    assert abs(d["refinements"] - ref.refinements) <= 2
    assert rel(x.cpu().numpy(), s.u) <= 1e-6


def test_deterministic(conv64):
    s, M = conv64
    say("determinism")
    b = dev_tensor(s.b)
    xa, da, _ = B.solve(M, b, restart=30, inner="fp32", rtol=1e-10)
    xb, db, _ = B.solve(M, b, restart=30, inner="fp32", rtol=1e-10)
    assert torch.equal(xa, xb) and da["iters"] == db["iters"]


def test_graph_replay_matches_direct_launches(conv64):
    """Systems up to 2^18 rows run their cycles as a recorded HIP graph,
    replayed once per refinement with eager kernels (residual, cast, host
    read) in between; profiling switches to direct launches.  Both give the
    same bits on every refinement (fp32 inner, fp64 inner, bf16 basis, a
    multi-cycle inner cap, and two solves in a row)."""
    s, M = conv64
    b = dev_tensor(s.b)
    for kw in (dict(restart=50, inner="fp32"), dict(restart=30, inner="fp64"),
               dict(restart=40, inner="fp32", basis="bf16"), dict(restart=20, inner="fp32", inner_cap=60)):
        say("graph vs direct", kw)
        xg, dg, hg = B.solve(M, b, rtol=1e-10, hist_cap=20000, **kw)
        xg2, dg2, _ = B.solve(M, b, rtol=1e-10, **kw)
        xd, dd, hd = B.solve(M, b, rtol=1e-10, hist_cap=20000, profile=1, **kw)
        assert dg["refinements"] >= 3
        assert torch.equal(xg, xd) and torch.equal(xg, xg2)
        assert dg["iters"] == dd["iters"] and dg["refinements"] == dd["refinements"]
        assert np.array_equal(hg, hd)


def test_resume_equals_single_call(conv64):
    s, M = conv64
    say("resume")
    b = dev_tensor(s.b)
    full, df, _ = B.solve(M, b, restart=30, inner="fp64", rtol=1e-10, check_mode=0)
    part, dp, _ = B.solve(M, b, restart=30, inner="fp64", rtol=1e-10, check_mode=0, max_iters=90)
    assert dp["status"] == B.NOT_CONVERGED and dp["iters"] == 90
    rest, dr, _ = B.solve(M, b, x0=part, restart=30, inner="fp64", rtol=1e-10, check_mode=0)
    assert dp["iters"] + dr["iters"] == df["iters"]
    assert torch.equal(rest, full)


def test_inner_cap_multi_cycle(conv64):
    s, M = conv64
    say("inner cap 75, m 25")
    b = dev_tensor(s.b)
    x, d, _ = B.solve(M, b, restart=25, inner="fp32", inner_cap=75, rtol=1e-10)
    ref = L.gmres_ir(s.A, s.b, m=25, rtol=1e-10, inner="fp32", cap=75, check_mode=1)
    assert d["status"] == B.OK and d["rel_resid_true"] <= 1e-10
    assert d["cycles"] > d["refinements"]
    assert abs(d["refinements"] - ref.refinements) <= 1


@pytest.mark.parametrize("m", [1, 7, 64, 70, 130])
def test_restart_lengths_and_fallbacks(m):
    """m=1 (degenerate), ragged, and restart lengths past the fused kernels'
    column limits (fp64 56, fp32 128) which take the fallback kernels."""
    A = P.conv_diff(2, 20, 15.0, (1.0, 1.0))
    u = np.random.default_rng(m).uniform(-1, 1, A.n)
    bb = A.scipy() @ u
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    for inner in ("fp64", "fp32"):
        say("restart", m, inner)
        maxit = 4000 if m > 1 else 20000
        x, d, h = B.solve(M, b, restart=m, inner=inner, rtol=1e-12, max_iters=maxit, check_mode=1,
                          hist_cap=200)
        ref = (L.gmres(A, bb, m=m, rtol=1e-12, max_iters=maxit, check_mode=1) if inner == "fp64" else
               L.gmres_ir(A, bb, m=m, rtol=1e-12, inner="fp32", max_iters=maxit, check_mode=1))
        assert d["status"] == ref.status
        if d["status"] == B.OK:
            assert d["rel_resid_true"] <= 1e-12
            assert rel(x.cpu().numpy(), ref.x) <= 1e-8
        # first cycle only: after an implicit early exit the next cycle's input is
        # the rounding noise of the correction, which differs between the sides
        k = min(len(h), ref.cycle_starts[1] if len(ref.cycle_starts) > 1 else len(ref.hist), m)
        tol = 1e-10 if inner == "fp64" else HIST_TOL_FP32
        assert np.max(np.abs(h[:k] - np.array(ref.hist[:k]))) <= tol


@pytest.mark.parametrize("m", [20, 70, 100, 130])
@pytest.mark.parametrize("inner,basis", [("fp64", "fp64"), ("fp32", "fp32"), ("fp32", "bf16")])
def test_ragged_rows_every_basis_width(m, inner, basis):
    """n = 37^2 = 1369 (not a multiple of the 4- and 8-row groups of the
    vector loads, so the padded rows must be masked), every column-count
    class of the fused kernels (4/8 waves, packed 8-row bf16 loads) and the
    fallbacks past 128 columns: the first cycle against the oracle's."""
    A = P.conv_diff(2, 37, 40.0, (1.0, -0.5))
    u = np.random.default_rng(m).uniform(-1, 1, A.n)
    bb = A.scipy() @ u
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    say("ragged", m, inner, basis)
    x, d, h = B.solve(M, b, restart=m, inner=inner, basis=basis, rtol=1e-10, check_mode=0, max_iters=20000,
                      hist_cap=20000)
    if inner == "fp64":
        ref = L.gmres(A, bb, m=m, rtol=1e-10, check_mode=0, max_iters=m)
        tol = 1e-10
    else:
        ref = L.gmres_ir(A, bb, m=m, rtol=1e-10, inner="fp32", basis=basis, check_mode=0, max_iters=m)
        tol = HIST_TOL_FP32
    k = min(m, len(ref.hist))
    if basis == "bf16":
        ok, info = bf16_hist_ok(h[:k], ref.hist[:k])
        assert ok, info
    else:
        assert np.max(np.abs(h[:k] - np.array(ref.hist[:k]))) <= tol
    assert d["status"] == B.OK and d["rel_resid_true"] <= 1e-10
    assert np.linalg.norm(bb - A.scipy() @ x.cpu().numpy()) / np.linalg.norm(bb) <= 1e-10


@pytest.mark.parametrize("m", [20, 64, 100, 128])
@pytest.mark.parametrize("inner,basis", [("fp64", "fp64"), ("fp32", "fp32"), ("fp32", "bf16")])
def test_sliced_path_ragged_rows(m, inner, basis):
    """The fused sliced kernels (shared-offset layout) on n = 259^2 = 67081
    rows (1049 slices; n = 1 mod 4 and 9 mod 64, so the last row group of
    the branch-free basis loads straddles n and only the mask keeps the
    padded rows out): every column-count class, the first cycle against the
    oracle's, and the whole solve's fp64 residual for the fp32 and fp64
    bases."""
    A = P.conv_diff(2, 259, 30.0, (1.0, -0.5))
    u = np.random.default_rng(m).uniform(-1, 1, A.n)
    bb = A.scipy() @ u
    M = B.Matrix.from_csr(A)
    assert M.layout == 3
    b = dev_tensor(bb)
    say("sliced ragged", m, inner, basis)
    x, d, h = B.solve(M, b, restart=m, inner=inner, basis=basis, rtol=1e-10, check_mode=0, max_iters=m,
                      hist_cap=m + 8)
    if inner == "fp64":
        ref = L.gmres(A, bb, m=m, rtol=1e-10, check_mode=0, max_iters=m)
        tol = 1e-10
    else:
        ref = L.gmres_ir(A, bb, m=m, rtol=1e-10, inner="fp32", basis=basis, check_mode=0, max_iters=m)
        tol = HIST_TOL_FP32
    k = min(m, len(ref.hist))
    if basis == "bf16":
        ok, info = bf16_hist_ok(h[:k], ref.hist[:k])
        assert ok, info
    else:
        assert np.max(np.abs(h[:k] - np.array(ref.hist[:k]))) <= tol
        x, d, _ = B.solve(M, b, restart=m, inner=inner, basis=basis, rtol=1e-10, check_mode=1, max_iters=50000)
        assert d["status"] == B.OK
        assert np.linalg.norm(bb - A.scipy() @ x.cpu().numpy()) / np.linalg.norm(bb) <= 1e-10
    M.close()


def test_row_tiled_path_solve():
    """A row longer than the sliced-ELLPACK limit (512) keeps the matrix on
    the row-tiled CSR kernels (LDS-staged products, block-reduced long row):
    fp32 IR and fp64 GMRES against the oracle on such a system."""
    A0 = P.conv_diff(2, 40, 20.0, (1.0, 0.3))
    S = A0.scipy().tolil()
    cols = np.arange(0, A0.n, 2)[:700]
    S[5, cols] = S[5, cols].toarray() + 1e-3  # a 700-entry row, still diagonally dominant
    S = S.tocsr()
    S.sort_indices()
    A = P.CSR(A0.n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)
    u = np.random.default_rng(11).uniform(-1, 1, A.n)
    bb = S @ u
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    for inner in ("fp32", "fp64"):
        say("row-tiled solve", inner)
        x, d, h = B.solve(M, b, restart=30, inner=inner, rtol=1e-10, check_mode=0, hist_cap=20000)
        ref = (L.gmres(A, bb, m=30, rtol=1e-10, check_mode=0, max_iters=30) if inner == "fp64" else
               L.gmres_ir(A, bb, m=30, rtol=1e-10, inner="fp32", check_mode=0, max_iters=30))
        tol = 1e-10 if inner == "fp64" else HIST_TOL_FP32
        assert np.max(np.abs(h[:30] - np.array(ref.hist[:30]))) <= tol
        assert d["status"] == B.OK
        assert np.linalg.norm(bb - S @ x.cpu().numpy()) / np.linalg.norm(bb) <= 1e-10


@pytest.mark.parametrize("far", [True, False])
def test_far_column_solve(far):
    """Rows of a slice that do not share their column offsets keep the
    per-entry sliced copy -- 32-bit columns beyond the 16-bit offset range
    (far), 16-bit offsets otherwise; at 69696 rows the fused SpMV +
    projection runs its sliced kernel on them.  First cycle against the
    oracle's, then the fp64 residual."""
    A, S = far_column_matrix(far=far)
    u = np.random.default_rng(12).uniform(-1, 1, A.n)
    bb = S @ u
    M = B.Matrix.from_csr(A)
    assert M.layout == (1 if far else 2)
    b = dev_tensor(bb)
    for inner in ("fp32", "fp64"):
        say("far-column solve", far, inner)
        x, d, h = B.solve(M, b, restart=30, inner=inner, rtol=1e-10, check_mode=0, hist_cap=20000)
        ref = (L.gmres(A, bb, m=30, rtol=1e-10, check_mode=0, max_iters=30) if inner == "fp64" else
               L.gmres_ir(A, bb, m=30, rtol=1e-10, inner="fp32", check_mode=0, max_iters=30))
        tol = 1e-10 if inner == "fp64" else HIST_TOL_FP32
        assert np.max(np.abs(h[:30] - np.array(ref.hist[:30]))) <= tol
        assert d["status"] == B.OK
        assert np.linalg.norm(bb - S @ x.cpu().numpy()) / np.linalg.norm(bb) <= 1e-10


def test_exact_breakdown_small_system():
    """n = 12 < m: GMRES terminates in at most n steps with a lucky breakdown."""
    A = P.conv_diff(2, 3, 5.0, (1.0, 0.0))
    M = B.Matrix.from_csr(A)
    bb = np.arange(1.0, A.n + 1)
    b = dev_tensor(bb)
    for inner in ("fp64", "fp32"):
        say("breakdown", inner)
        x, d, _ = B.solve(M, b, restart=30, inner=inner, rtol=1e-10)
        assert d["status"] == B.OK and d["rel_resid_true"] <= 1e-10
        assert d["iters"] <= 2 * A.n
        assert rel(x.cpu().numpy(), np.linalg.solve(A.scipy().toarray(), bb)) <= 1e-8


# ---------------------------------------------------------------------------
# failure handling (forced from the host)
# ---------------------------------------------------------------------------

def test_failure_modes(conv64):
    s, M = conv64
    b = dev_tensor(s.b)
    say("nan rhs")
    bn = s.b.copy()
    bn[17] = np.nan
    with pytest.raises(B.GmresirError) as e:
        B.gmresir_solve(M, dev_tensor(bn), torch.zeros_like(b), B.make_params(restart=20))
    assert e.value.status == B.ERR_NUMERIC
    say("max_iters")
    x = torch.zeros_like(b)
    st, d, _ = B.gmresir_solve(M, b, x, B.make_params(restart=20, max_iters=40))
    assert st == B.NOT_CONVERGED and d["iters"] == 40 and d["rel_resid_true"] < 1
    say("stagnation")
    x = torch.zeros_like(b)
    res = B.Result()
    import ctypes
    p = B.make_params(restart=50, rtol=1e-20, max_iters=5000)
    ws = torch.empty(B.gmresir_workspace_bytes(M, p), dtype=torch.uint8, device="cuda")
    hist = np.zeros(5000)
    st = B.lib().gmresir_solve(M.handle, B._ptr(b), B._ptr(x), ctypes.byref(p), None, B._ptr(ws), ws.numel(),
                               ctypes.byref(res), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 5000,
                               B._stream())
    print("stagnation case:", st, res.as_dict(), B.last_error(), flush=True)
    assert st == B.STAGNATED and res.rel_resid_true <= 1e-12
    say("zero rhs")
    x = torch.ones_like(b)
    st, d, _ = B.gmresir_solve(M, torch.zeros_like(b), x, B.make_params())
    assert st == B.OK and not torch.any(x)
    say("bad params")
    with pytest.raises(B.GmresirError) as e:
        B.gmresir_solve(M, b, torch.zeros_like(b), B.make_params(inner="fp64", basis="bf16"))
    assert e.value.status == B.ERR_INVALID_ARG
    say("small workspace")
    p = B.make_params()
    need = B.gmresir_workspace_bytes(M, p)
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    res = B.Result()
    import ctypes
    st = B.lib().gmresir_solve(M.handle, B._ptr(b), B._ptr(torch.zeros_like(b)), ctypes.byref(p), None,
                               B._ptr(ws), ws.numel(), ctypes.byref(res), None, 0, B._stream())
    assert st == B.ERR_WORKSPACE


# ---------------------------------------------------------------------------
# polynomial preconditioner
# ---------------------------------------------------------------------------

def aniso_small(n=14, seed=0):
    A = P.conv_diff(3, n, 10.0, (1, 1, 1), (1, 1, 1e-2))
    u = np.random.default_rng(seed).uniform(-1, 1, A.n)
    return A, A.scipy() @ u


@pytest.mark.parametrize("d", [1, 2, 5, 10, 20, 40])
def test_poly_apply_matches_oracle(d):
    """Same roots on both sides (drawn from the oracle), fp32 product form."""
    A, _ = aniso_small()
    roots = PO.poly_roots(A, d, seed=4, dtype=np.float64)
    M = B.Matrix.from_csr(A)
    v = np.random.default_rng(d).standard_normal(A.n).astype(np.float32)
    vd = dev_tensor(v)
    yd = torch.empty_like(vd)
    say("poly apply", d)
    B.gmresir_poly_apply(M, roots, vd, yd)
    torch.cuda.synchronize()
    ref = PO.apply_product_form(L.csr_matrix(A, np.float32), roots, v, np.float32)
    ref64 = PO.apply_product_form(L.csr_matrix(A, np.float64), roots, v.astype(np.float64), np.float64)
    got = yd.cpu().numpy()
    # element by element against the oracle's fp32 evaluation of the same
    # roots: two fp32 evaluations, each within the fp32 rounding error e of the
    # exact (fp64) value, differ by at most 2 e
    scale = np.abs(ref).max()
    gap = np.abs(got - ref).max() / scale
    e_or = np.abs(ref - ref64).max() / scale
    assert gap <= max(8 * d * U32, 2.5 * e_or), (gap, e_or)
    assert np.abs(got - ref64).max() / scale <= max(8 * d * U32, 2.5 * e_or)


def test_poly_setup_matches_oracle():
    A, _ = aniso_small()
    M = B.Matrix.from_csr(A)
    start = PO.start_vector(A.n, 11)
    say("poly setup, given start")
    roots, hbar = B.gmresir_poly_setup(M, 10, start=dev_tensor(start), with_hbar=True)
    ref_cyc = L.gmres_cycle(lambda z: L.spmv(L.csr_matrix(A, np.float32), z), start.astype(np.float32), 11,
                            np.float32)
    assert rel(hbar, ref_cyc.Hbar) <= 1e-5
    ref = PO.poly_roots(A, 10, start=start, dtype=np.float32)
    assert len(roots) == 11
    assert np.allclose(np.sort_complex(roots), np.sort_complex(ref), rtol=1e-3, atol=1e-3 * np.abs(ref).max())
    say("poly setup, splitmix start")
    r2 = B.gmresir_poly_setup(M, 10, seed=11)
    assert np.allclose(np.sort_complex(r2), np.sort_complex(roots), rtol=1e-5, atol=1e-5 * np.abs(ref).max())


def test_poly_preconditioned_solve():
    A, bb = aniso_small()
    M = B.Matrix.from_csr(A)
    b = dev_tensor(bb)
    say("poly solve d=10, roots built on the GPU")
    groots = B.gmresir_poly_setup(M, 10, seed=3)
    xg, dg, _ = B.solve(M, b, restart=30, inner="fp32", rtol=1e-10, poly_degree=10, poly_roots=groots)
    assert dg["status"] == B.OK and dg["rel_resid_true"] <= 1e-10
    # parity on identical inputs: the oracle builds the roots, both sides use them
    roots = PO.poly_roots(A, 10, start=PO.start_vector(A.n, 3), dtype=np.float32)
    say("poly solve d=10, oracle roots")
    x0, d0, _ = B.solve(M, b, restart=30, inner="fp32", rtol=1e-10)
    x1, d1, h1 = B.solve(M, b, restart=30, inner="fp32", rtol=1e-10, poly_degree=10, poly_roots=roots,
                         hist_cap=5000)
    assert d1["status"] == B.OK and d1["rel_resid_true"] <= 1e-10
    assert d1["iters"] < d0["iters"]
    true = np.linalg.norm(bb - A.scipy() @ x1.cpu().numpy()) / np.linalg.norm(bb)
    assert true <= 1e-10
    # parity at rtol 1e-12 (measured: history gap 8e-9, solution gap 9e-12, same iteration count)
    for deg in (5, 10, 20):
        roots = PO.poly_roots(A, deg, start=PO.start_vector(A.n, 3), dtype=np.float32)
        say("poly solve parity d", deg)
        x2, d2, h2 = B.solve(M, b, restart=30, inner="fp32", rtol=1e-12, poly_degree=deg, poly_roots=roots,
                             hist_cap=5000)
        ref = L.gmres_ir(A, bb, m=30, rtol=1e-12, inner="fp32", poly_roots=roots, check_mode=1)
        assert ref.status == L.OK and d2["status"] == B.OK and d2["rel_resid_true"] <= 1e-12
        assert abs(d2["iters"] - ref.iters) <= 2
        k1 = ref.cycle_starts[1] if len(ref.cycle_starts) > 1 else len(ref.hist)
        assert np.max(np.abs(h2[:k1] - np.array(ref.hist[:k1]))) <= HIST_TOL_FP32
        assert rel(x2.cpu().numpy(), ref.x) <= 1e-8
