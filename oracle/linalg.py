"""GMRES(m) with CGS2 and Givens least squares, and GMRES-IR -- oracle.

Test infrastructure only (see the package docstring).

Paper passages followed:

* Algorithm 1 "GMRES(m) (CGS)": the Arnoldi loop, the least-squares problem
  ``argmin ||gamma e1 - Hbar y||``, the correction ``x = x0 + V y`` and the
  restart from the explicit residual ``b - A x``.
* Section "GMRES": every iteration uses two passes of classical Gram-Schmidt
  (CGS2); each pass is one transposed product ``V^T w`` and one update
  ``w - V h``.
* Algorithm 2 "GMRES-IR": the residual and the solution update in double, the
  inner GMRES(m) on ``A u = r`` in single precision.
* Section "GMRES-IR": convergence of GMRES-IR is checked at restarts only
  (``check_mode=0``); the implicit early exit (``check_mode=1``) is the
  improvement the same section names for future implementations.

Readings where the paper is silent (each listed in the design notes):
the convergence test uses ``||b||`` (Section "GMRES" defines convergence by
``||b - A x|| / ||b||``); ``H[:, j] = h1 + h2`` after the two CGS passes; the
least-squares problem is solved by Givens rotations with
``rho = hypot(h_jj, h_j+1,j)``, ``c = h_jj / rho``, ``s = h_j+1,j / rho``;
lucky breakdown is declared when ``h_j+1,j <= 100 u ||H[:, j]||`` (u the unit
roundoff of the working precision); the inner right-hand side is
``round(r / ||r||)`` and the inner initial guess is zero; all roundings are
round-to-nearest-even.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

# status codes (same meaning as the library's, defined independently here)
OK = 0
NOT_CONVERGED = 1
STAGNATED = 2
ERR_NUMERIC = -4


# ----------------------------------------------------------------------------
# rounding and basic kernels
# ----------------------------------------------------------------------------

def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returns float32.

    bfloat16 keeps the top 16 bits of the IEEE binary32 pattern.  Rounding to
    nearest-even adds ``0x7FFF + lsb`` to the pattern (lsb = bit 16) and
    truncates; NaNs stay NaN (quiet bit set); overflow rounds to infinity.
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    nan = np.isnan(x)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = (bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    rounded = np.where(nan, (bits | np.uint64(0x00400000)) & np.uint64(0xFFFF0000), rounded)
    return rounded.astype(np.uint32).view(np.float32)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """The 16-bit patterns of ``round_bf16(x)``."""
    return (round_bf16(x).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def csr_matrix(A, dtype) -> sp.csr_matrix:
    """The CSR matrix ``A`` (``problems.CSR``) with values rounded to ``dtype``."""
    return sp.csr_matrix((A.vals.astype(dtype), A.colidx, A.rowptr), shape=(A.n, A.n))


def spmv(M: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y = M x; each row summed in column order in the matrix's precision."""
    return M @ x.astype(M.dtype, copy=False)


def norm2(x: np.ndarray) -> np.floating:
    """Euclidean norm in the precision of ``x``."""
    return np.sqrt(np.dot(x, x))


def unit_roundoff(dtype) -> float:
    return float(np.finfo(dtype).eps) / 2.0


# ----------------------------------------------------------------------------
# one GMRES cycle (Algorithm 1 body with CGS2 and Givens rotations)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Cycle:
    k: int  # number of Arnoldi steps taken
    V: np.ndarray  # n x (k+1) basis as stored (columns 0..k; column k only if formed)
    Hbar: np.ndarray  # (k+1) x k unrotated Hessenberg matrix
    y: np.ndarray  # k least-squares coefficients
    gamma: float  # norm of the cycle's right-hand side
    hist: list  # |g_{j+1}| / gamma after each step j
    g: np.ndarray  # rotated right-hand side, length k+1
    breakdown: bool
    stopped: bool  # implicit residual reached the requested threshold
    numeric_error: bool


def gmres_cycle(op, r, m, dtype=np.float64, basis="same", kmax=None, stop_abs=None) -> Cycle:
    """One restart cycle of GMRES(m) from initial guess 0 on right-hand side ``r``.

    ``op(v)`` applies the operator in working precision ``dtype``.  ``basis``
    is ``"same"`` (basis stored in ``dtype``) or ``"bf16"`` (each new basis
    vector rounded to bfloat16; every later product uses the rounded vector).
    At most ``kmax`` (default ``m``) steps are taken; ``stop_abs`` stops the
    cycle once the implicit residual ``|g_{j+1}|`` falls to it.
    """
    dtype = np.dtype(dtype)
    one = dtype.type(1)
    store = (lambda v: round_bf16(v)) if basis == "bf16" else (lambda v: v)
    r = np.asarray(r, dtype=dtype)
    n = r.shape[0]
    kmax = m if kmax is None else min(kmax, m)
    u = unit_roundoff(dtype)

    gamma = norm2(r)
    V = np.zeros((n, m + 1), dtype=dtype)
    Hbar = np.zeros((m + 1, m), dtype=dtype)
    R = np.zeros((m + 1, m), dtype=dtype)  # rotated columns
    cs = np.zeros(m, dtype=dtype)
    sn = np.zeros(m, dtype=dtype)
    g = np.zeros(m + 1, dtype=dtype)
    hist = []
    if not np.isfinite(gamma):
        return Cycle(0, V[:, :1], Hbar[:1, :0], np.zeros(0, dtype), float(gamma), hist, g[:1],
                     False, False, True)
    if gamma == 0:
        return Cycle(0, V[:, :1], Hbar[:1, :0], np.zeros(0, dtype), 0.0, hist, g[:1],
                     True, True, False)
    V[:, 0] = store(r / gamma)
    g[0] = gamma
    k = 0
    breakdown = stopped = numeric_error = False
    for j in range(kmax):
        w = np.asarray(op(V[:, j]), dtype=dtype)
        Vj = V[:, : j + 1]
        # CGS2: two classical Gram-Schmidt passes
        h1 = Vj.T @ w
        w = w - Vj @ h1
        h2 = Vj.T @ w
        w = w - Vj @ h2
        col = h1 + h2
        hn = norm2(w)
        Hbar[: j + 1, j] = col
        Hbar[j + 1, j] = hn
        colnorm = np.sqrt(np.dot(col, col) + hn * hn)
        if not (np.isfinite(hn) and np.isfinite(colnorm)):
            numeric_error = True
            k = j
            break
        # apply the earlier rotations to the new column, then form a new one
        R[: j + 2, j] = Hbar[: j + 2, j]
        for i in range(j):
            t = cs[i] * R[i, j] + sn[i] * R[i + 1, j]
            R[i + 1, j] = -sn[i] * R[i, j] + cs[i] * R[i + 1, j]
            R[i, j] = t
        rho = dtype.type(np.hypot(R[j, j], R[j + 1, j]))
        if rho == 0:
            cs[j], sn[j] = one, dtype.type(0)
        else:
            cs[j], sn[j] = R[j, j] / rho, R[j + 1, j] / rho
        R[j, j] = rho
        R[j + 1, j] = 0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        hist.append(float(abs(g[j + 1]) / gamma))
        k = j + 1
        if hn <= 100.0 * u * colnorm:
            breakdown = True
            break
        if stop_abs is not None and abs(g[j + 1]) <= stop_abs:
            stopped = True
            break
        V[:, j + 1] = store(w / hn)
    y = back_substitute(R[:k, :k], g[:k])
    return Cycle(k, V[:, : k + 1], Hbar[: k + 1, :k], y, float(gamma), hist, g[: k + 1],
                 breakdown, stopped, numeric_error)


def gmres_cycle_lowsync(op, r, m, dtype=np.float64, kmax=None, stop_abs=None) -> Cycle:
    """One restart cycle of GMRES(m) whose Arnoldi process orthogonalises with
    classical Gram-Schmidt twice, the second pass and the normalisation
    delayed by one iteration so that each iteration needs one global reduction
    (the "DCGS2" Arnoldi of Bielich, Langou, Thomas, Swirydowicz, Yamazaki and
    Boman, "Low-synch Gram-Schmidt with delayed reorthogonalization for Krylov
    solvers", Parallel Computing 112, 2022; the paper under study runs CGS2 as
    two separate passes, Section "GMRES", and names the launch count of
    unfused kernels as a cost, Section "Software Implementation").

    Iteration j >= 1 starts from u_j, the vector of iteration j-1 after one
    Gram-Schmidt pass against Q = [v_0 .. v_{j-1}] (not normalised), and from
    p = A u_j.  One reduction gives a = Q^T u_j, alpha = u_j^T u_j,
    c = Q^T p and gam = u_j^T p.  Then, in exact arithmetic the same as CGS2:

    * second pass and norm of u_j: v_j = (u_j - Q a) / rho with
      rho = sqrt(alpha - a^T a) (Pythagoras, Q orthonormal);
    * Hessenberg column j-1 completed: H[:j, j-1] += a, H[j, j-1] = rho (then
      its Givens rotation, the implicit residual and the stop tests, as in
      gmres_cycle);
    * A v_j = (p - A Q a) / rho and A Q = V_{j+1} H[:j+1, :j] (the Arnoldi
      relation of the completed columns), so with t = H[:j+1, :j] a the first
      pass of w = A v_j needs no further reduction:
      h1_i = (c_i - t_i) / rho for i < j,
      h1_j = ((gam - a^T c) / rho - t_j) / rho;
    * u_{j+1} = w - V_{j+1} h1 = p / rho - V_{j+1} (t / rho + h1).

    Iteration 0 is the first pass of w = A v_0 alone; the last iteration only
    completes its column (no SpMV).  Working precision ``dtype`` throughout;
    the basis is stored in ``dtype`` (no bf16 variant: the correction of A v_j
    uses the Arnoldi relation, which a rounded basis breaks).
    """
    dtype = np.dtype(dtype)
    one = dtype.type(1)
    zero = dtype.type(0)
    r = np.asarray(r, dtype=dtype)
    n = r.shape[0]
    kmax = m if kmax is None else min(kmax, m)
    u_ro = unit_roundoff(dtype)

    gamma = norm2(r)
    V = np.zeros((n, m + 1), dtype=dtype)
    Hbar = np.zeros((m + 1, m), dtype=dtype)
    R = np.zeros((m + 1, m), dtype=dtype)
    cs = np.zeros(m, dtype=dtype)
    sn = np.zeros(m, dtype=dtype)
    g = np.zeros(m + 1, dtype=dtype)
    hist = []
    if not np.isfinite(gamma):
        return Cycle(0, V[:, :1], Hbar[:1, :0], np.zeros(0, dtype), float(gamma), hist, g[:1],
                     False, False, True)
    if gamma == 0:
        return Cycle(0, V[:, :1], Hbar[:1, :0], np.zeros(0, dtype), 0.0, hist, g[:1],
                     True, True, False)
    V[:, 0] = r / gamma
    g[0] = gamma
    # iteration 0: first pass of w = A v_0
    p = np.asarray(op(V[:, 0]), dtype=dtype)
    h1 = V[:, :1].T @ p
    Hbar[:1, 0] = h1
    u = p - V[:, :1] @ h1
    k = 0
    breakdown = stopped = numeric_error = False
    for j in range(1, kmax + 1):
        Q = V[:, :j]
        last = j == kmax
        p = None if last else np.asarray(op(u), dtype=dtype)
        # the one reduction of the iteration
        a = Q.T @ u
        alpha = np.dot(u, u)
        if not last:
            c = Q.T @ p
            gam = np.dot(u, p)
        rho = np.sqrt(max(alpha - np.dot(a, a), zero))
        # column j-1 complete: H[:j, j-1] = h1 + h2 (h2 = a), H[j, j-1] = rho
        Hbar[:j, j - 1] += a
        Hbar[j, j - 1] = rho
        col = Hbar[:j, j - 1]
        colnorm = np.sqrt(np.dot(col, col) + rho * rho)
        if not (np.isfinite(rho) and np.isfinite(colnorm)):
            numeric_error = True
            k = j - 1
            break
        # Givens rotation of column j-1 (as in gmres_cycle)
        jj = j - 1
        R[: jj + 2, jj] = Hbar[: jj + 2, jj]
        for i in range(jj):
            tt = cs[i] * R[i, jj] + sn[i] * R[i + 1, jj]
            R[i + 1, jj] = -sn[i] * R[i, jj] + cs[i] * R[i + 1, jj]
            R[i, jj] = tt
        rr = dtype.type(np.hypot(R[jj, jj], R[jj + 1, jj]))
        if rr == 0:
            cs[jj], sn[jj] = one, zero
        else:
            cs[jj], sn[jj] = R[jj, jj] / rr, R[jj + 1, jj] / rr
        R[jj, jj] = rr
        R[jj + 1, jj] = 0
        g[jj + 1] = -sn[jj] * g[jj]
        g[jj] = cs[jj] * g[jj]
        hist.append(float(abs(g[jj + 1]) / gamma))
        k = j
        if rho <= 100.0 * u_ro * colnorm:
            breakdown = True
            break
        # second pass and normalisation of u_j
        V[:, j] = (u - Q @ a) / rho
        if stop_abs is not None and abs(g[jj + 1]) <= stop_abs:
            stopped = True
            break
        if last:
            break
        # first pass of w = A v_j from the same reduction
        t = Hbar[: j + 1, :j] @ a
        h1 = np.empty(j + 1, dtype=dtype)
        h1[:j] = (c - t[:j]) / rho
        h1[j] = ((gam - np.dot(a, c)) / rho - t[j]) / rho
        Hbar[: j + 1, j] = h1
        u = p / rho - V[:, : j + 1] @ (t / rho + h1)
    y = back_substitute(R[:k, :k], g[:k])
    return Cycle(k, V[:, : k + 1], Hbar[: k + 1, :k], y, float(gamma), hist, g[: k + 1],
                 breakdown, stopped, numeric_error)


def back_substitute(Rk: np.ndarray, gk: np.ndarray) -> np.ndarray:
    """Solve the upper-triangular system ``Rk y = gk`` by back substitution."""
    k = gk.shape[0]
    y = np.zeros(k, dtype=gk.dtype)
    for i in range(k - 1, -1, -1):
        s = gk[i] - np.dot(Rk[i, i + 1:k], y[i + 1:k])
        y[i] = s / Rk[i, i]
    return y


# ----------------------------------------------------------------------------
# restarted GMRES(m) (Algorithm 1) and GMRES-IR (Algorithm 2)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    x: np.ndarray
    status: int
    iters: int
    refinements: int
    rel_resid: float  # explicit ||b - A x|| / ||b|| in fp64
    hist: list  # per-step cycle-normalised implicit residuals
    cycle_starts: list  # index into hist where each cycle starts
    outer: list  # explicit relative residual after each refinement/restart
    xs: list  # iterate after each refinement (only if keep_iterates)


def gmres(A, b, x0=None, m=50, rtol=1e-10, max_iters=100000, check_mode=0, keep_iterates=False,
          ortho="cgs2"):
    """Restarted GMRES(m) in fp64, Algorithm 1 with CGS2 (plain double baseline).

    ``ortho="dcgs2"``: the one-reduction CGS2 of ``gmres_cycle_lowsync``."""
    M = csr_matrix(A, np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    beta = float(norm2(b))
    res = Result(x, OK, 0, 0, 0.0, [], [], [], [])
    if beta == 0.0:
        res.x = np.zeros(A.n)
        return res
    r = b - spmv(M, x)
    gamma = float(norm2(r))
    best, stall = gamma, 0
    while True:
        rel = gamma / beta
        res.outer.append(rel)
        if not math.isfinite(rel):
            res.status = ERR_NUMERIC
            break
        if rel <= rtol:
            break
        if res.iters >= max_iters:
            res.status = NOT_CONVERGED
            break
        stop = rtol * beta if check_mode == 1 else None
        if ortho == "dcgs2":
            cyc = gmres_cycle_lowsync(lambda v: spmv(M, v), r, m, np.float64,
                                      kmax=min(m, max_iters - res.iters), stop_abs=stop)
        else:
            cyc = gmres_cycle(lambda v: spmv(M, v), r, m, np.float64, "same",
                              kmax=min(m, max_iters - res.iters), stop_abs=stop)
        if cyc.numeric_error:
            res.status = ERR_NUMERIC
            break
        res.cycle_starts.append(len(res.hist))
        res.hist.extend(cyc.hist)
        res.iters += cyc.k
        x = x + cyc.V[:, : cyc.k] @ cyc.y
        r = b - spmv(M, x)
        gamma = float(norm2(r))
        res.refinements += 1
        if keep_iterates:
            res.xs.append(x.copy())
        if gamma < best:
            best, stall = gamma, 0
        else:
            stall += 1
            if stall >= 3:
                res.outer.append(gamma / beta)
                res.status = STAGNATED
                break
    res.x = x
    res.rel_resid = float(norm2(b - spmv(M, x)) / beta)
    return res


def block_jacobi_inverses(A, bs: int, dtype=np.float64) -> list:
    """Inverses of the diagonal blocks of ``A`` (rows and columns
    ``[k bs, (k+1) bs)``, the last block ragged), computed in ``dtype`` from
    the matrix rounded to ``dtype`` (LAPACK LU inverse in that precision).

    Block-Jacobi preconditioning is named in Sections "Preconditioning" and
    "SpMV Speedup: A Large Test Set"; for GMRES-IR (case (b) of Section
    "Preconditioning") the fp32 preconditioner is both computed and applied in
    fp32, so the inner solve of GMRES-IR takes ``dtype = float32``; the fp64
    solve keeps an fp64 preconditioner.
    """
    S = csr_matrix(A, dtype)
    out = []
    for r0 in range(0, A.n, bs):
        r1 = min(A.n, r0 + bs)
        out.append(np.linalg.inv(S[r0:r1, r0:r1].toarray()))
    return out


def block_jacobi_apply(inverses, v: np.ndarray, dtype) -> np.ndarray:
    """``M^{-1} v`` block by block in ``dtype`` (the inverses' own precision)."""
    v = np.asarray(v, dtype=dtype)
    y = np.empty_like(v)
    r0 = 0
    for Bi in inverses:
        k = Bi.shape[0]
        y[r0:r0 + k] = Bi.astype(dtype, copy=False) @ v[r0:r0 + k]
        r0 += k
    return y


def gmres_ir(A, b, x0=None, m=50, rtol=1e-10, inner="fp32", basis="same", cap=0,
             max_iters=100000, check_mode=0, poly_roots=None, keep_iterates=False, max_refinements=0,
             poly_prec=None, bj_block=0, ortho="cgs2"):
    """GMRES-IR (Algorithm 2): fp64 residual and update around an inner GMRES(m).

    ``inner`` is ``"fp32"`` or ``"fp64"``; ``basis`` is ``"same"`` or ``"bf16"``
    (bf16 needs an fp32 inner solve).  ``cap`` bounds the inner iterations per
    refinement (0 means ``m``, one cycle); when ``cap > m`` the inner solve
    restarts in its own precision from ``rhat - A_in u``.  ``poly_roots``
    (ordered, see ``oracle.poly``) turns on right preconditioning by
    ``M = p(A_in)``: the inner operator is ``A_in p(A_in)`` and the correction is
    ``p(A_in) V y``; residuals are those of ``A``.  ``max_refinements > 0``
    stops (``NOT_CONVERGED``) after that many refinements.  ``poly_prec="fp32"``
    with an fp64 inner solve applies the polynomial in single precision
    (Section "Preconditioning": each application of an fp32 ``M`` to an fp64
    vector casts it to fp32, multiplies by ``M`` with the fp32 matrix and
    casts the result back); every other operation stays in fp64.
    ``bj_block > 0``: right block-Jacobi preconditioning instead, the inverses
    of the diagonal blocks computed and applied in the inner precision.
    ``ortho="dcgs2"``: the inner cycles use the one-reduction CGS2 of
    ``gmres_cycle_lowsync`` (basis kept in working precision).
    """
    wp = np.float32 if inner == "fp32" else np.float64
    if ortho == "dcgs2" and basis != "same":
        raise ValueError("the one-reduction CGS2 keeps the basis in working precision")
    if basis == "bf16" and wp != np.float32:
        raise ValueError("bf16 basis needs an fp32 inner solve")
    M64 = csr_matrix(A, np.float64)
    Min = csr_matrix(A, wp)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    cap = m if cap <= 0 else cap
    beta = float(norm2(b))
    res = Result(x, OK, 0, 0, 0.0, [], [], [], [])
    if beta == 0.0:
        res.x = np.zeros(A.n)
        return res

    if poly_roots is not None and len(poly_roots) > 1:
        from .poly import apply_product_form

        if poly_prec == "fp32" and wp == np.float64:
            M32 = csr_matrix(A, np.float32)
            papply = lambda v: apply_product_form(M32, poly_roots, v.astype(np.float32),
                                                  np.float32).astype(np.float64)
        else:
            papply = lambda v: apply_product_form(Min, poly_roots, v, wp)
    elif bj_block > 0:
        inverses = block_jacobi_inverses(A, bj_block, wp)
        papply = lambda v: block_jacobi_apply(inverses, v, wp)
    else:
        papply = None
    op = (lambda v: spmv(Min, papply(v))) if papply else (lambda v: spmv(Min, v))

    r = b - spmv(M64, x)
    gamma = float(norm2(r))
    best, stall = gamma, 0
    while True:
        rel = gamma / beta
        res.outer.append(rel)
        if not math.isfinite(rel):
            res.status = ERR_NUMERIC
            break
        if rel <= rtol:
            break
        if res.iters >= max_iters or (max_refinements > 0 and res.refinements >= max_refinements):
            res.status = NOT_CONVERGED
            break
        rhat = (r / gamma).astype(wp)
        u = np.zeros(A.n, dtype=wp)
        rin = rhat
        budget = min(cap, max_iters - res.iters)
        stop = wp(rtol * beta / gamma) if check_mode == 1 else None
        used = 0
        numeric = False
        while used < budget:
            if ortho == "dcgs2":
                cyc = gmres_cycle_lowsync(op, rin, m, wp, kmax=min(m, budget - used), stop_abs=stop)
            else:
                cyc = gmres_cycle(op, rin, m, wp, basis, kmax=min(m, budget - used), stop_abs=stop)
            if cyc.numeric_error:
                numeric = True
                break
            res.cycle_starts.append(len(res.hist))
            res.hist.extend(cyc.hist)
            used += cyc.k
            z = (cyc.V[:, : cyc.k] @ cyc.y).astype(wp)
            u = u + (papply(z) if papply else z)
            if cyc.stopped or cyc.breakdown or cyc.k == 0 or used >= budget:
                break
            rin = rhat - spmv(Min, u)
        if numeric:
            res.status = ERR_NUMERIC
            break
        res.iters += used
        x = x + gamma * u.astype(np.float64)
        r = b - spmv(M64, x)
        gamma = float(norm2(r))
        res.refinements += 1
        if keep_iterates:
            res.xs.append(x.copy())
        if gamma < best:
            best, stall = gamma, 0
        else:
            stall += 1
            if stall >= 3:
                res.outer.append(gamma / beta)
                res.status = STAGNATED
                break
    res.x = x
    res.rel_resid = float(norm2(b - spmv(M64, x)) / beta)
    return res


def gmres_fd(A, b, switch, m=50, rtol=1e-10, max_iters=100000, check_mode=0, basis="same"):
    """GMRES-FD (Section "Mixed Precision GMRES-FD"): GMRES(m) in single
    precision for ``switch`` iterations, then GMRES(m) in double precision
    with the single-precision solution as its initial vector.

    The single-precision phase is written as one refinement of ``gmres_ir``
    with an fp32 inner solve of ``switch`` iterations restarted in fp32: that
    is fp32 GMRES(m) on the system scaled by ``1 / ||b||`` (a scaling that
    changes nothing in exact arithmetic; in fp32 it keeps the right-hand side
    in range), whose solution is scaled back in fp64.  Its implicit early
    exit is off, so the phase runs its full length; if the explicit fp64
    residual at the switch already meets ``rtol`` the double phase is skipped.
    Returns a ``Result`` whose counters cover both phases and whose ``xs``
    holds the iterate at the switch.
    """
    x = np.zeros(A.n)
    total = Result(x, NOT_CONVERGED, 0, 0, 0.0, [], [], [], [])
    if switch > 0:
        single = gmres_ir(A, b, m=m, rtol=rtol, inner="fp32", basis=basis, cap=switch,
                          max_iters=min(switch, max_iters), check_mode=0, max_refinements=1)
        total.status, total.iters, total.refinements = single.status, single.iters, single.refinements
        total.hist.extend(single.hist)
        total.cycle_starts.extend(single.cycle_starts)
        total.outer.extend(single.outer)
        total.xs.append(single.x.copy())
        x = single.x
    if total.status == NOT_CONVERGED and total.iters < max_iters:
        double = gmres(A, b, x0=x, m=m, rtol=rtol, max_iters=max_iters - total.iters, check_mode=check_mode)
        offset = len(total.hist)
        total.status = double.status
        total.iters += double.iters
        total.refinements += double.refinements
        total.hist.extend(double.hist)
        total.cycle_starts.extend(c + offset for c in double.cycle_starts)
        total.outer.extend(double.outer)
        x = double.x
    total.x = x
    total.rel_resid = float(norm2(np.asarray(b, dtype=np.float64) - spmv(csr_matrix(A, np.float64), x))
                            / max(float(norm2(np.asarray(b, dtype=np.float64))), np.finfo(float).tiny))
    return total


def gmres_single(A, b, m=50, rtol=1e-10, max_iters=5000):
    """Restarted GMRES(m) entirely in fp32 (matrix, vectors, restart residual).

    The "single precision GMRES(50)" curve of Section "Convergence and Kernel
    Speedup for GMRES vs GMRES-IR", which stalls well above 1e-10.  Returns
    the fp64-evaluated relative residual history after each restart.
    """
    M32 = csr_matrix(A, np.float32)
    M64 = csr_matrix(A, np.float64)
    b32 = np.asarray(b, dtype=np.float32)
    x = np.zeros(A.n, dtype=np.float32)
    beta = float(norm2(np.asarray(b, dtype=np.float64)))
    outer = []
    iters = 0
    while iters < max_iters:
        r = b32 - spmv(M32, x)
        cyc = gmres_cycle(lambda v: spmv(M32, v), r, m, np.float32, "same")
        if cyc.k == 0:
            break
        iters += cyc.k
        x = x + cyc.V[:, : cyc.k] @ cyc.y
        rel = float(norm2(np.asarray(b, dtype=np.float64) - spmv(M64, x.astype(np.float64))) / beta)
        outer.append(rel)
        if rel <= rtol:
            break
    return x, outer
