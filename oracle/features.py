"""The 16 features of the learned parameter chooser -- oracle.

Test infrastructure only (see the package docstring).  The paper has no
learned component; its Section "Choosing a Restart Size for GMRES-IR" shows
that the best restart length depends on the problem (orthogonalisation cost
versus stalling of the fp32 inner solve), which is what the chooser learns.
Parity unpinned by the paper: the definitions below are this project's, and
the tests pin them by closed forms on matrices whose features are known.

Row statistics (fp64), with ``d_i = |a_ii|``, ``S_i = sum_{j != i} |a_ij|``,
``L_i = sum_{j < i} a_ij``, ``U_i = sum_{j > i} a_ij``,
``rowsum_i = sum_j a_ij``, ``D = mean_i d_i``:

 0  log10(N)
 1  nnz / N
 2  max_i nnz_i
 3  mean_i  d_i / (d_i + S_i)        (0 for an all-zero row)
 4  min_i   d_i / (d_i + S_i)
 5  fraction of rows with d_i >= S_i
 6  mean_i rowsum_i / D
 7  log10(||A||_F / sqrt(N))
 8  std_i(a_ii) / D
 9  mean_i |U_i - L_i| / (S_i + tiny)   (0 for rows with S_i = 0)

Ten fp32 Arnoldi steps (CGS2) from ``b / ||b||`` (the first GMRES cycle with
x0 = 0) give the implicit residuals rho_j and the Ritz values theta of the
square k x k Hessenberg matrix (k <= 10, fewer on breakdown), eigenvalues
computed in fp64:

10  log10(rho_min(5,k))
11  log10(rho_k)
12  log10(max|theta| / min|theta|)
13  max|Im theta| / max|theta|
14  min Re(theta) / max|theta|
15  log10(max|theta| / D)

log10 arguments are floored at 1e-30.
"""

from __future__ import annotations

import numpy as np

from .linalg import csr_matrix, gmres_cycle, spmv

TINY = 1e-30


def _log10(x):
    return float(np.log10(max(float(x), TINY)))


def row_features(A) -> np.ndarray:
    n = A.n
    rp = A.rowptr.astype(np.int64)
    rows = np.repeat(np.arange(n), np.diff(rp))
    v = A.vals
    c = A.colidx.astype(np.int64)
    d = np.zeros(n)
    S = np.zeros(n)
    L = np.zeros(n)
    U = np.zeros(n)
    rs = np.zeros(n)
    diag_mask = c == rows
    np.add.at(d, rows[diag_mask], np.abs(v[diag_mask]))
    diag_signed = np.zeros(n)
    np.add.at(diag_signed, rows[diag_mask], v[diag_mask])
    off = ~diag_mask
    np.add.at(S, rows[off], np.abs(v[off]))
    np.add.at(L, rows[c < rows], v[c < rows])
    np.add.at(U, rows[c > rows], v[c > rows])
    np.add.at(rs, rows, v)
    D = d.mean()
    tot = d + S
    frac = np.where(tot > 0, d / np.where(tot > 0, tot, 1.0), 0.0)
    asym = np.where(S > 0, np.abs(U - L) / (S + TINY), 0.0)
    f = np.zeros(10)
    f[0] = np.log10(n)
    f[1] = A.nnz / n
    f[2] = np.diff(rp).max()
    f[3] = frac.mean()
    f[4] = frac.min()
    f[5] = np.mean(d >= S)
    f[6] = rs.mean() / max(D, TINY)
    f[7] = _log10(np.sqrt(np.dot(v, v)) / np.sqrt(n))
    f[8] = diag_signed.std() / max(D, TINY)
    f[9] = asym.mean()
    return f


def arnoldi_features(A, b, D, steps=10) -> np.ndarray:
    M = csr_matrix(A, np.float32)
    cyc = gmres_cycle(lambda z: spmv(M, z), np.asarray(b, dtype=np.float32), steps, np.float32)
    k = cyc.k
    f = np.zeros(6)
    if k == 0:
        return f
    hist = cyc.hist
    f[0] = _log10(hist[min(5, k) - 1])
    f[1] = _log10(hist[k - 1])
    theta = np.linalg.eigvals(cyc.Hbar[:k, :k].astype(np.float64))
    amax = np.abs(theta).max()
    amin = np.abs(theta).min()
    f[2] = _log10(amax / max(amin, TINY))
    f[3] = np.abs(theta.imag).max() / max(amax, TINY)
    f[4] = theta.real.min() / max(amax, TINY)
    f[5] = _log10(amax / max(D, TINY))
    return f


def features(A, b) -> np.ndarray:
    """The 16 chooser features as float32."""
    fr = row_features(A)
    D = np.abs(A.scipy().diagonal()).mean()
    fa = arnoldi_features(A, b, D)
    return np.concatenate([fr, fa]).astype(np.float32)
