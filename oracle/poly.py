"""GMRES-polynomial right preconditioner -- oracle.

Test infrastructure only (see the package docstring).

Section "Preconditioning" of the paper uses right preconditioning (solve
``A M y = b``, then ``x = M y``) with ``M = p(A) = sum_k c_k A^k``, a
polynomial of degree d built from the GMRES polynomial; the construction
itself is only cited there.  The reading used here:

* d+1 Arnoldi steps (CGS2, working precision fp32 as in case (b) of that
  section, where the polynomial is both computed and applied in fp32) from a
  start vector give the (d+2) x (d+1) Hessenberg matrix ``Hbar``.
* The roots of the GMRES residual polynomial ``pi`` of degree d+1 are the
  harmonic Ritz values: the eigenvalues of
  ``H + h_{d+2,d+1}^2 H^{-T} e_{d+1} e_{d+1}^T`` with H the square top of Hbar
  (computed in fp64).
* ``pi(a) = prod_i (1 - a / theta_i)`` and ``p(a) = (1 - pi(a)) / a`` (degree d).
* Roots are put in modified Leja order (first the largest modulus, then each
  next root maximises the product of distances to those already chosen;
  a complex root is followed by its conjugate).
* ``p(A) v`` is applied in product form with d SpMVs.
"""

from __future__ import annotations

import numpy as np

from .linalg import gmres_cycle, spmv


MASK64 = (1 << 64) - 1


def splitmix64(z: int) -> int:
    """One output of Vigna's SplitMix64 for state ``z`` (all arithmetic mod 2^64)."""
    z = (z + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def start_vector(n: int, seed: int) -> np.ndarray:
    """Counter-based start vector: ``v_i = 2 * (splitmix64(seed ^ i) >> 11) * 2^-53 - 1`` (fp64).

    Vectorised with wrapping uint64 arithmetic; ``splitmix64`` above is the
    scalar definition it is tested against.
    """
    z = np.uint64(seed & MASK64) ^ np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return 2.0 * ((z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53) - 1.0


def arnoldi_hessenberg(Min, v, steps, dtype=np.float32):
    """``steps`` Arnoldi steps (CGS2) on ``Min`` from ``v``; returns Hbar ((steps+1) x steps)."""
    cyc = gmres_cycle(lambda z: spmv(Min, z), np.asarray(v, dtype=dtype), steps, dtype, "same")
    return cyc.Hbar.astype(np.float64), cyc.k


def harmonic_ritz(Hbar: np.ndarray) -> np.ndarray:
    """Harmonic Ritz values from a (k+1) x k Hessenberg matrix (fp64)."""
    k = Hbar.shape[1]
    H = Hbar[:k, :k].astype(np.float64)
    hk = float(Hbar[k, k - 1])
    ek = np.zeros(k)
    ek[-1] = 1.0
    f = np.linalg.solve(H.T, ek)
    Hh = H.copy()
    Hh[:, -1] += hk * hk * f
    return np.linalg.eigvals(Hh)


def leja_order(theta: np.ndarray) -> np.ndarray:
    """Modified Leja ordering; conjugate pairs adjacent (positive imaginary part first)."""
    rest = [complex(t) for t in theta]
    out = []
    while rest:
        if not out:
            i = int(np.argmax([abs(t) for t in rest]))
        else:
            score = []
            for t in rest:
                d = [abs(t - c) for c in out]
                score.append(-np.inf if min(d) == 0.0 else float(np.sum(np.log(d))))
            i = int(np.argmax(score))
        t = rest.pop(i)
        if t.imag != 0.0:
            j = int(np.argmin([abs(c - t.conjugate()) for c in rest]))
            tc = rest.pop(j)
            hi, lo = (t, tc) if t.imag > 0 else (tc, t)
            out.extend([hi, complex(hi.real, -hi.imag)])
        else:
            out.append(t)
    return np.array(out, dtype=np.complex128)


def poly_roots(A, degree, seed=None, start=None, dtype=np.float32):
    """Ordered roots (degree+1 of them) of the GMRES residual polynomial."""
    from .linalg import csr_matrix

    Min = csr_matrix(A, dtype)
    v = start if start is not None else start_vector(A.n, seed)
    Hbar, k = arnoldi_hessenberg(Min, v, degree + 1, dtype)
    if k < degree + 1:
        raise ValueError("Arnoldi broke down before degree+1 steps")
    return leja_order(harmonic_ritz(Hbar))


def apply_product_form(Min, roots, v, dtype=np.float32):
    """``p(A) v`` with ``p(a) = (1 - prod(1 - a/theta_i)) / a`` in product form.

    Real root: ``y += w / theta``; ``w -= A w / theta``.
    Conjugate pair ``a +- ib`` (mu = a^2 + b^2):
    ``y += (2a w - A w) / mu``; ``w += -(2a/mu) A w + (1/mu) A (A w)``.
    The update of ``w`` after the last root is not needed and is skipped, so a
    polynomial of degree d costs d SpMVs.
    """
    w = np.asarray(v, dtype=dtype).copy()
    y = np.zeros_like(w)
    roots = list(roots)
    i = 0
    nr = len(roots)
    while i < nr:
        t = roots[i]
        if t.imag == 0.0:
            th = dtype(t.real)
            y = y + w / th
            if i + 1 < nr:
                w = w - spmv(Min, w) / th
            i += 1
        else:
            a = t.real
            mu = dtype(a * a + t.imag * t.imag)
            a2 = dtype(2.0 * a)
            Aw = spmv(Min, w)
            y = y + (a2 * w - Aw) / mu
            if i + 2 < nr:
                w = w - (a2 / mu) * Aw + spmv(Min, Aw) / mu
            i += 2
    return y


def residual_poly_dense(Adense: np.ndarray, roots) -> np.ndarray:
    """``pi(A) = prod_i (I - A/theta_i)`` as a dense fp64/complex matrix product."""
    n = Adense.shape[0]
    P = np.eye(n, dtype=np.complex128)
    for t in roots:
        P = P @ (np.eye(n) - Adense / t)
    return P


def p_dense(Adense: np.ndarray, roots) -> np.ndarray:
    """Dense ``p(A)`` from its monomial coefficients (expand ``pi`` then divide by a)."""
    # pi(a) = prod (1 - a/theta) has coefficients c_0 = 1, c_1 ... c_{d+1};
    # p(a) = -(c_1 + c_2 a + ... + c_{d+1} a^d)
    c = np.array([1.0 + 0j])
    for t in roots:
        c = np.convolve(c, np.array([1.0, -1.0 / t]))
    coeffs = -c[1:]
    n = Adense.shape[0]
    P = np.zeros((n, n), dtype=np.complex128)
    Ak = np.eye(n)
    for ck in coeffs:
        P = P + ck * Ak
        Ak = Ak @ Adense
    return P.real
