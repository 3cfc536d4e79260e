"""Planted mistakes in the oracle must be caught by its pins.

Each case copies an oracle module's source, applies one plausible mistake (a
dropped term, a wrong sign or index, a transposed operand), executes the
mutant on the CPU and checks that at least one of the pin checks below fails
for it.  The unmodified oracle passes every check (asserted first).
"""
import sys
import types

import numpy as np
import pytest

import oracle.linalg as L_orig
import oracle.poly as PO_orig
from paper_2109_01232_amd import problems as P


def mutant(module, old, new):
    path = module.__file__
    with open(path) as f:
        src = f.read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    src = src.replace(old, new, 1)
    name = module.__name__ + "_mutant"
    m = types.ModuleType(name)
    m.__dict__["__package__"] = "oracle"
    sys.modules[name] = m  # dataclasses look their module up by name
    try:
        exec(compile(src, path + " (mutant)", "exec"), m.__dict__)
    except Exception:
        sys.modules.pop(name, None)
        raise
    return m


def dense_system(n=24, seed=3, shift=1.5):
    rng = np.random.default_rng(seed)
    Ad = rng.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)
    import scipy.sparse as sp

    S = sp.csr_matrix(Ad)
    S.sort_indices()
    A = P.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)
    return A, Ad, rng.standard_normal(n)


def gmres_pins(L):
    """Returns the list of failed pin names for an oracle.linalg-like module."""
    failed = []
    A, Ad, b = dense_system()
    try:
        r = L.gmres(A, b, m=A.n, rtol=1e-12, check_mode=1)
        x = np.linalg.solve(Ad, b)
        if not (r.status == 0 and np.linalg.norm(r.x - x) / np.linalg.norm(x) <= 1e-10):
            failed.append("dense LU")
    except Exception:
        failed.append("dense LU (exception)")
    s = P.parity_system()
    M = L.csr_matrix(s.A, np.float64)
    try:
        cyc = L.gmres_cycle(lambda v: L.spmv(M, v), s.b, 40, np.float64)
        V = cyc.V[:, : cyc.k + 1]
        AV = np.column_stack([L.spmv(M, V[:, j]) for j in range(cyc.k)])
        if np.linalg.norm(AV - V @ cyc.Hbar) / np.linalg.norm(cyc.Hbar) > 1e-12:
            failed.append("Arnoldi relation")
        if np.linalg.norm(np.eye(cyc.k + 1) - V.T @ V) > 1e-12:
            failed.append("orthogonality")
        h = np.array(cyc.hist)
        if np.any(np.diff(h) > 1e-15):
            failed.append("monotone residual")
        x = cyc.V[:, : cyc.k] @ cyc.y
        if abs(np.linalg.norm(s.b - L.spmv(M, x)) / np.linalg.norm(s.b) - h[-1]) > 1e-8 * h[-1]:
            failed.append("explicit = implicit residual")
    except Exception:
        failed.append("cycle (exception)")
    try:
        ref = L.gmres(s.A, s.b, m=30, rtol=1e-10, check_mode=0)
        ir = L.gmres_ir(s.A, s.b, m=30, rtol=1e-10, inner="fp64", check_mode=0)
        if ref.status != 0 or np.linalg.norm(ref.x - ir.x) / np.linalg.norm(ref.x) > 1e-12:
            failed.append("IR(fp64) = GMRES(m)")
        if np.linalg.norm(ir.x - s.u) / np.linalg.norm(s.u) > 1e-6:
            failed.append("solution")
        ir32 = L.gmres_ir(s.A, s.b, m=50, rtol=1e-10, inner="fp32")
        if ir32.status != 0 or ir32.rel_resid > 1e-10:
            failed.append("IR fp32 converges")
    except Exception:
        failed.append("IR (exception)")
    x = np.random.default_rng(0).standard_normal(1000).astype(np.float32) * 1e3
    bits = L.to_bf16_bits(x)
    import torch

    if not np.array_equal(bits, torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)):
        failed.append("bf16 vs torch")
    return failed


def poly_pins(PO):
    failed = []
    A = P.conv_diff(2, 8, 30.0, (1.0, 0.5))
    Ad = A.scipy().toarray()
    M = L_orig.csr_matrix(A, np.float64)
    for d in (1, 4, 7):
        try:
            roots = PO.poly_roots(A, d, seed=2, dtype=np.float64)
            v = np.random.default_rng(d).standard_normal(A.n)
            y = PO.apply_product_form(M, roots, v, np.float64)
            # independent dense reference: p(A) = A^{-1} (I - prod(I - A/theta))
            Pi = np.eye(A.n, dtype=complex)
            for t in roots:
                Pi = Pi @ (np.eye(A.n) - Ad / t)
            ref = np.linalg.solve(Ad, (np.eye(A.n) - Pi).real @ v)
            if np.linalg.norm(y - ref) > 1e-8 * np.linalg.norm(ref):
                failed.append(f"product form d={d}")
            cyc = L_orig.gmres_cycle(lambda z: L_orig.spmv(M, z), PO.start_vector(A.n, 2), d + 1, np.float64)
            th = PO.harmonic_ritz(cyc.Hbar)
            r = PO.start_vector(A.n, 2) - Ad @ (cyc.V[:, : cyc.k] @ cyc.y)
            Pi2 = np.eye(A.n, dtype=complex)
            for t in th:
                Pi2 = Pi2 @ (np.eye(A.n) - Ad / t)
            if np.linalg.norm(r - (Pi2 @ PO.start_vector(A.n, 2)).real) > 1e-8 * np.linalg.norm(r):
                failed.append(f"harmonic Ritz d={d}")
        except Exception:
            failed.append(f"poly d={d} (exception)")
    if PO.splitmix64(0) != 0xE220A8397B1DCDAF:
        failed.append("splitmix64")
    return failed


def test_unmodified_oracle_passes_all_pins():
    assert gmres_pins(L_orig) == []
    assert poly_pins(PO_orig) == []


LINALG_MUTATIONS = [
    ("single CGS pass", "        h2 = Vj.T @ w\n", "        h2 = 0 * h1\n"),
    ("second pass not subtracted", "        w = w - Vj @ h2\n", "        w = w\n"),
    # (Dropping h2 from the Hessenberg column is not listed: with V orthonormal to
    # working precision h2 = O(u ||A v_j||), so it changes H only at rounding level
    # and no pin can or should separate it; what the second pass buys is the
    # orthogonality of V, which "second pass not subtracted" covers.)
    ("transposed projection operand", "h1 = Vj.T @ w", "h1 = (Vj.T @ w)[::-1].copy()"),
    ("sign of rotated rhs", "g[j + 1] = -sn[j] * g[j]", "g[j + 1] = sn[j] * g[j]"),
    ("rotation sign", "t = cs[i] * R[i, j] + sn[i] * R[i + 1, j]", "t = cs[i] * R[i, j] - sn[i] * R[i + 1, j]"),
    ("rotation index", "R[i + 1, j] = -sn[i] * R[i, j] + cs[i] * R[i + 1, j]",
     "R[i + 1, j] = -sn[i] * R[i, j] + cs[i] * R[i, j]"),
    ("cosine/sine swapped", "cs[j], sn[j] = R[j, j] / rho, R[j + 1, j] / rho",
     "cs[j], sn[j] = R[j + 1, j] / rho, R[j, j] / rho"),
    ("back substitution drops a term", "s = gk[i] - np.dot(Rk[i, i + 1:k], y[i + 1:k])", "s = gk[i]"),
    ("basis vector not normalised", "V[:, j + 1] = store(w / hn)", "V[:, j + 1] = store(w)"),
    ("first vector not normalised", "V[:, 0] = store(r / gamma)", "V[:, 0] = store(r)"),
    ("IR correction not scaled", "x = x + gamma * u.astype(np.float64)", "x = x + u.astype(np.float64)"),
    ("IR residual sign", "r = b - spmv(M64, x)\n        gamma = float(norm2(r))\n        res.refinements += 1\n        if keep_iterates:\n            res.xs.append(x.copy())\n        if gamma < best:\n            best, stall = gamma, 0\n        else:\n            stall += 1\n            if stall >= 3:\n                res.outer.append(gamma / beta)\n                res.status = STAGNATED\n                break\n    res.x = x\n    res.rel_resid = float(norm2(b - spmv(M64, x)) / beta)\n    return res",
     "r = spmv(M64, x) - b\n        gamma = float(norm2(r))\n        res.refinements += 1\n        if keep_iterates:\n            res.xs.append(x.copy())\n        if gamma < best:\n            best, stall = gamma, 0\n        else:\n            stall += 1\n            if stall >= 3:\n                res.outer.append(gamma / beta)\n                res.status = STAGNATED\n                break\n    res.x = x\n    res.rel_resid = float(norm2(b - spmv(M64, x)) / beta)\n    return res"),
    ("GMRES restart drops x0", "x = x + cyc.V[:, : cyc.k] @ cyc.y", "x = cyc.V[:, : cyc.k] @ cyc.y"),
    ("bf16 rounds by truncation", "rounded = (bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)",
     "rounded = bits & np.uint64(0xFFFF0000)"),
]


@pytest.mark.parametrize("name,old,new", LINALG_MUTATIONS, ids=[m[0] for m in LINALG_MUTATIONS])
def test_linalg_mutation_is_caught(name, old, new):
    m = mutant(L_orig, old, new)
    assert gmres_pins(m), f"no pin caught the planted mistake: {name}"


POLY_MUTATIONS = [
    ("real root: multiply instead of divide", "            y = y + w / th\n", "            y = y + w * th\n"),
    ("real root: w update sign", "w = w - spmv(Min, w) / th", "w = w + spmv(Min, w) / th"),
    ("pair: drops A w in y", "y = y + (a2 * w - Aw) / mu", "y = y + (a2 * w) / mu"),
    ("pair: wrong modulus", "mu = dtype(a * a + t.imag * t.imag)", "mu = dtype(a * a - t.imag * t.imag)"),
    ("pair: drops A^2 w", "w = w - (a2 / mu) * Aw + spmv(Min, Aw) / mu", "w = w - (a2 / mu) * Aw"),
    ("harmonic Ritz: no correction", "Hh[:, -1] += hk * hk * f", "Hh[:, -1] += 0 * f"),
    ("harmonic Ritz: transposed solve", "f = np.linalg.solve(H.T, ek)", "f = np.linalg.solve(H, ek)"),
    ("splitmix64 constant", "0xBF58476D1CE4E5B9) & MASK64", "0xBF58476D1CE4E5B8) & MASK64"),
]


@pytest.mark.parametrize("name,old,new", POLY_MUTATIONS, ids=[m[0] for m in POLY_MUTATIONS])
def test_poly_mutation_is_caught(name, old, new):
    m = mutant(PO_orig, old, new)
    assert poly_pins(m), f"no pin caught the planted mistake: {name}"
