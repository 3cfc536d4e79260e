"""SpMV cache model of the paper and algorithmic byte counts -- oracle.

Test infrastructure only (see the package docstring).

Section "Matrix Structure, Cache Reuse, and SpMV Performance": for a CSR
matrix with n rows and w nonzeros per row, fp64 without reuse of x moves
``n w (4 + 2*8) = 20 w n`` bytes; fp32 with perfect caching of x moves
``n w (4 + 4) + 4 n = (8 w + 4) n`` bytes; the predicted speedup is
``5 w / (2 w + 1)`` (2.27 for w = 5, 2.33 for w = 7).

Algorithmic bytes (every input read once, every output written once):
SpMV ``(s + 4) nnz + 4 (n + 1) + 2 s n`` with s the value size;
one CGS2 pass sweep of V with k columns of element size sb: ``sb n k``.
"""

from __future__ import annotations


def fp64_no_reuse_bytes(n: int, w: int) -> int:
    return n * w * (4 + 2 * 8)


def fp32_perfect_cache_bytes(n: int, w: int) -> int:
    return n * w * (4 + 4) + n * 4


def predicted_speedup(w: float) -> float:
    return 5.0 * w / (2.0 * w + 1.0)


def spmv_bytes(n: int, nnz: int, s: int) -> int:
    return (s + 4) * nnz + 4 * (n + 1) + 2 * s * n
