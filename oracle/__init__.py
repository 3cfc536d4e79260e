"""CPU oracle for the GMRES-IR hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct NumPy implementation of what the HIP path
computes, written from the paper (Loe, Glusa, Yamazaki, Boman,
Rajamanickam, "A Study of Mixed Precision Strategies for GMRES on GPUs",
arXiv 2109.01232): Algorithm 1 (GMRES(m), CGS), the CGS2 description in
Section "GMRES", Algorithm 2 (GMRES-IR), right polynomial preconditioning in
Section "Preconditioning", and the SpMV cache model of Section "Matrix
Structure, Cache Reuse, and SpMV Performance".

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path;
the only common module is the seeded input generator
``paper_2109_01232_amd.problems``.

Floating point is fp64 unless the paper fixes the precision: the inner solve
of GMRES-IR is fp32 by definition (Algorithm 2), and the Krylov-basis storage
variant rounds each basis vector to bfloat16.

Modules
-------
``linalg``    SpMV, bf16 rounding, the GMRES cycle (CGS2 + Givens), GMRES(m),
              GMRES-IR and GMRES-FD (Section "Mixed Precision GMRES-FD").
``poly``      GMRES-polynomial preconditioner: harmonic Ritz values, Leja
              ordering, product-form application, dense evaluation.
``features``  the 16 matrix/residual features of the parameter chooser.
``mlp``       the 16-64-64-3 chooser network: forward, MSE backward, Adam.
``spmv_model`` the paper's SpMV byte model and the algorithmic byte counts.

Parity status: the MLP and the features have no counterpart in the paper
(parity unpinned by the paper; pinned by finite differences and by
closed forms in the tests).
"""
