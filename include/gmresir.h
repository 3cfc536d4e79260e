/*
 * gmresir.h -- C ABI of the MI355X (gfx950) GMRES-IR library.
 *
 * The library solves a sparse linear system A x = b to a relative residual
 * tolerance ||b - A x||_2 / ||b||_2 <= rtol (Section "GMRES": convergence is
 * measured by the relative residual of the original system) with restarted
 * GMRES(m) (Algorithm 1, classical Gram-Schmidt applied twice per iteration,
 * CGS2) either in fp64 throughout or as GMRES-IR (Algorithm 2): an fp32 inner
 * GMRES(m) whose right-hand side is the fp64 residual and whose correction is
 * added to x in fp64 at every restart.  Optional: the Krylov basis stored in
 * bfloat16 with fp32 arithmetic, and a right polynomial preconditioner
 * M = p(A) (Section "Preconditioning") built from fp32 harmonic Ritz values.
 *
 * Conventions for every entry point:
 *  - Pointers are HIP device pointers owned by the caller unless the
 *    parameter name ends in _host.  The library never calls hipMalloc or
 *    hipFree: every device buffer holding data is passed in.  (Host-side
 *    handles are allocated with malloc/new; gmresir_solve on systems of at
 *    most 2^18 rows records its inner cycle as a HIP graph, and profiling
 *    creates HIP events -- runtime objects the HIP runtime backs itself.)
 *  - Work is enqueued on the caller's `stream` (a hipStream_t passed as
 *    void*; NULL is the legacy default stream).  Functions that return host
 *    values synchronise that stream before returning.
 *  - The CSR matrix uses int32 row pointers (n+1 entries, rowptr[0] = 0) and
 *    int32 column indices, ascending within each row, fp64 values.
 *  - Return value: 0 on success, a positive solver outcome (x then holds the
 *    best fp64 iterate), or a negative error (see gmresir_status).  On
 *    argument errors nothing is enqueued and outputs are unchanged.  A
 *    readable reason for the last error of the calling thread is returned by
 *    gmresir_last_error().
 *  - Thread safety: a matrix handle is read-only after creation; concurrent
 *    calls are safe when each uses its own workspace and stream.
 */
#ifndef GMRESIR_H
#define GMRESIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum gmresir_status {
  GMRESIR_OK = 0,
  GMRESIR_NOT_CONVERGED = 1,  /* max_iters reached; x = last fp64 iterate */
  GMRESIR_STAGNATED = 2,      /* no decrease of ||b - A x|| over 3 restarts */
  GMRESIR_BREAKDOWN = 3,      /* polynomial setup: Arnoldi broke down early */
  GMRESIR_ERR_INVALID_ARG = -1,
  GMRESIR_ERR_HIP = -2,       /* a HIP runtime call failed */
  GMRESIR_ERR_WORKSPACE = -3, /* workspace smaller than gmresir_*_workspace_bytes */
  GMRESIR_ERR_NUMERIC = -4,   /* NaN or Inf met in a norm or a residual */
  GMRESIR_ERR_UNSUPPORTED = -5
};

enum gmresir_precision { GMRESIR_FP64 = 0, GMRESIR_FP32 = 1, GMRESIR_BF16 = 2 };

/* Time categories of gmresir_result.cat_* (filled when params.profile = 1).
   They follow the kernel split of the paper's Figure "BentPipeTiming"
   (SpMV, GEMV-Trans, GEMV-NoTrans, Norm, Other), merged where this library
   fuses the operations into one kernel. */
enum gmresir_category {
  GMRESIR_CAT_SPMV_PROJ = 0,   /* w = A v_j and h1 = V^T w (first CGS pass projection); ortho 1: the
                                  SpMV with the partial sums of the iteration's one reduction */
  GMRESIR_CAT_UPDATE_PROJ = 1, /* w -= V h1 and h2 = V^T w (second pass projection) */
  GMRESIR_CAT_UPDATE_NORM = 2, /* w -= V h2 and the partial sums of ||w||^2; ortho 1: the update sweep
                                  (second pass and normalisation of v_j, first pass of the next vector) */
  GMRESIR_CAT_POLY = 3,        /* SpMV steps of p(A) */
  GMRESIR_CAT_REFINE = 4,      /* correction x += gamma V y, r = b - A x (fp64), cast of r */
  GMRESIR_CAT_OTHER = 5,       /* fallbacks for restart lengths beyond the fused limit */
  GMRESIR_CAT_TAIL = 6,        /* one-block tails: sums of h1, h2, ||w||^2; Hessenberg column, Givens update */
  GMRESIR_NCAT = 7
};

typedef struct gmresir_matrix gmresir_matrix; /* opaque host-side handle */

typedef struct {
  int32_t restart;     /* m >= 1: Krylov basis size of one cycle (Algorithm 1). Paper default 50. */
  int32_t inner_cap;   /* max inner iterations per refinement; 0 means = restart (one cycle) */
  int64_t max_iters;   /* limit on the total number of inner iterations (> 0) */
  double rtol;         /* relative residual target, ||b - A x|| / ||b|| (> 0) */
  int32_t inner_prec;  /* GMRESIR_FP64: plain restarted GMRES(m) in fp64;
                          GMRESIR_FP32: GMRES-IR with an fp32 inner solve */
  int32_t basis_prec;  /* storage of the Krylov basis: FP64 (needs FP64 inner),
                          FP32 or BF16 (need FP32 inner) */
  int32_t poly_degree; /* 0: no preconditioner; d >= 1: right preconditioner p(A) of degree d,
                          whose d+1 ordered roots are passed to gmresir_solve */
  int32_t check_mode;  /* 0: convergence checked only at restarts (GMRES-IR as in the paper);
                          1: also stop a cycle once the implicit residual reaches rtol,
                          then verify with the explicit fp64 residual */
  int32_t profile;     /* 1: time every kernel with HIP events (slower; fills cat_*) */
  int32_t poly_prec;   /* precision of the polynomial p(A) (poly_degree > 0): 0 = that of the inner
                          solve; GMRESIR_FP32 with inner_prec FP64 = an fp32 p(A) inside fp64 GMRES(m)
                          (Section "Preconditioning", the case of an fp32 M applied to fp64 vectors:
                          each application casts its fp64 input to fp32, runs the d fp32 SpMV steps on
                          the fp32 copy of A and widens the result; every other operation stays fp64) */
  int32_t bj_block;    /* 0: none; 1..64: right block-Jacobi preconditioner M = blockdiag of the
                          diagonal blocks of A of bj_block consecutive rows (the last one ragged),
                          computed and applied in the inner precision (Section "Preconditioning":
                          for GMRES-IR the fp32 M is both computed and applied in fp32, from the fp32
                          copy of A; the fp64 solve keeps M in fp64): each block is inverted by
                          Gauss-Jordan elimination with partial pivoting at the start of every
                          solve.  Excludes poly_degree > 0.  A singular block gives NUMERIC. */
  int32_t ortho;       /* 0: CGS2 as two separate passes per iteration (Section "GMRES"): three sweeps
                          of the basis and three reductions; 1: the same two classical Gram-Schmidt
                          passes with the second pass and the normalisation delayed by one
                          iteration (delayed reorthogonalisation, Bielich et al., Parallel Computing
                          2022): one reduction and two sweeps of the basis per iteration, results
                          equal to CGS2's in exact arithmetic.  1 needs basis_prec = inner_prec
                          (no BF16) and restart <= 128. */
} gmresir_params;

typedef struct {
  int32_t status;
  int32_t refinements;       /* fp64 residual evaluations after a correction (restarts) */
  int64_t iters;             /* total inner iterations (Arnoldi steps) */
  int64_t cycles;            /* inner GMRES cycles */
  double rel_resid_true;     /* ||b - A x||_2 / ||b||_2, fp64, of the returned x */
  double rel_resid_implicit; /* last implicit estimate (Givens) relative to ||b|| */
  double solve_s;            /* host wall time of the call */
  double cat_time_s[GMRESIR_NCAT];  /* device time per category (profile = 1) */
  double cat_bytes[GMRESIR_NCAT];   /* algorithmic HBM bytes per category (always filled) */
  int64_t cat_launches[GMRESIR_NCAT];
} gmresir_result;

/* ---- matrix ------------------------------------------------------------ */

/* Bytes of device storage gmresir_matrix_create needs for an n x n matrix
   with nnz nonzeros: the fp32 copy of the values (round to nearest even;
   Section "Mixed Precision GMRES-IR" keeps both an fp64 and an fp32 copy of A)
   and the row-tile table of the SpMV kernels.  0 on invalid sizes. */
size_t gmresir_matrix_storage_bytes(int64_t n, int64_t nnz);

/* Build a handle.  rowptr/colidx/vals: device CSR arrays, borrowed (they
   must stay alive and unchanged while the handle is used).  storage: device
   buffer of gmresir_matrix_storage_bytes(n, nnz) bytes, 256-byte aligned,
   owned by the caller and written here.  The row pointers are copied to the
   host once to cut the rows into tiles of at most 512 rows / 2560 nonzeros.
   When no row has more than 512 nonzeros and the padding stays bounded, a
   sliced ELLPACK copy (slices of 64 rows, one row per lane) is built too.
   When the rows of every slice share their column offsets c - r (stencils:
   each slice's sorted union of offsets is at most 1.25 times as many slots
   as its longest row gives; every row's columns strictly increasing), the
   copy keeps one offset list per slice and zeros for absent entries, and the
   SpMV reads only the values (4 bytes per fp32 slot, no row lengths).
   Otherwise its column indices are 16-bit offsets from the row when every
   entry lies within 32767 columns of its row (the SpMV then reads 6 bytes per
   fp32 nonzero instead of 8), else 32-bit indices.  colidx is copied to the
   host (in windows of at most 16 MB) to build the offset lists.  Errors: INVALID_ARG (null pointer, n < 1, nnz < 0, nnz >= 2^31, rowptr not
   monotone or rowptr[n] != nnz), WORKSPACE (storage too small), HIP. */
int gmresir_matrix_create(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                          const double* vals, void* storage, size_t storage_bytes, void* stream,
                          gmresir_matrix** out_host);
int gmresir_matrix_destroy(gmresir_matrix* A);
int64_t gmresir_matrix_n(const gmresir_matrix* A);
int64_t gmresir_matrix_nnz(const gmresir_matrix* A);
int64_t gmresir_matrix_tiles(const gmresir_matrix* A);
/* Layout the SpMV kernels read: 0 = row tiles of the CSR arrays only,
   1 = sliced ELLPACK copy with 32-bit columns, 2 = sliced copy with 16-bit
   column offsets, 3 = sliced copy with one offset list per slice; -1 for
   A == NULL. */
int32_t gmresir_matrix_layout(const gmresir_matrix* A);

/* y = A x (Algorithm 1, the SpMV).  prec GMRESIR_FP64: x, y fp64 and the fp64
   values; GMRESIR_FP32: x, y fp32 and the fp32 copy, fp32 accumulation.  Each
   row is summed in column order.  x and y must not overlap. */
int gmresir_spmv(const gmresir_matrix* A, int32_t prec, const void* x, void* y, void* stream);

/* ---- solver ------------------------------------------------------------ */

/* Workspace bytes of gmresir_solve for this matrix and parameters (0 if the
   parameters are invalid). */
size_t gmresir_workspace_bytes(const gmresir_matrix* A, const gmresir_params* p);

/* Solve A x = b.  b: device fp64[n].  x: device fp64[n], initial guess on
   entry, solution on exit.  poly_roots_host: 2*(poly_degree+1) doubles
   (re, im pairs) in application order, conjugate pairs adjacent (as written
   by gmresir_poly_setup), or NULL when poly_degree = 0.  ws: device buffer of
   gmresir_workspace_bytes(A, p) bytes, 256-byte aligned; its contents on
   entry do not matter.  res_host: filled on return (also on solver outcomes).
   hist_host (may be NULL): receives up to hist_cap per-iteration values
   |g_{j+1}| / |g_1|, the implicit residual of each inner iteration relative
   to the right-hand side of its cycle.  The stream is synchronised once per
   refinement.  b = 0 gives x = 0 and GMRESIR_OK.  For n <= 2^18 (and
   profile = 0) the kernels of one inner cycle are recorded once as a HIP
   graph and replayed for every later cycle of the same length (the same
   kernels and bits as direct launches; less host launch work). */
int gmresir_solve(const gmresir_matrix* A, const double* b, double* x, const gmresir_params* p,
                  const double* poly_roots_host, void* ws, size_t ws_bytes, gmresir_result* res_host,
                  double* hist_host, int64_t hist_cap, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the same
   solve as gmresir_solve, with its workspace taken from a static device
   array of GMRESIR_NOALLOC_MAX_BYTES bytes that the library holds on every
   GPU it runs on until the process ends.  The call allocates nothing (no
   hipMalloc / hipFree; no HIP graph is recorded: every kernel is launched
   directly).  Arguments as for gmresir_solve without ws / ws_bytes.  The
   device current at the call must be the matrix's device.  Errors as for
   gmresir_solve, plus WORKSPACE when gmresir_workspace_bytes(A, p) exceeds
   GMRESIR_NOALLOC_MAX_BYTES (nothing is enqueued), and INVALID_ARG for
   profile = 1 (per-kernel timing creates HIP events).  Every call on a GPU
   shares that GPU's array, which keeps the last call's contents (nothing in
   it needs to start at zero: every solve initialises its state first); calls
   that overlap in time on one GPU -- on different streams or threads -- race
   on it and must not be issued. */
#define GMRESIR_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int gmresir_solve_noalloc(const gmresir_matrix* A, const double* b, double* x, const gmresir_params* p,
                          const double* poly_roots_host, gmresir_result* res_host, double* hist_host,
                          int64_t hist_cap, void* stream);

/* ---- GMRES-FD (Section "Mixed Precision GMRES-FD") ---------------------- */

/* Workspace bytes of gmresir_solve_fd (0 if the arguments are invalid). */
size_t gmresir_fd_workspace_bytes(const gmresir_matrix* A, const gmresir_params* p, int64_t switch_iters);

/* GMRES-FD, the paper's float-to-double variant: restarted GMRES(m) run
   entirely in fp32 for switch_iters inner iterations, then fp64 GMRES(m)
   started from the fp32 solution, until the relative residual reaches rtol.
   The fp32 phase solves the system scaled by 1 / ||b|| (b / ||b|| rounded to
   fp32, x0 = 0 after the scaling; its restarts use the fp32 residual of the
   fp32 matrix copy) and its solution is scaled back and added to x in fp64;
   the explicit fp64 residual is evaluated once, at the switch (if it already
   meets rtol, the fp64 phase is skipped).  switch_iters = 0 is plain fp64
   GMRES(m).
   Parameters: restart, max_iters (the total over both phases), rtol and
   profile as for gmresir_solve; inner_prec must be FP32 and basis_prec FP32
   or BF16 (the fp32 phase's basis); inner_cap and poly_degree must be 0;
   check_mode applies to the fp64 phase only (the fp32 phase runs its full
   length).  b, x, ws, res_host, hist_host as for gmresir_solve (ws:
   gmresir_fd_workspace_bytes bytes); hist_host receives the fp32 phase's
   per-iteration values, then the fp64 phase's.  res_host->iters counts both
   phases; the status is that of the last phase run.  Errors: INVALID_ARG
   (as above, switch_iters < 0 or >= 2^31), WORKSPACE, HIP, NUMERIC. */
int gmresir_solve_fd(const gmresir_matrix* A, const double* b, double* x, const gmresir_params* p,
                     int64_t switch_iters, void* ws, size_t ws_bytes, gmresir_result* res_host,
                     double* hist_host, int64_t hist_cap, void* stream);

/* ---- polynomial preconditioner (Section "Preconditioning") -------------- */

/* Workspace bytes for gmresir_poly_setup / gmresir_poly_apply of degree <= max_degree. */
size_t gmresir_poly_workspace_bytes(const gmresir_matrix* A, int32_t max_degree);

/* Roots of the GMRES residual polynomial of degree d+1 (so that p has degree d):
   d+1 fp32 Arnoldi steps (CGS2) on the fp32 copy of A from start vector
   `start` (device fp64[n]; if NULL, start[i] = 2*(splitmix64(seed ^ i) >> 11)
   * 2^-53 - 1), then on the host in fp64 the harmonic Ritz values (eigenvalues
   of H + h_{d+2,d+1}^2 H^{-T} e_{d+1} e_{d+1}^T) in modified Leja order.
   roots_host: 2*(d+1) doubles (re, im).  hbar_host (may be NULL): the
   (d+2) x (d+1) Hessenberg matrix, column-major.  Returns BREAKDOWN if the
   Arnoldi process ends before d+1 steps. */
int gmresir_poly_setup(const gmresir_matrix* A, int32_t degree, const double* start, uint64_t seed,
                       void* ws, size_t ws_bytes, double* roots_host, double* hbar_host, void* stream);

/* y = p(A) v in fp32 with the fp32 copy of A, in product form (d SpMVs).
   roots_host as above (d+1 roots).  v, y: device fp32[n], distinct. */
int gmresir_poly_apply(const gmresir_matrix* A, int32_t degree, const double* roots_host, const float* v,
                       float* y, void* ws, size_t ws_bytes, void* stream);

/* ---- learned parameter chooser ----------------------------------------- */

/* The 16 chooser features (row statistics of A in fp64 and a 10-step fp32
   Arnoldi process from b / ||b||): see the feature list in the Python
   package.  feat_host: 16 floats.  ws: gmresir_poly_workspace_bytes(A, 10). */
int gmresir_features(const gmresir_matrix* A, const double* b, void* ws, size_t ws_bytes, float* feat_host,
                     void* stream);

/* Network 16-64-64-3: h1 = tanh(xn W1 + b1), h2 = tanh(h1 W2 + b2),
   y = h2 W3 + b3, xn = (x - shift) * scale.  params: device fp32[5443] laid
   out W1[16][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3] (row-major
   [in][out]).  shift, scale: device fp32[16].  X: device fp32[batch][16];
   Y: device fp32[batch][3]. */
int gmresir_mlp_forward(const float* params, const float* shift, const float* scale, const float* X,
                        float* Y, int32_t batch, void* stream);

/* Loss L = sum (y - t)^2 / (3 batch) and its gradient w.r.t. params
   (grad: device fp32[5443], loss: device fp32[1]).  T: device fp32[batch][3].
   1 <= batch <= 65536. */
int gmresir_mlp_loss_grad(const float* params, const float* shift, const float* scale, const float* X,
                          const float* T, int32_t batch, float* grad, float* loss, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
   on the gradient of the batch loss, all on the device in one launch.
   adam_m, adam_v: device fp32[5443] moments.  loss: device fp32[1] (batch
   loss before the update). */
int gmresir_mlp_train_step(float* params, float* adam_m, float* adam_v, const float* shift, const float* scale,
                           const float* X, const float* T, int32_t batch, float lr, int32_t step, float* loss,
                           void* stream);

/* ---- host-side helpers (no GPU needed) --------------------------------- */

/* Eigenvalues of a real upper Hessenberg matrix (n <= 512, column-major,
   leading dimension ld) by the Francis double-shift QR algorithm; wr/wi:
   real and imaginary parts, conjugate pairs adjacent.  H is not modified. */
int gmresir_host_hessenberg_eigvals(int32_t n, const double* H_host, int32_t ld, double* wr_host,
                                    double* wi_host);

/* Harmonic Ritz values of a (k+1) x k Hessenberg matrix (column-major,
   leading dimension ld >= k+1), put in modified Leja order; out: 2k doubles. */
int gmresir_host_harmonic_ritz_leja(int32_t k, const double* Hbar_host, int32_t ld, double* roots_host);

const char* gmresir_status_string(int status);
const char* gmresir_last_error(void);
int32_t gmresir_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GMRESIR_H */
