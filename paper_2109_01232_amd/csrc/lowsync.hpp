// HIP kernels of the one-reduction CGS2 Arnoldi step (gfx950).
//
// Classical Gram-Schmidt applied twice (Section "GMRES"), with the second
// pass and the normalisation of each new vector delayed by one iteration so
// that an iteration needs one global reduction and two sweeps of the basis V
// instead of three reductions and three sweeps (the delayed
// reorthogonalisation of Bielich, Langou, Thomas, Swirydowicz, Yamazaki and
// Boman, "Low-synch Gram-Schmidt with delayed reorthogonalization for Krylov
// solvers", Parallel Computing 112, 2022).  Iteration j >= 1 starts from q_j,
// the previous iteration's vector after one Gram-Schmidt pass against
// Q = V[:, 0:j] (not normalised):
//
//   k_ls_spmv_dots_sell  p = A q_j (sliced ELLPACK SpMV) and, from the same
//                        rows, the partial sums of the one reduction:
//                        alpha = q.q, gam = q.p, a = Q^T q, c = Q^T p
//                        (k_spmv + k_ls_dots when the matrix has no sliced copy)
//   k_reduce_cols        the column sums (fixed order)
//   k_ls_dense           one block: rho = sqrt(alpha - a.a) (Pythagoras);
//                        Hessenberg column j-1 = first pass + a, subdiagonal
//                        rho, its Givens rotation (stop and breakdown tests);
//                        then, with t = H[0:j+1, 0:j] a (the Arnoldi relation
//                        A Q = V[:, 0:j+1] H of the completed columns), the
//                        first-pass coefficients of A v_j without another
//                        reduction: h_i = (c_i - t_i) / rho (i < j),
//                        h_j = ((gam - a.c) / rho - t_j) / rho, and the update
//                        coefficients d = t / rho + h
//   k_ls_update          v_j = (q_j - Q a) / rho into V[:, j] and
//                        q_{j+1} = p / rho - V[:, 0:j+1] d (both from one read
//                        of the rows of V; no reduction)
//
// Iteration 0 is the first pass of A v_0 alone (v_0 is formed on the fly from
// the cycle's right-hand side, as in the two-pass kernels); after the last
// iteration k_ls_dots (no SpMV) and k_ls_dense complete the last column.
#pragma once

#include "kernels.hpp"

namespace gir {

// restart lengths up to this many columns run the one-reduction cycle
constexpr int LS_MAX_RESTART = 128;
// basis-column loads of the fused reduction in flight per row group (150^3
// GMRES(100): 183.3 -> 163.9 us per launch against 169.5 us with 4)
constexpr int LS_PROJ_BATCH = 8;
// partial-sum columns of one reduction: alpha, gam, a[0..j), c[0..j)
constexpr int LS_ALPHA = 0, LS_GAM = 1, LS_A = 2;
constexpr int LS_PART_COLS = LS_A + 2 * LS_MAX_RESTART;

// Rows staged in LDS: own value q (or v_0) and the SpMV result p.  Wave w
// takes the columns c = w, w + NW, ... of the staged rows; each lane
// multiplies one group of G consecutive rows of a column (one 16-byte load)
// with both staged vectors, so every element of V is loaded once and used
// twice.
template <typename T, typename S, int SLOTS, int NW>
__device__ __forceinline__ void ls_project_rows(const S* __restrict__ V, long ldv, int C, int base, int nrows,
                                                const T* ps, const T* qs, T (&acc_a)[SLOTS], T (&acc_c)[SLOTS],
                                                int lane, int wid) {
  using PG = ProjGroup<S, T>;
  constexpr int G = PG::G;
  const bool aligned = (base % G) == 0;
  const int ngroups = (nrows + G - 1) / G;
  if (aligned) {
    // as project_rows: unconditional loads (columns past C read column 0 of
    // the same rows), LS_PROJ_BATCH in flight, rows past the stage masked
    constexpr int QB = SLOTS < LS_PROJ_BATCH ? SLOTS : LS_PROJ_BATCH;
    for (int g = lane; g < ngroups; g += WAVE) {
      const int rb = g * G;
      T pv[G], qv[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        pv[i] = zero_unless(ps[rb + i], rb + i < nrows);
        qv[i] = zero_unless(qs[rb + i], rb + i < nrows);
      }
#pragma unroll
      for (int s0 = 0; s0 < SLOTS; s0 += QB) {
        typename PG::raw rv[QB];
#pragma unroll
        for (int u = 0; u < QB; ++u) {
          const int c = wid + NW * (s0 + u);
          rv[u] = PG::load_raw(V + (size_t)(c < C ? c : 0) * ldv + base + rb);
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
          const int c = wid + NW * (s0 + u);
          if (c < C) {
#pragma unroll
            for (int i = 0; i < G; ++i) {
              const T v = zero_unless(PG::get(rv[u], i), rb + i < nrows);
              acc_a[s0 + u] += v * qv[i];
              acc_c[s0 + u] += v * pv[i];
            }
          }
        }
      }
    }
    return;
  }
  for (int g = lane; g < ngroups; g += WAVE) {
    const int rb = g * G;
    const bool full = aligned && rb + G <= nrows;
    T pv[G], qv[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      pv[i] = (rb + i < nrows) ? ps[rb + i] : T(0);
      qv[i] = (rb + i < nrows) ? qs[rb + i] : T(0);
    }
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int c = wid + NW * s;
      if (c < C) {
        T vv[G];
        if (full) {
          ProjGroup<S, T>::load(V + (size_t)c * ldv + base + rb, vv);
        } else {
#pragma unroll
          for (int i = 0; i < G; ++i)
            vv[i] = (rb + i < nrows) ? Basis<S, T>::load(V + (size_t)c * ldv + base + rb + i) : T(0);
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
          acc_a[s] += vv[i] * qv[i];
          acc_c[s] += vv[i] * pv[i];
        }
      }
    }
  }
}

// Block-wide end of a one-reduction producer: wave sums of the per-column
// accumulators and of the lanes' alpha / gam, combined over the waves in
// wave order, stored as partial column `col` of this block.
template <typename T, int SLOTS, int NW>
__device__ __forceinline__ void ls_store_partials(int C, bool has_p, T alpha, T gam, const T (&acc_a)[SLOTS],
                                                  const T (&acc_c)[SLOTS], T* s_ag, T* s_vals, T* __restrict__ part,
                                                  int lane, int wid) {
  alpha = wave_sum(alpha);
  gam = wave_sum(gam);
  if (lane == 0) {
    s_ag[2 * wid] = alpha;
    s_ag[2 * wid + 1] = gam;
  }
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int c = wid + NW * s;
    if (c < C) {
      const T va = wave_sum(acc_a[s]);
      const T vc = wave_sum(acc_c[s]);
      if (lane == 0) {
        s_vals[LS_A + c] = va;
        s_vals[LS_A + C + c] = vc;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    T a = s_ag[0], g = s_ag[1];
    for (int w = 1; w < NW; ++w) {
      a += s_ag[2 * w];
      g += s_ag[2 * w + 1];
    }
    s_vals[LS_ALPHA] = a;
    s_vals[LS_GAM] = has_p ? g : T(0);
  }
  __syncthreads();
  const int ncols = LS_A + (has_p ? 2 * C : C);
  for (int c = threadIdx.x; c < ncols; c += NW * WAVE) part[(size_t)c * MAX_BLOCKS + blockIdx.x] = s_vals[c];
}

// p = A q_j (or A v_0) over the sliced ELLPACK copy and the partial sums of
// the iteration's one reduction.  SCALED (iteration 0 without a
// preconditioner): the gathered vector is v_0 = round(src * inv), inv from the
// cycle start, and v_0 is stored as basis column 0; own[r] is then v_0[r].
// Otherwise the gather reads gsrc (q_j, or M^{-1} q_j with a preconditioner)
// and the own-row value comes from own (q_j, or v_0 at iteration 0).
template <typename T, typename S, int SLOTS, bool SCALED, int NW, bool WIDE>
__global__ __launch_bounds__(NW * WAVE) void k_ls_spmv_dots_sell(Csr A, const T* __restrict__ gsrc,
                                                              const T* __restrict__ own, S* __restrict__ V, long ldv,
                                                              int j, T* __restrict__ p_out, State st,
                                                              T* __restrict__ part) {
  const int flags = load_flags(st.hdr);  // tested after the prologue
  constexpr int STAGE = sizeof(T) == 8 ? TILE_ROWS : 2 * TILE_ROWS;
  constexpr int SPS = STAGE / SELL_C;  // slices per stage
  __shared__ T ps[STAGE];
  __shared__ T qs[STAGE];
  __shared__ T s_ag[2 * NW];
  __shared__ T s_vals[LS_A + 2 * NW * SLOTS];
  const T inv = SCALED ? (T)st.hdr->inv_h : T(1);
  if (flags & F_DONE) return;
  const XScaled<T, S> xs{gsrc, inv};
  const int C = j;  // basis columns projected (j <= NW * SLOTS)
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  T acc_a[SLOTS], acc_c[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) acc_a[s] = acc_c[s] = T(0);
  T alpha = T(0), gam = T(0);
  const int nstages = (A.nslices + SPS - 1) / SPS;
  const int B = gridDim.x, lb = logical_block();
  const int g0 = (int)((long)nstages * lb / B);
  const int g1 = (int)((long)nstages * (lb + 1) / B);
  for (int g = g0; g < g1; ++g) {
    for (int i = wid; i < SPS; i += NW) {
      const int sl = g * SPS + i;
      const int r = sl * SELL_C + lane;
      T y = T(0), qv = T(0);
      if (sl < A.nslices) {
        if (SCALED) y = sell_row<T, WIDE>(A, xs, sl, r, lane);
        else y = sell_row<T, WIDE>(A, XPlain<T>{gsrc}, sl, r, lane);
        if (r < A.n) {
          p_out[r] = y;
          if (SCALED) {
            qv = xs(r);
            Basis<S, T>::store(V + r, qv);
          } else {
            qv = own[r];
          }
          alpha += qv * qv;
          gam += qv * y;
        } else {
          y = T(0);
        }
      }
      ps[i * SELL_C + lane] = y;
      qs[i * SELL_C + lane] = qv;
    }
    __syncthreads();
    if (C > 0) {
      const int base = g * STAGE;
      const int nrows = A.n - base < STAGE ? A.n - base : STAGE;
      ls_project_rows<T, S, SLOTS, NW>(V, ldv, C, base, nrows, ps, qs, acc_a, acc_c, lane, wid);
    }
    __syncthreads();
  }
  ls_store_partials<T, SLOTS, NW>(C, true, alpha, gam, acc_a, acc_c, s_ag, s_vals, part, lane, wid);
}

// The same reduction from vectors in memory (no SpMV fused): q (and p when
// HAS_P) against the j basis columns.  The WV waves of a block share its rows
// and split the columns (wave w: c = w, w + WV, ...); wave 0 also sums
// alpha and gam.  Used after a plain SpMV when the matrix has no sliced copy,
// and (HAS_P = false) to complete a cycle's last column.
template <typename T, typename S, int SLOTS, bool HAS_P, int WV>
__global__ __launch_bounds__(WV * WAVE) void k_ls_dots(int n, const T* __restrict__ q, const T* __restrict__ p,
                                                       const S* __restrict__ V, long ldv, int j, State st,
                                                       T* __restrict__ part) {
  const int flags = load_flags(st.hdr);
  __shared__ T s_ag[2 * WV];
  __shared__ T s_vals[LS_A + 2 * WV * SLOTS];
  if (flags & F_DONE) return;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  T acc_a[SLOTS], acc_c[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) acc_a[s] = acc_c[s] = T(0);
  T alpha = T(0), gam = T(0);
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + lane; r < r1; r += WAVE) {
    const T qv = q[r];
    const T pv = HAS_P ? p[r] : T(0);
    if (wid == 0) {
      alpha += qv * qv;
      gam += qv * pv;
    }
    // every column's load unconditional (columns past j read column 0, not
    // used): under a branch each load was waited for before the next
    T vb[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int c = wid + WV * s;
      vb[s] = Basis<S, T>::load(V + (size_t)(c < j ? c : 0) * ldv + r);
    }
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int c = wid + WV * s;
      if (c < j) {
        acc_a[s] += vb[s] * qv;
        if (HAS_P) acc_c[s] += vb[s] * pv;
      }
    }
  }
  ls_store_partials<T, SLOTS, WV>(j, HAS_P, alpha, gam, acc_a, acc_c, s_ag, s_vals, part, lane, wid);
}

// v_0 = round(src * inv) into basis column 0 (iteration 0 of a cycle when the
// SpMV is not the fused sliced kernel); inv from the cycle start.
template <typename T, typename S>
__global__ __launch_bounds__(BLOCK) void k_ls_form_v0(int n, const T* __restrict__ src, S* __restrict__ V, State st) {
  const int flags = load_flags(st.hdr);
  const T inv = (T)st.hdr->inv_h;
  if (flags & F_DONE) return;
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) Basis<S, T>::store(V + r, Basis<S, T>::round(src[r] * inv));
}

// p = A x (plain SpMV), skipped once the cycle has stopped (matrices whose
// SpMV is not the fused sliced kernel).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_ls_spmv(Csr A, const T* __restrict__ x, T* __restrict__ y, State st) {
  if (load_flags(st.hdr) & F_DONE) return;  // the same value for the whole block
  T* prod = dyn_lds<T>();  // one entry per nonzero of the largest tile
  __shared__ T s_scr[NWAVES * WAVE];
  PlainEpi<T> epi{y};
  if (A.sell) sell_rows<T>(A, XPlain<T>{x}, epi);
  else spmv_tiles<T>(A, XPlain<T>{x}, epi, prod, s_scr);
}

// One block: complete Hessenberg column j-1 from the reduction (red: the
// column sums of k_reduce_cols in the LS_* layout), make its Givens step, and
// prepare iteration j's update (first-pass coefficients of A v_j into
// h1_of(j), update coefficients d, rho).  At j = 0 only the first pass of
// A v_0 (h = gam, rho = 1).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_ls_dense(State st, const double* __restrict__ red, double* __restrict__ dco,
                                                    int j, int kmax) {
  __shared__ T s_a[LS_MAX_RESTART + 1];
  __shared__ T s_c[LS_MAX_RESTART + 1];
  __shared__ T s_t[LS_MAX_RESTART + 2];
  __shared__ T s_col[MAX_RESTART + 2];
  __shared__ T s_cs[MAX_RESTART];
  __shared__ T s_sn[MAX_RESTART];
  __shared__ T s_red[16];
  StateHdr* hd = st.hdr;
  if (load_flags(hd) & F_DONE) return;
  if (j == 0) {
    if (threadIdx.x == 0) {
      const T h = (T)red[LS_GAM];
      st.h1_of(0)[0] = (double)h;
      dco[0] = (double)h;
      hd->lsrho = 1.0;
    }
    return;
  }
  // second-pass coefficients a of column j-1 (h2), and a.a
  T aa = T(0);
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    const T a = (T)red[LS_A + i];
    s_a[i] = a;
    st.h2[i] = (double)a;
    aa += a * a;
  }
  aa = block_sum_any(aa, s_red);  // ends with a barrier: s_a and h2 complete
  const T nrm2 = fmax((T)red[LS_ALPHA] - aa, T(0));
  const int flags = givens_tail<T>(st, j - 1, kmax, nrm2, s_col, s_cs, s_sn);
  if (flags & F_DONE) return;  // stop, breakdown, NaN, or the cycle's last column
  const T rho = sqrt(nrm2);
  const int ld = st.ld;
  // H[0:j+1, 0:j] staged in LDS (dynamic, (j + 1) j entries) with coalesced
  // loads of whole columns; a row-by-row walk through global memory made this
  // block latency bound (j dependent-address loads per thread).  The loads are
  // unconditional (a load under a branch is waited for where the branch ends,
  // which made the batch one round trip per load): past the end a thread
  // reads entry 0, and every (l, i) with l < j <= m, i <= j lies inside the
  // (m + 1) x m array; entries below the subdiagonal are discarded after the
  // load.  The empty asm keeps each load ahead of the branch of its store.
  T* sH = dyn_lds<T>();
  const int hj = j + 1;
  const int tot = hj * j;
  constexpr int BATCH = 16;  // loads in flight per thread before their LDS stores
  for (int e0 = 0; e0 < tot; e0 += BLOCK * BATCH) {
    double v[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + (int)threadIdx.x + BLOCK * u;
      const int ec = e < tot ? e : 0;
      const int l = ec / hj, i = ec - l * hj;
      v[u] = st.Hbar[(size_t)l * ld + i];
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) asm volatile("" : "+v"(v[u]));
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + (int)threadIdx.x + BLOCK * u;
      const int l = e / hj, i = e - l * hj;
      if (e < tot) sH[e] = i <= l + 1 ? (T)v[u] : T(0);
    }
  }
  __syncthreads();
  // t = H[0:j+1, 0:j] a (upper Hessenberg: row i starts at column i - 1),
  // unrolled so several LDS reads are in flight
  T ac = T(0);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    T t = T(0);
#pragma unroll 8
    for (int l = i > 0 ? i - 1 : 0; l < j; ++l) t += sH[l * hj + i] * s_a[l];
    s_t[i] = t;
    if (i < j) {
      const T c = (T)red[LS_A + j + i];
      s_c[i] = c;
      ac += s_a[i] * c;
    }
  }
  ac = block_sum_any(ac, s_red);  // ends with a barrier: s_t, s_c complete
  const T gam = (T)red[LS_GAM];
  double* h1 = st.h1_of(j);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    const T h = i < j ? (s_c[i] - s_t[i]) / rho : ((gam - ac) / rho - s_t[j]) / rho;
    h1[i] = (double)h;
    dco[i] = (double)(s_t[i] / rho + h);
  }
  if (threadIdx.x == 0) hd->lsrho = (double)rho;
}

// v_j = round((q - Q a) / rho) into V[:, j] and, in place,
// q <- p / rho - V[:, 0:j+1] d (j = 0: v_0 is read from V[:, 0], rho = 1).
// Four rows per lane (16-byte loads for fp32); padded rows past n are masked.
// NT = 512 threads: the row grid is capped at MAX_BLOCKS blocks, and eight
// waves per block fill the CUs' wave slots.
template <typename T, typename S, int NT>
__global__ __launch_bounds__(NT) void k_ls_update(int n, const T* __restrict__ p, T* __restrict__ q,
                                                  S* __restrict__ V, long ldv, int j, State st,
                                                  const double* __restrict__ dco) {
  const int flags = load_flags(st.hdr);  // tested after the coefficients are staged
  __shared__ T s_a[LS_MAX_RESTART + 1];
  __shared__ T s_d[LS_MAX_RESTART + 1];
  for (int c = threadIdx.x; c <= j; c += NT) {
    s_a[c] = c < j ? (T)st.h2[c] : T(0);
    s_d[c] = (T)dco[c];
  }
  const T rho = j > 0 ? (T)st.hdr->lsrho : T(1);
  __syncthreads();
  if (flags & F_DONE) return;
  const T dj = s_d[j];
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + 4 * threadIdx.x; r < r1; r += 4 * NT) {
    const int nv = r1 - r < 4 ? r1 - r : 4;
    T pv[4], qv[4], sa[4] = {T(0), T(0), T(0), T(0)}, sd[4] = {T(0), T(0), T(0), T(0)};
    Quad<T, T>::load(p + r, pv);
    if (j > 0) Quad<T, T>::load(q + r, qv);
#pragma unroll 4
    for (int c = 0; c < j; ++c) {
      T v[4];
      Quad<S, T>::load(V + (size_t)c * ldv + r, v);
      const T a = s_a[c], d = s_d[c];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        sa[i] += v[i] * a;
        sd[i] += v[i] * d;
      }
    }
    T vj[4], out[4];
    if (j > 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) vj[i] = Basis<S, T>::round((qv[i] - sa[i]) / rho);
#pragma unroll
      for (int i = 0; i < 4; ++i) out[i] = pv[i] / rho - (sd[i] + vj[i] * dj);
    } else {
      Quad<S, T>::load(V + r, vj);
#pragma unroll
      for (int i = 0; i < 4; ++i) out[i] = pv[i] - vj[i] * dj;
    }
    if (nv == 4) {
      QuadStore<T>::store(q + r, out);
      if (j > 0) {
        if constexpr (sizeof(S) == sizeof(T)) QuadStore<T>::store((T*)(V + (size_t)j * ldv + r), vj);
      }
    } else {
      for (int i = 0; i < nv; ++i) {
        q[r + i] = out[i];
        if (j > 0) Basis<S, T>::store(V + (size_t)j * ldv + r + i, vj[i]);
      }
    }
  }
}

}  // namespace gir
