// HIP kernels of the GMRES-IR hot path (gfx950).
//
// One inner GMRES iteration (Algorithm 1 with two classical Gram-Schmidt
// passes, Section "GMRES") is three kernels that each sweep the Krylov basis
// V once -- the minimum for two-pass CGS -- plus two one-block tails that
// finish the cross-block sums:
//   k_spmv_proj    w = A v_j (row-tiled CSR SpMV, products staged in LDS)
//                  and h1 = V^T w from the same rows (first-pass projection).
//                  v_j itself is formed on the fly as round(wtmp / ||wtmp||)
//                  and stored into V, so no separate normalisation pass.
//   k_reduce_h1_givens  sums h1 (one wave per column) and, in one more
//                  block, forms the previous Hessenberg column, applies the
//                  earlier Givens rotations, makes the new one and updates
//                  the implicit residual (the paper's host-side least-squares
//                  step, moved to the device so a cycle needs no host round
//                  trip).
//   k_update_proj  w' = w - V h1 and h2 = V^T w' (each row of V is loaded
//                  into registers once and used for both).
//   k_reduce_cols  sums h2.
//   k_update_norm  w'' = w' - V h2 and the partial sums of ||w''||^2.
// Every reduction is two-stage with a fixed summation order, so results are
// bitwise reproducible run to run.
#pragma once

#include "device.hpp"

namespace gir {

constexpr int MAX_RESTART = 512;

// ---------------------------------------------------------------------------
// source-vector accessors of the SpMV gather
// ---------------------------------------------------------------------------

// v = round_to_basis(src * inv): the next basis vector built from the
// unnormalised vector of the previous iteration.
template <typename T, typename S>
struct XScaled {
  const T* src;
  T inv;
  __device__ __forceinline__ T operator()(int c) const { return Basis<S, T>::round(src[c] * inv); }
};

template <typename T>
struct XPlain {
  const T* src;
  __device__ __forceinline__ T operator()(int c) const { return src[c]; }
};

// prod[i] = vals[p0 + i] * x(col[p0 + i]) for i < len (a tile staged in LDS).
// The loads of SPMV_UNROLL nonzeros per thread are issued before their
// gathers, and the gathers before the products, so a tile costs two memory
// round trips per batch instead of one per nonzero.  Each product is rounded
// on its own (no fused multiply-add with the row sum).
template <typename T, typename XF>
__device__ __forceinline__ void stage_products(const Csr& A, int p0, int len, const XF& xf, T* prod) {
  const T* vals = (const T*)A.vals;
  for (int i0 = 0; i0 < len; i0 += BLOCK * SPMV_UNROLL) {
    int cc[SPMV_UNROLL];
    T vv[SPMV_UNROLL], xv[SPMV_UNROLL];
#pragma unroll
    for (int k = 0; k < SPMV_UNROLL; ++k) {
      const int i = i0 + (int)threadIdx.x + k * BLOCK;
      const int ic = i < len ? i : len - 1;
      cc[k] = A.col[p0 + ic];
      vv[k] = vals[p0 + ic];
    }
#pragma unroll
    for (int k = 0; k < SPMV_UNROLL; ++k) xv[k] = xf(cc[k]);
#pragma unroll
    for (int k = 0; k < SPMV_UNROLL; ++k) {
      const int i = i0 + (int)threadIdx.x + k * BLOCK;
      if (i < len) prod[i] = vv[k] * xv[k];
    }
  }
}

// One row of the sliced ELLPACK copy, summed in column order by the lane that
// owns it (the same order, and so the same bits, as the tiled CSR kernels).
// Loads of U entries are issued before their gathers; padding entries past
// the row length are loaded (valid addresses) but not added.
// LAYOUT 1: 32-bit columns; 2: 16-bit offsets from the row (rows past n: from
// row 0); 3: the slice's shared offsets (a wave-uniform load), every slot
// added -- an absent entry adds 0 * x[c] = +-0 to a sum that started at +0,
// which leaves it unchanged (x finite), so the bits match the CSR row sum --
// and the gathered index clamped to [0, n) (absent neighbours, rows past n).
template <typename T, int LAYOUT, int U, typename XF>
__device__ __forceinline__ T sell_row_cols(const Csr& A, const XF& xf, int s, int r, int lane, int base, int K) {
#pragma clang fp contract(off)
  const T* vals = (const T*)A.svals;
  const int len = LAYOUT == 3 ? K : (r < A.n ? A.rowptr[r + 1] - A.rowptr[r] : 0);
  const int rr = r < A.n ? r : 0;
  const int* soff = A.scol + base / SELL_C;
  T sum = T(0);
  for (int k0 = 0; k0 < K; k0 += U) {
    int cc[U];
    T vv[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u < K ? k0 + u : K - 1;
      if constexpr (LAYOUT == 3) cc[u] = min(max(r + soff[k], 0), A.n - 1);
      else if constexpr (LAYOUT == 2) cc[u] = rr + (int)A.scol16[base + SELL_C * k + lane];
      else cc[u] = A.scol[base + SELL_C * k + lane];
      vv[u] = vals[base + SELL_C * k + lane];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = xf(cc[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T p = vv[u] * xv[u];
      if (k0 + u < len) sum = sum + p;
    }
  }
  return sum;
}

// The entries whose loads go out together follow the slice's width K (a
// wave-uniform value): rounds of U in {5, 7, 9} entries, the U that loads the
// fewest padded entries (ceil(K / U) U), the larger U on ties -- a 27-point
// row in three rounds of 9, a 13-point one in two of 7, a 19-point one in
// four of 5 (measured: 27-point 128^3 SpMV + projection 124 -> 119 us with 9
// instead of 5; rounds of 9 on 5-, 13- and 19-entry rows, which load 4, 5
// and 8 entries for nothing, ran 5-15 % slower).
__device__ __forceinline__ int sell_round(int K) {
  const int l5 = (K + 4) / 5 * 5, l7 = (K + 6) / 7 * 7, l9 = (K + 8) / 9 * 9;
  return (l9 <= l7 && l9 <= l5) ? 9 : (l7 <= l5 ? 7 : 5);
}

template <typename T, int LAYOUT, bool WIDE, typename XF>
__device__ __forceinline__ T sell_row_k(const Csr& A, const XF& xf, int s, int r, int lane) {
  const int base = A.sptr[s];
  const int K = (A.sptr[s + 1] - base) / SELL_C;
  // WIDE (shared offsets, slices wider than 9): no index registers per entry,
  // so a slice 10..27 wide issues all its loads in one round (27-point 128^3
  // SpMV + projection 94 -> 93 us fp32, 76 -> 69 us with a bf16 basis, against
  // rounds of 9; 19-point fp64 SpMV 77 -> 73 us).  A template choice: the
  // wide rounds' registers would cost the narrow stencils occupancy (7-point
  // 150^3 one-reduction SpMV 184 -> 221 us when compiled in).
  if constexpr (LAYOUT == 3 && WIDE) {
    if (K > 9 && K <= 14) return sell_row_cols<T, LAYOUT, 14>(A, xf, s, r, lane, base, K);
    if (K > 14 && K <= 19) return sell_row_cols<T, LAYOUT, 19>(A, xf, s, r, lane, base, K);
    if (K > 19 && K <= 27) return sell_row_cols<T, LAYOUT, 27>(A, xf, s, r, lane, base, K);
  }
  const int U = sell_round(K);
  if (U == 5) return sell_row_cols<T, LAYOUT, 5>(A, xf, s, r, lane, base, K);
  if (U == 7) return sell_row_cols<T, LAYOUT, 7>(A, xf, s, r, lane, base, K);
  return sell_row_cols<T, LAYOUT, 9>(A, xf, s, r, lane, base, K);
}

// The layout and the round size are chosen once per slice (wave-uniform
// branches), not per load: a load under a branch is waited for at the
// branch's end.
template <typename T, bool WIDE = false, typename XF>
__device__ __forceinline__ T sell_row(const Csr& A, const XF& xf, int s, int r, int lane) {
  if (A.shared) return sell_row_k<T, 3, WIDE>(A, xf, s, r, lane);
  return A.d16 ? sell_row_k<T, 2, false>(A, xf, s, r, lane) : sell_row_k<T, 1, false>(A, xf, s, r, lane);
}

// SpMV over the sliced ELLPACK copy: the block takes a contiguous range of
// slices, its waves take every fourth of them, each lane one row; epi(r, y)
// per row as in spmv_tiles.
template <typename T, bool WIDE = false, typename XF, typename EPI>
__device__ __forceinline__ void sell_rows(const Csr& A, const XF& xf, EPI& epi) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int B = gridDim.x, lb = logical_block();
  const int s0 = (int)((long)A.nslices * lb / B);
  const int s1 = (int)((long)A.nslices * (lb + 1) / B);
  for (int s = s0 + wid; s < s1; s += NWAVES) {
    const int r = s * SELL_C + lane;
    const T y = sell_row<T, WIDE>(A, xf, s, r, lane);
    if (r < A.n) epi(r, y);
  }
}

// Row-tiled CSR SpMV: a block takes a contiguous range of tiles; per tile the
// nonzeros are streamed with coalesced loads, multiplied by the gathered x and
// staged in LDS, then each thread sums one row in column order.  epi(r, y) is
// called once per row by the thread owning it.
template <typename T, typename XF, typename EPI>
__device__ __forceinline__ void spmv_tiles(const Csr& A, const XF& xf, EPI& epi, T* prod, T* red) {
  const T* vals = (const T*)A.vals;
  const int B = gridDim.x, lb = logical_block();
  const int t0 = (int)((long)A.ntiles * lb / B);
  const int t1 = (int)((long)A.ntiles * (lb + 1) / B);
  for (int t = t0; t < t1; ++t) {
    const int r0 = A.tile_row[t], r1 = A.tile_row[t + 1];
    const int p0 = A.rowptr[r0], p1 = A.rowptr[r1];
    const int len = p1 - p0;
    if (len <= TILE_NNZ) {
      stage_products<T>(A, p0, len, xf, prod);
      __syncthreads();
      for (int rr = threadIdx.x; rr < r1 - r0; rr += BLOCK) {
        const int r = r0 + rr;
        const int q0 = A.rowptr[r] - p0, q1 = A.rowptr[r + 1] - p0;
        T s = T(0);
        for (int q = q0; q < q1; ++q) s += prod[q];
        epi(r, s);
      }
      __syncthreads();
    } else {
      // a single row longer than a tile: block-wide dot product
      T s = T(0);
      for (int i = threadIdx.x; i < len; i += BLOCK) s += vals[p0 + i] * xf(A.col[p0 + i]);
      s = block_sum(s, red);
      if (threadIdx.x == 0) epi(r0, s);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// first kernel of an iteration: SpMV + first-pass projection
// ---------------------------------------------------------------------------

// Four consecutive basis entries (rows r..r+3 of one column, r % 4 == 0) with
// one 16-byte (fp32, 2 x fp64) or 8-byte (bf16) load.
template <typename S, typename T>
struct Quad;
template <>
struct Quad<float, float> {
  static __device__ __forceinline__ void load(const float* p, float (&v)[4]) {
    const float4 q = *(const float4*)p;
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  }
};
template <>
struct Quad<double, double> {
  static __device__ __forceinline__ void load(const double* p, double (&v)[4]) {
    const double2 a = *(const double2*)p;
    const double2 b = *(const double2*)(p + 2);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
  }
};
template <>
struct Quad<bf16_t, float> {
  static __device__ __forceinline__ void load(const bf16_t* p, float (&v)[4]) {
    const uint2 q = *(const uint2*)p;
    v[0] = __uint_as_float(q.x << 16);
    v[1] = __uint_as_float(q.x & 0xffff0000u);
    v[2] = __uint_as_float(q.y << 16);
    v[3] = __uint_as_float(q.y & 0xffff0000u);
  }
};

// Two consecutive entries (rows r, r+1; r even) with one 8-byte (fp32),
// 16-byte (fp64) or 4-byte (bf16) load.
template <typename S, typename T>
struct Pair;
template <>
struct Pair<float, float> {
  static __device__ __forceinline__ void load(const float* p, float (&v)[2]) {
    const float2 q = *(const float2*)p;
    v[0] = q.x;
    v[1] = q.y;
  }
  static __device__ __forceinline__ void store(float* p, const float (&v)[2]) { *(float2*)p = make_float2(v[0], v[1]); }
};
template <>
struct Pair<double, double> {
  static __device__ __forceinline__ void load(const double* p, double (&v)[2]) {
    const double2 q = *(const double2*)p;
    v[0] = q.x;
    v[1] = q.y;
  }
  static __device__ __forceinline__ void store(double* p, const double (&v)[2]) {
    *(double2*)p = make_double2(v[0], v[1]);
  }
};
template <>
struct Pair<bf16_t, float> {
  static __device__ __forceinline__ void load(const bf16_t* p, float (&v)[2]) {
    const uint32_t q = *(const uint32_t*)p;
    v[0] = __uint_as_float(q << 16);
    v[1] = __uint_as_float(q & 0xffff0000u);
  }
};

template <typename T>
struct QuadStore;
template <>
struct QuadStore<float> {
  static __device__ __forceinline__ void store(float* p, const float (&v)[4]) {
    *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
  }
};
template <>
struct QuadStore<double> {
  static __device__ __forceinline__ void store(double* p, const double (&v)[4]) {
    *(double2*)p = make_double2(v[0], v[1]);
    *(double2*)(p + 2) = make_double2(v[2], v[3]);
  }
};

// R consecutive rows of one basis column as one vector load, kept packed in
// registers (bf16: 8 rows in 16 bytes) and unpacked to T on use.
template <typename S, typename T, int R>
struct Packed;
template <>
struct Packed<float, float, 4> {
  using type = float4;
  static __device__ __forceinline__ type load(const float* p) { return *(const float4*)p; }
  static __device__ __forceinline__ type zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  static __device__ __forceinline__ float get(const type& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
  static __device__ __forceinline__ void hold(type&) {}
};
template <>
struct Packed<double, double, 2> {
  using type = double2;
  static __device__ __forceinline__ type load(const double* p) { return *(const double2*)p; }
  static __device__ __forceinline__ type zero() { return make_double2(0.0, 0.0); }
  static __device__ __forceinline__ double get(const type& v, int i) { return i == 0 ? v.x : v.y; }
  static __device__ __forceinline__ void hold(type&) {}
};
template <>
struct Packed<double, double, 1> {
  using type = double;
  static __device__ __forceinline__ type load(const double* p) { return *p; }
  static __device__ __forceinline__ type zero() { return 0.0; }
  static __device__ __forceinline__ double get(const type& v, int) { return v; }
  static __device__ __forceinline__ void hold(type&) {}
};
template <>
struct Packed<bf16_t, float, 8> {
  using type = uint4;
  static __device__ __forceinline__ type load(const bf16_t* p) { return *(const uint4*)p; }
  static __device__ __forceinline__ type zero() { return make_uint4(0u, 0u, 0u, 0u); }
  static __device__ __forceinline__ float get(const type& v, int i) {
    const uint32_t w = (i >> 1) == 0 ? v.x : (i >> 1) == 1 ? v.y : (i >> 1) == 2 ? v.z : v.w;
    return __uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
  }
  // keeps the 8 rows packed between their two uses (otherwise the compiler
  // holds all 8 unpacked values, twice the registers)
  static __device__ __forceinline__ void hold(type& v) { asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w)); }
};

template <>
struct Packed<bf16_t, float, 4> {
  using type = uint2;
  static __device__ __forceinline__ type load(const bf16_t* p) { return *(const uint2*)p; }
  static __device__ __forceinline__ type zero() { return make_uint2(0u, 0u); }
  static __device__ __forceinline__ float get(const type& v, int i) {
    const uint32_t w = (i >> 1) == 0 ? v.x : v.y;
    return __uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
  }
  static __device__ __forceinline__ void hold(type& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }
};

// 1 / ||w''|| of the previous iteration, the scale of the next basis vector:
// summed from the partials k_update_norm left (nB > 0) in the order the
// Givens step sums them (so both get the same bits), or read from the state
// at a cycle start (nB == 0).  Called by every thread of the block.
template <typename T>
__device__ __forceinline__ T prev_inv_norm(const State& st, const T* norm_part, int nB) {
  if (nB == 0) return (T)st.hdr->inv_h;
  __shared__ T s_n[1];
  reduce_partials(norm_part, 1, nB, s_n);
  return T(1) / sqrt(s_n[0]);
}

// x where keep holds, else +0 (also for NaN x: the padded rows past n are
// never written), by a bit mask: a select fed by LDS reads is turned into a
// branch by the compiler, and a branch makes its waits for memory inexact
__device__ __forceinline__ float zero_unless(float x, bool keep) {
  return __uint_as_float(__float_as_uint(x) & (keep ? 0xffffffffu : 0u));
}
__device__ __forceinline__ double zero_unless(double x, bool keep) {
  return __longlong_as_double(__double_as_longlong(x) & (keep ? -1ll : 0ll));
}

// Basis-column loads of the fused projection issued together per row group
// (one 16-byte load each).  Written as branches, each column's load was
// waited for before the next one went out; a batch keeps PROJ_BATCH in
// flight at a moderate register cost (27-point 128^3 SpMV + projection 92.6
// -> 88.7 us, 150^3 169.3 -> 165.3 us; batches of 8 and 16 measured no better
// here, having fewer blocks per CU).
constexpr int PROJ_BATCH = 4;

// w = A v_j and the partial sums of h1 = V_{j+1}^T w.
//
// Per tile: the SpMV products are staged in LDS and summed per row (one
// thread per row); the row results y and (SCALED) the new basis vector
// v_j = round(wtmp / ||wtmp||) are staged in LDS, v_j is stored into V[:, j].
// Consecutive tiles of the block are staged until up to 1024 rows (fp32;
// 512 for fp64) are collected (a 27-point tile has ~95 rows, a 7-point one
// ~365), then wave w takes the columns
// c = w, w + 4, ... of those rows and each lane multiplies a group of
// consecutive rows of a column (one 16-byte load: 4 fp32 or 8 bf16 rows) with
// the staged y.  Each lane keeps
// SLOTS running sums (k/4 registers instead of k), reduced across the wave
// once at the end.  Columns c >= 4*SLOTS are left to k_dots.
template <typename S, typename T>
struct ProjGroup;  // rows per lane of the projection: one 16-byte load (fp64: two)
template <>
struct ProjGroup<float, float> {
  static constexpr int G = 4;
  using raw = float4;
  static __device__ __forceinline__ raw load_raw(const float* p) { return *(const float4*)p; }
  static __device__ __forceinline__ float get(const raw& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
  static __device__ __forceinline__ void load(const float* p, float (&v)[4]) { Quad<float, float>::load(p, v); }
};
struct Double4 {
  double2 lo, hi;
};
template <>
struct ProjGroup<double, double> {
  static constexpr int G = 4;
  using raw = Double4;
  static __device__ __forceinline__ raw load_raw(const double* p) { return {*(const double2*)p, *(const double2*)(p + 2)}; }
  static __device__ __forceinline__ double get(const raw& v, int i) {
    return i == 0 ? v.lo.x : i == 1 ? v.lo.y : i == 2 ? v.hi.x : v.hi.y;
  }
  static __device__ __forceinline__ void load(const double* p, double (&v)[4]) { Quad<double, double>::load(p, v); }
};
template <>
struct ProjGroup<bf16_t, float> {
  static constexpr int G = 8;
  using raw = uint4;
  static __device__ __forceinline__ raw load_raw(const bf16_t* p) { return *(const uint4*)p; }
  static __device__ __forceinline__ float get(const raw& v, int i) { return Packed<bf16_t, float, 8>::get(v, i); }
  static __device__ __forceinline__ void load(const bf16_t* p, float (&v)[8]) {
    const uint4 q = *(const uint4*)p;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = Packed<bf16_t, float, 8>::get(q, i);
  }
};

template <typename T, typename S, int SLOTS, bool SCALED, int NW = NWAVES>
__device__ __forceinline__ void project_rows(const S* __restrict__ V, long ldv, int j, int C, int base, int nrows,
                                             const T* ys, const T* vs, T (&acc)[SLOTS], int lane, int wid) {
  using PG = ProjGroup<S, T>;
  constexpr int G = PG::G;
  const bool aligned = (base % G) == 0;
  const int ngroups = (nrows + G - 1) / G;
  if (aligned) {
    // every load unconditional: columns past C, and column j (whose values
    // come from vs), read column 0 of the same rows, which lie below the
    // padded length ldv; rows past the batch are masked by bit, since the
    // padded rows past n are never written
    constexpr int QB = SLOTS < PROJ_BATCH ? SLOTS : PROJ_BATCH;
    for (int g = lane; g < ngroups; g += WAVE) {
      const int rb = g * G;
      T yv[G];
#pragma unroll
      for (int i = 0; i < G; ++i) yv[i] = zero_unless(ys[rb + i], rb + i < nrows);
#pragma unroll
      for (int q0 = 0; q0 < SLOTS; q0 += QB) {
        typename PG::raw rv[QB];
#pragma unroll
        for (int u = 0; u < QB; ++u) {
          const int c = wid + NW * (q0 + u);
          const bool from_v = c < C && !(SCALED && c == j);
          rv[u] = PG::load_raw(V + (size_t)(from_v ? c : 0) * ldv + base + rb);
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
          const int c = wid + NW * (q0 + u);
          if (c < C) {
            T vv[G];
            if (SCALED && c == j) {
#pragma unroll
              for (int i = 0; i < G; ++i) vv[i] = zero_unless(vs[rb + i], rb + i < nrows);
            } else {
#pragma unroll
              for (int i = 0; i < G; ++i) vv[i] = zero_unless(PG::get(rv[u], i), rb + i < nrows);
            }
#pragma unroll
            for (int i = 0; i < G; ++i) acc[q0 + u] += vv[i] * yv[i];
          }
        }
      }
    }
    return;
  }
  for (int g = lane; g < ngroups; g += WAVE) {
    const int rb = g * G;
    const bool full = aligned && rb + G <= nrows;
    T yv[G];
#pragma unroll
    for (int i = 0; i < G; ++i) yv[i] = (rb + i < nrows) ? ys[rb + i] : T(0);
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
      const int c = wid + NW * q;
      if (c < C) {
        T vv[G];
        if (SCALED && c == j) {
#pragma unroll
          for (int i = 0; i < G; ++i) vv[i] = (rb + i < nrows) ? vs[rb + i] : T(0);
        } else if (full) {
          ProjGroup<S, T>::load(V + (size_t)c * ldv + base + rb, vv);
        } else {
#pragma unroll
          for (int i = 0; i < G; ++i)
            vv[i] = (rb + i < nrows) ? Basis<S, T>::load(V + (size_t)c * ldv + base + rb + i) : T(0);
        }
#pragma unroll
        for (int i = 0; i < G; ++i) acc[q] += vv[i] * yv[i];
      }
    }
  }
}

template <typename T, typename S, int SLOTS, bool SCALED>
__global__ __launch_bounds__(BLOCK) void k_spmv_proj(Csr A, const T* __restrict__ src, S* __restrict__ V, long ldv,
                                                     int j, T* __restrict__ w_out, State st, T* __restrict__ part,
                                                     const T* __restrict__ norm_part, int nB) {
  // the stop flag is read first and tested after the prologue, whose loads
  // are harmless either way: one memory round trip instead of two
  const int flags = load_flags(st.hdr);
  constexpr int KMAX = NWAVES * SLOTS;
  // rows staged for one projection pass: several short tiles at once, so
  // the 64 lanes of a wave get whole groups of 4 rows (fp64 keeps 512 rows
  // to leave LDS for occupancy)
  constexpr int STAGE_ROWS = sizeof(T) == 8 ? TILE_ROWS : 2 * TILE_ROWS;
  T* prod = dyn_lds<T>();  // one entry per nonzero of the largest tile
  __shared__ T ys[STAGE_ROWS];
  __shared__ T vs[STAGE_ROWS];
  __shared__ T s_vals[KMAX];
  __shared__ T s_red[NWAVES];
  const T* vals = (const T*)A.vals;
  const T inv = SCALED ? prev_inv_norm<T>(st, norm_part, nB) : T(1);
  if (flags & F_DONE) return;
  const XScaled<T, S> xs{src, inv};
  const int C = (j + 1 < KMAX) ? j + 1 : KMAX;  // columns handled here
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  T acc[SLOTS];
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) acc[q] = T(0);
  const int B = gridDim.x, lb = logical_block();
  const int t0 = (int)((long)A.ntiles * lb / B);
  const int t1 = (int)((long)A.ntiles * (lb + 1) / B);
  int base = t0 < t1 ? A.tile_row[t0] : 0;  // first row staged in ys / vs
  int end = base;                            // one past the last staged row
  for (int t = t0; t < t1; ++t) {
    const int r0 = A.tile_row[t], r1 = A.tile_row[t + 1];
    const int p0 = A.rowptr[r0], p1 = A.rowptr[r1];
    const int len = p1 - p0;
    const int nrows = r1 - r0;
    if (r1 - base > STAGE_ROWS) {
      // the staged rows are full: project them, then start a new batch
      project_rows<T, S, SLOTS, SCALED>(V, ldv, j, C, base, end - base, ys, vs, acc, lane, wid);
      __syncthreads();
      base = r0;
    }
    const int off = r0 - base;
    if (len <= TILE_NNZ) {
      if (SCALED) stage_products<T>(A, p0, len, xs, prod);
      else stage_products<T>(A, p0, len, XPlain<T>{src}, prod);
      __syncthreads();
      for (int rr = threadIdx.x; rr < nrows; rr += BLOCK) {
        const int r = r0 + rr;
        const int q0 = A.rowptr[r] - p0, q1 = A.rowptr[r + 1] - p0;
        T y = T(0);
        for (int q = q0; q < q1; ++q) y += prod[q];
        w_out[r] = y;
        ys[off + rr] = y;
        if (SCALED) {
          const T vj = xs(r);
          Basis<S, T>::store(V + (size_t)j * ldv + r, vj);
          vs[off + rr] = vj;
        }
      }
    } else {
      // a single row longer than a tile: block-wide dot product
      T y = T(0);
      for (int i = threadIdx.x; i < len; i += BLOCK) y += vals[p0 + i] * (SCALED ? xs(A.col[p0 + i]) : src[A.col[p0 + i]]);
      y = block_sum(y, s_red);
      if (threadIdx.x == 0) {
        w_out[r0] = y;
        ys[off] = y;
        if (SCALED) {
          const T vj = xs(r0);
          Basis<S, T>::store(V + (size_t)j * ldv + r0, vj);
          vs[off] = vj;
        }
      }
    }
    end = r1;
    __syncthreads();  // y staged; prod free for the next tile
  }
  if (end > base) project_rows<T, S, SLOTS, SCALED>(V, ldv, j, C, base, end - base, ys, vs, acc, lane, wid);
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) {
    const int c = wid + NWAVES * q;
    if (c < C) {
      const T v = wave_sum(acc[q]);
      if (lane == 0) s_vals[c] = v;
    }
  }
  __syncthreads();
  store_partials(s_vals, C, part);
}

// The same over the sliced ELLPACK copy: a block of NW waves takes a
// contiguous range of stages of STAGE rows (16 slices in fp32, 8 in fp64); per
// stage each wave sums its slices' rows (one row per lane), stores w and v_j
// and stages them in LDS, then the block projects the stage's rows as above
// (wave w: columns w, w + NW, ...).  Eight waves per block double the loads in
// flight per CU at the same number of blocks, and so of partial sums.
template <typename T, typename S, int SLOTS, bool SCALED, int NW, bool WIDE>
__global__ __launch_bounds__(NW * WAVE) void k_spmv_proj_sell(Csr A, const T* __restrict__ src, S* __restrict__ V,
                                                          long ldv, int j, T* __restrict__ w_out, State st,
                                                          T* __restrict__ part, const T* __restrict__ norm_part,
                                                          int nB) {
  const int flags = load_flags(st.hdr);  // tested after the prologue, as above
  constexpr int KMAX = NW * SLOTS;
  constexpr int STAGE = sizeof(T) == 8 ? TILE_ROWS : 2 * TILE_ROWS;
  constexpr int SPS = STAGE / SELL_C;  // slices per stage
  __shared__ T ys[STAGE];
  __shared__ T vs[STAGE];
  __shared__ T s_vals[KMAX];
  const T inv = SCALED ? prev_inv_norm<T>(st, norm_part, nB) : T(1);
  if (flags & F_DONE) return;
  const XScaled<T, S> xs{src, inv};
  const int C = (j + 1 < KMAX) ? j + 1 : KMAX;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  T acc[SLOTS];
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) acc[q] = T(0);
  const int nstages = (A.nslices + SPS - 1) / SPS;
  const int B = gridDim.x, lb = logical_block();
  const int g0 = (int)((long)nstages * lb / B);
  const int g1 = (int)((long)nstages * (lb + 1) / B);
  for (int g = g0; g < g1; ++g) {
    for (int i = wid; i < SPS; i += NW) {
      const int sl = g * SPS + i;
      const int r = sl * SELL_C + lane;
      T y = T(0), vj = T(0);
      if (sl < A.nslices) {
        if (SCALED) y = sell_row<T, WIDE>(A, xs, sl, r, lane);
        else y = sell_row<T, WIDE>(A, XPlain<T>{src}, sl, r, lane);
        if (r < A.n) {
          w_out[r] = y;
          if (SCALED) {
            vj = xs(r);
            Basis<S, T>::store(V + (size_t)j * ldv + r, vj);
          }
        } else {
          y = T(0);
        }
      }
      ys[i * SELL_C + lane] = y;
      if (SCALED) vs[i * SELL_C + lane] = vj;
    }
    __syncthreads();
    const int base = g * STAGE;
    const int nrows = A.n - base < STAGE ? A.n - base : STAGE;
    project_rows<T, S, SLOTS, SCALED, NW>(V, ldv, j, C, base, nrows, ys, vs, acc, lane, wid);
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) {
    const int c = wid + NW * q;
    if (c < C) {
      const T v = wave_sum(acc[q]);
      if (lane == 0) s_vals[c] = v;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += NW * WAVE) part[(size_t)c * MAX_BLOCKS + blockIdx.x] = s_vals[c];
}

// h[c0 + c] = V[:, c0 + c]^T w for c < nc <= 64 (restart lengths beyond the
// fused kernels' register budget).
template <typename T, typename S>
__global__ __launch_bounds__(BLOCK) void k_dots(int n, const S* __restrict__ V, long ldv, int c0, int nc,
                                                const T* __restrict__ w, State st, int check_done,
                                                T* __restrict__ part) {
  if (check_done && (st.hdr->flags & F_DONE)) return;
  __shared__ T s_red[NWAVES * 64];
  __shared__ T s_vals[65];
  int r0, r1;
  block_rows(n, r0, r1);
  T acc[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) acc[c] = T(0);
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) {
    const T wv = w[r];
    const uint32_t roff = (uint32_t)r * (uint32_t)sizeof(S);
#pragma unroll
    for (int cb = 0; cb < 64; cb += 32) {
#pragma unroll
      for (int c = cb; c < cb + 32; ++c)
        if (c < nc) acc[c] += vload<S, T>(V, ldv, c0 + c, roff) * wv;
      asm volatile("" ::: "memory");
    }
  }
  block_reduce_vec(acc, nc, s_red, s_vals);
  store_partials(s_vals, nc, part);
}

// ---------------------------------------------------------------------------
// second kernel: first-pass update + second-pass projection
// ---------------------------------------------------------------------------

// R consecutive rows of one column (R = 4, 2, 1; the first row a multiple of R).
template <typename S, typename T, int R>
struct Rows;
template <typename S, typename T>
struct Rows<S, T, 4> {
  static __device__ __forceinline__ void load(const S* p, T (&v)[4]) { Quad<S, T>::load(p, v); }
};
template <typename S, typename T>
struct Rows<S, T, 2> {
  static __device__ __forceinline__ void load(const S* p, T (&v)[2]) { Pair<S, T>::load(p, v); }
};
template <typename S, typename T>
struct Rows<S, T, 1> {
  static __device__ __forceinline__ void load(const S* p, T (&v)[1]) { v[0] = Basis<S, T>::load(p); }
};
template <typename T, int R>
__device__ __forceinline__ void store_rows(T* p, const T (&v)[R]) {
  if constexpr (R == 4) QuadStore<T>::store(p, v);
  else if constexpr (R == 2) Pair<T, T>::store(p, v);
  else p[0] = v[0];
}

// R consecutive rows of a work vector (T) with 16-byte accesses.
template <typename T, int R>
__device__ __forceinline__ void load_vec(const T* p, T (&v)[R]) {
  if constexpr (R == 8) {
    const float4 a = *(const float4*)p, b = *(const float4*)(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    Rows<T, T, R>::load(p, v);
  }
}
template <typename T, int R>
__device__ __forceinline__ void store_vec(T* p, const T (&v)[R]) {
  if constexpr (R == 8) {
    *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
    *(float4*)(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
  } else {
    store_rows<T, R>(p, v);
  }
}

// The steps of k_update_proj with the basis loads of step s + 1 issued
// before the barrier of step s (two register sets used in turn), so they are
// in flight while the block waits and finishes step s.  Every load is
// unconditional, so the compiler's waits stay exact: lanes past the block's
// rows and columns past k read a stand-in row of column 0 (h is zero past k,
// rows past the range are masked where used, and no partial past k is kept);
// w of a step is loaded before the next step's basis, so waiting for it
// leaves those loads outstanding; the steps run in pairs (an odd count gets
// one step with every row masked), so the loop has no conditional step.
// Used for a bf16 basis (27-point 128^3: 35.5 -> 24.0 us per launch, 3.3 ->
// 5.0 TB/s; 150^3 108.5 -> 73.9 us), with 4 rows (8 bytes) per lane so the
// widest column classes keep both register sets without spills; fp32
// measured the same either way, and fp64 would lose occupancy to the second
// register set.
template <typename T, typename S, int SLOTS, int R, int WV>
__device__ __forceinline__ void update_proj_pipelined(int r0, int r1, const T* __restrict__ w_in, T* __restrict__ w_out,
                                                      const S* __restrict__ V, long ldv, int k, const T (&hq)[SLOTS],
                                                      T (&acc)[SLOTS], T (*s_part)[WV][WAVE * R], int lane, int wid) {
  constexpr int STEP = WAVE * R;
  using P = Packed<S, T, R>;
  using VR = typename P::type[SLOTS];
  // stand-in row, 64-aligned: below n whenever the range is not empty (only
  // then are w and the steps touched); an empty range (r0 = n) makes just the
  // first basis load below, which stays inside V's m + 1 >= 2 columns
  const int rz = r0 & ~63;
  auto load_step = [&](int base, VR& dst) {
    const int r = base + R * lane;
    const bool rows_ok = r1 - r > 0;
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
      const int c = wid + WV * q;
      dst[q] = P::load(c < k && rows_ok ? V + (size_t)c * ldv + r : V + rz);
    }
  };
  auto step = [&](int base, int buf, VR& vr, VR& vn) {
    const int r = base + R * lane;
    const int nv = r1 - r;
    T wv[R];
    load_vec<T, R>(w_in + (nv > 0 ? r : rz), wv);
    T sp[R];
#pragma unroll
    for (int i = 0; i < R; ++i) sp[i] = T(0);
#pragma unroll
    for (int q = 0; q < SLOTS; ++q)
#pragma unroll
      for (int i = 0; i < R; ++i) sp[i] += hq[q] * ((i < nv) ? P::get(vr[q], i) : T(0));
#pragma unroll
    for (int i = 0; i < R; ++i) s_part[buf][wid][R * lane + i] = sp[i];
    load_step(base + STEP, vn);  // past r1 every lane reads the stand-in row (unused)
    // an LDS-only barrier: the basis loads just issued stay in flight
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) P::hold(vr[q]);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = R * lane + i;
      T t = (s_part[buf][0][e] + s_part[buf][1][e]) + (s_part[buf][2][e] + s_part[buf][3][e]);
      if constexpr (WV == 8) t += (s_part[buf][4][e] + s_part[buf][5][e]) + (s_part[buf][6][e] + s_part[buf][7][e]);
      wv[i] = zero_unless(wv[i] - t, i < nv);
    }
    if (wid == 0 && nv > 0) {
      if (nv >= R) {
        store_vec<T, R>(w_out + r, wv);
      } else {
#pragma unroll
        for (int i = 0; i < R; ++i)
          if (i < nv) w_out[r + i] = wv[i];
      }
    }
#pragma unroll
    for (int q = 0; q < SLOTS; ++q)
#pragma unroll
      for (int i = 0; i < R; ++i) acc[q] += ((i < nv) ? P::get(vr[q], i) : T(0)) * wv[i];
  };
  VR va, vb;
  const int npairs = (r1 - r0 + 2 * STEP - 1) / (2 * STEP);
  load_step(r0, va);
  for (int p = 0; p < npairs; ++p) {
    step(r0 + 2 * p * STEP, 0, va, vb);
    step(r0 + (2 * p + 1) * STEP, 1, vb, va);
  }
}

// The block's WV waves (4 or 8) share rows and split the columns: wave w
// holds columns c = w + WV q (q < SLOTS) of R rows per lane in registers.
// Per step of 64 R rows: each wave forms its part of (V h1)[r] over its
// columns, the parts meet in LDS and are added in a fixed order, every wave
// computes w' = w - V h1 for the step's rows, and then accumulates
// V[r, c] w'[r] for its own columns from the registers.  So each V element is
// loaded once and each lane keeps only SLOTS accumulators.  (Eight waves for
// the widest bases keep SLOTS, and so the registers per lane, at 16.)
// Workspace vectors and basis columns are padded to ldv rows, so whole R-row
// loads stay in bounds; the padded rows are masked to zero.
template <typename T, typename S, int SLOTS, int R, int WV>
__global__ __launch_bounds__(WV * WAVE) void k_update_proj(int n, const T* __restrict__ w_in, T* __restrict__ w_out,
                                                           const S* __restrict__ V, long ldv, int k, State st,
                                                           T* __restrict__ part) {
  const int flags = load_flags(st.hdr);  // tested after h1 is staged (one round trip for both)
  constexpr int KMAX = WV * SLOTS;
  constexpr int STEP = WAVE * R;
  __shared__ T s_h[KMAX];
  __shared__ T s_part[2][WV][STEP];
  __shared__ T s_vals[KMAX];
  const double* h1 = st.h1_of(k - 1);
  for (int c = threadIdx.x; c < KMAX; c += WV * WAVE) s_h[c] = c < k ? (T)h1[c] : T(0);
  __syncthreads();
  if (flags & F_DONE) return;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);  // wave-uniform: hq in scalar registers
  T hq[SLOTS], acc[SLOTS];
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) {
    hq[q] = s_h[wid + WV * q];
    acc[q] = T(0);
  }
  int r0, r1;
  block_rows(n, r0, r1);
  if constexpr (sizeof(S) == 2) {
    update_proj_pipelined<T, S, SLOTS, R, WV>(r0, r1, w_in, w_out, V, ldv, k, hq, acc, s_part, lane, wid);
  } else {
    int buf = 0;
    for (int base = r0; base < r1; base += STEP, buf ^= 1) {
      const int r = base + R * lane;
      const int nv = r1 - r;  // rows of this lane inside the block's range (may be <= 0 or > R)
      using P = Packed<S, T, R>;
      typename P::type vr[SLOTS];
      T s[R];
      // narrow bases: w's load goes out with V's, before the barrier (with few
      // columns the step is otherwise two dependent memory round trips); wide
      // ones load it after the barrier to keep registers for V.  Lanes past
      // the block's rows load the step's first row (below n, and loaded by
      // lane 0 for the same column) instead of branching: a load under a
      // per-lane branch is waited for where the branch ends, which split a
      // step's basis loads into two round trips; only the wave-uniform column
      // test stays a branch (rows past the range are masked where used, w' by
      // a bit mask).  27-point 128^3: 42.2 -> 39.8 us per launch.
      constexpr bool W_EARLY = SLOTS <= 4;
      T wv[R];
      if constexpr (W_EARLY) load_vec<T, R>(w_in + (nv > 0 ? r : base), wv);
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) {
        const int c = wid + WV * q;
        vr[q] = c < k ? P::load(V + (size_t)c * ldv + (nv > 0 ? r : base)) : P::zero();
      }
#pragma unroll
      for (int i = 0; i < R; ++i) s[i] = T(0);
#pragma unroll
      for (int q = 0; q < SLOTS; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) s[i] += hq[q] * ((i < nv) ? P::get(vr[q], i) : T(0));
#pragma unroll
      for (int i = 0; i < R; ++i) s_part[buf][wid][R * lane + i] = s[i];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < SLOTS; ++q) P::hold(vr[q]);
      if constexpr (!W_EARLY) load_vec<T, R>(w_in + (nv > 0 ? r : base), wv);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int e = R * lane + i;
        T t = (s_part[buf][0][e] + s_part[buf][1][e]) + (s_part[buf][2][e] + s_part[buf][3][e]);
        if constexpr (WV == 8) t += (s_part[buf][4][e] + s_part[buf][5][e]) + (s_part[buf][6][e] + s_part[buf][7][e]);
        wv[i] = zero_unless(wv[i] - t, i < nv);
      }
      if (wid == 0 && nv > 0) {
        if (nv >= R) {
          store_vec<T, R>(w_out + r, wv);
        } else {
          for (int i = 0; i < nv; ++i) w_out[r + i] = wv[i];
        }
      }
#pragma unroll
      for (int q = 0; q < SLOTS; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) acc[q] += ((i < nv) ? P::get(vr[q], i) : T(0)) * wv[i];
    }
  }
#pragma unroll
  for (int q = 0; q < SLOTS; ++q) {
    const int c = wid + WV * q;
    if (c < k) {
      const T v = wave_sum(acc[q]);
      if (lane == 0) s_vals[c] = v;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += WV * WAVE) part[(size_t)c * MAX_BLOCKS + blockIdx.x] = s_vals[c];
}

// w_out = w_in - V h (any k <= MAX_RESTART+1); h from h_src.
template <typename T, typename S>
__global__ __launch_bounds__(BLOCK) void k_update(int n, const T* __restrict__ w_in, T* __restrict__ w_out,
                                                  const S* __restrict__ V, long ldv, int k, const double* h_src,
                                                  State st) {
  if (st.hdr->flags & F_DONE) return;
  __shared__ T s_h[MAX_RESTART + 1];
  for (int c = threadIdx.x; c < k; c += BLOCK) s_h[c] = (T)h_src[c];
  __syncthreads();
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) {
    T wv = w_in[r];
    const uint32_t roff = (uint32_t)r * (uint32_t)sizeof(S);
#pragma unroll 8
    for (int c = 0; c < k; ++c) wv -= s_h[c] * vload<S, T>(V, ldv, c, roff);
    w_out[r] = wv;
  }
}

// ---------------------------------------------------------------------------
// third kernel: second-pass update + norm; the Givens step
// ---------------------------------------------------------------------------

// The least-squares update of Algorithm 1 done incrementally with Givens
// rotations, by one block of any size (the extra block of
// k_reduce_h1_givens, or k_norm_givens after a cycle's last step).  The
// column and the earlier rotations are staged in LDS so the sequential part
// (thread 0) touches no global memory.  Returns the flags it set (the same
// value in every thread).
template <typename T>
__device__ __forceinline__ int givens_tail(const State& st, int j, int kmax, T nrm2, T* s_col, T* s_cs, T* s_sn) {
  __shared__ T s_sq[16];
  __shared__ int s_flags;
  __shared__ T s_g[2];
  StateHdr* hd = st.hdr;
  const int ld = st.ld;
  const double* h1 = st.h1_of(j);
  double* Hc = st.Hbar + (size_t)j * ld;
  double* Rc = st.R + (size_t)j * ld;
  // read before the stores below, which the compiler cannot tell apart from
  // these fields (written only at a cycle's set-up)
  const double gin_d = hd->gamma_in, stop_abs = hd->stop_abs;
  T sq = T(0);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    const T v = (T)h1[i] + (T)st.h2[i];
    Hc[i] = (double)v;
    s_col[i] = v;
    sq += v * v;
  }
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    s_cs[i] = (T)st.cs[i];
    s_sn[i] = (T)st.sn[i];
  }
  if (threadIdx.x == 0) s_g[0] = (T)st.g[j];
  sq = block_sum_any(sq, s_sq);  // ends with a barrier
  if (threadIdx.x == 0) {
    const T hn = sqrt(nrm2);
    Hc[j + 1] = (double)hn;
    const T colnorm = sqrt(sq + hn * hn);
    int flags;
    if (!isfinite(hn) || !isfinite(colnorm)) {
      flags = F_DONE | F_NUMERIC;
      hd->k = j;
    } else {
      T cur = s_col[0];
      // unrolled so the LDS reads of several rotations are in flight at once
#pragma unroll 8
      for (int i = 0; i < j; ++i) {
        T nxt = s_col[i + 1];
        const T c = s_cs[i], s = s_sn[i];
        s_col[i] = c * cur + s * nxt;
        cur = -s * cur + c * nxt;
      }
      const T rho = hypot(cur, hn);
      T c, s;
      if (rho == T(0)) {
        c = T(1);
        s = T(0);
      } else {
        c = cur / rho;
        s = hn / rho;
      }
      s_col[j] = rho;
      s_col[j + 1] = T(0);
      st.cs[j] = (double)c;
      st.sn[j] = (double)s;
      const T gj = s_g[0];
      const T gj1 = -s * gj;
      st.g[j] = (double)(c * gj);
      st.g[j + 1] = (double)gj1;
      const T gin = (T)gin_d;
      st.hist[j] = (double)(fabs(gj1) / gin);
      hd->k = j + 1;
      hd->implicit = (double)fabs(gj1);
      hd->inv_h = (double)(T(1) / hn);
      const bool breakdown = hn <= (T)(100.0 * Unit<T>::roundoff) * colnorm;
      const bool stopped = stop_abs >= 0.0 && fabs(gj1) <= (T)stop_abs;
      flags = (breakdown ? F_BREAKDOWN : 0) | (stopped ? F_STOPPED : 0);
      if (breakdown || stopped || j + 1 >= kmax) flags |= F_DONE;
    }
    s_flags = flags;
    hd->flags = flags;
  }
  __syncthreads();
  if (!(s_flags & F_NUMERIC))
    for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) Rc[i] = (double)s_col[i];
  // keep both matrices clean below row j+1 (the workspace is not zeroed)
  for (int i = j + 2 + threadIdx.x; i < ld; i += blockDim.x) {
    Hc[i] = 0.0;
    Rc[i] = 0.0;
  }
  return s_flags;
}

// Each lane owns four consecutive rows (16-byte loads for fp32); the padded
// rows past n are masked out.  NT threads per block: 512 (eight waves), since
// the grid is capped at MAX_BLOCKS blocks by the partial-sum slots and four
// waves per block then leave half of each CU's wave slots empty.
template <typename T, typename S, int NT>
__global__ __launch_bounds__(NT) void k_update_norm(int n, const T* __restrict__ w_in, T* __restrict__ wtmp,
                                                    const S* __restrict__ V, long ldv, int j, State st,
                                                    T* __restrict__ part) {
  const int flags = load_flags(st.hdr);  // tested after h2 is staged (one round trip for both)
  __shared__ T s_h[MAX_RESTART + 2];
  __shared__ T s_vals[1];
  __shared__ T s_scr[16];
  const int k = j + 1;
  for (int c = threadIdx.x; c < k; c += NT) s_h[c] = (T)st.h2[c];
  __syncthreads();
  if (flags & F_DONE) return;
  int r0, r1;
  block_rows(n, r0, r1);
  T nrm = T(0);
  for (int r = r0 + 4 * threadIdx.x; r < r1; r += 4 * NT) {
    const int nv = r1 - r < 4 ? r1 - r : 4;
    T wv[4];
    Quad<T, T>::load(w_in + r, wv);
    // 16 columns' loads per unrolled step: 27-point 128^3 36.8 -> 33.8 us per
    // launch, 150^3 126.6 -> 118.3 us (unrolling by 8 measured slower than 4)
#pragma unroll 16
    for (int c = 0; c < k; ++c) {
      T v[4];
      Quad<S, T>::load(V + (size_t)c * ldv + r, v);
      const T h = s_h[c];
#pragma unroll
      for (int i = 0; i < 4; ++i) wv[i] -= h * v[i];
    }
    if (nv == 4) {
      QuadStore<T>::store(wtmp + r, wv);
#pragma unroll
      for (int i = 0; i < 4; ++i) nrm += wv[i] * wv[i];
    } else {
      for (int i = 0; i < nv; ++i) {
        wtmp[r + i] = wv[i];
        nrm += wv[i] * wv[i];
      }
    }
  }
  const T bs = block_sum_any(nrm, s_scr);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// ---------------------------------------------------------------------------
// one-block tail kernels of the cross-block reductions
// ---------------------------------------------------------------------------

// h[c] = sum of the partials of column c < nv.  Grid ceil(nv / 4): wave w
// of block b sums column 4 b + w, so the partials are read by many CUs at
// once (one CU alone is latency bound on them).  It does not test the stop
// flag: after a cycle has stopped, the h it writes is read by nothing before
// the next cycle writes it again, and a flag test would put one more memory
// round trip in front of the reduction.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_reduce_cols(const T* __restrict__ part, int nv, int B, double* h) {
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int c = blockIdx.x * NWAVES + wid;
  if (c >= nv) return;
  const T v = wave_reduce_column(part + (size_t)c * MAX_BLOCKS, B);
  if ((threadIdx.x & (WAVE - 1)) == 0) h[c] = (double)v;
}

// Blocks 0 .. ceil(nv/4)-1: h1 of iteration jg + 1 from the partials of
// k_spmv_proj, as k_reduce_cols.  For jg >= 0 one more block makes the Givens
// step of iteration jg from the ||w''||^2 partials of its k_update_norm (it
// reads the other h1 buffer, so both run at once).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_reduce_h1_givens(const T* __restrict__ part, int nv, int B,
                                                            const T* __restrict__ norm_part, int nB, State st, int jg,
                                                            int kmax) {
  const int ncb = (nv + NWAVES - 1) / NWAVES;
  if ((int)blockIdx.x < ncb) {
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int c = blockIdx.x * NWAVES + wid;
    if (c >= nv) return;
    // no flag test here, as in k_reduce_cols
    const T v = wave_reduce_column(part + (size_t)c * MAX_BLOCKS, B);
    if ((threadIdx.x & (WAVE - 1)) == 0) st.h1_of(jg + 1)[c] = (double)v;
    return;
  }
  __shared__ T s_n[1];
  __shared__ T s_col[MAX_RESTART + 2];
  __shared__ T s_cs[MAX_RESTART];
  __shared__ T s_sn[MAX_RESTART];
  const int flags = load_flags(st.hdr);  // tested after the partials are in
  reduce_partials(norm_part, 1, nB, s_n);
  if (flags & F_DONE) return;
  givens_tail<T>(st, jg, kmax, s_n[0], s_col, s_cs, s_sn);
}

// ||w''||^2 from the partials of k_update_norm, then the Givens update (the
// last iteration of a cycle).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_norm_givens(const T* __restrict__ part, int B, State st, int j, int kmax) {
  const int flags = load_flags(st.hdr);  // tested after the partials are in, as above
  __shared__ T s_col[MAX_RESTART + 2];
  __shared__ T s_cs[MAX_RESTART];
  __shared__ T s_sn[MAX_RESTART];
  __shared__ T s_out[1];
  reduce_partials(part, 1, B, s_out);
  if (flags & F_DONE) return;
  givens_tail<T>(st, j, kmax, s_out[0], s_col, s_cs, s_sn);
}

// *dst = sqrt(sum of the partials) (fp64 norms of b and r).
__global__ __launch_bounds__(BLOCK) void k_sqrt_tail(const double* __restrict__ part, int B, double* dst) {
  __shared__ double s_out[1];
  reduce_partials(part, 1, B, s_out);
  if (threadIdx.x == 0) *dst = sqrt(s_out[0]);
}

// ---------------------------------------------------------------------------
// cycle end: back substitution R y = g (one block)
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_backsolve(State st) {
  unsigned char* s_dyn = dyn_lds<unsigned char>();
  const int flags = st.hdr->flags;
  const int k = st.hdr->k;
  if (threadIdx.x == 0) {
    st.hdr->cycle_k = k;
    st.hdr->cycle_flags = flags;
  }
  if (flags & F_NUMERIC) return;
  if (k <= 0) return;
  T* s_g = (T*)s_dyn;                 // k
  T* s_R = s_g + ((k + 1) & ~1);      // packed columns of the upper triangle (if it fits)
  const int ld = st.ld;
  const bool in_lds = (size_t)k * (k + 1) / 2 * sizeof(T) <= 40960;
  for (int i = threadIdx.x; i < k; i += BLOCK) s_g[i] = (T)st.g[i];
  if (in_lds) {
    // the k columns as one flat range, four loads per thread in flight
    // (column by column the loads would wait for each other)
    const int tot = k * ld;
    for (int i0 = 0; i0 < tot; i0 += 4 * BLOCK) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int id = i0 + threadIdx.x + u * BLOCK;
        v[u] = id < tot ? st.R[id] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int id = i0 + threadIdx.x + u * BLOCK;
        const int c = id / ld, i = id - c * ld;
        if (id < tot && i <= c) s_R[(size_t)c * (c + 1) / 2 + i] = (T)v[u];
      }
    }
  }
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const T rii = in_lds ? s_R[(size_t)i * (i + 1) / 2 + i] : (T)st.R[(size_t)i * ld + i];
    const T yi = s_g[i] / rii;
    __syncthreads();
    for (int l = threadIdx.x; l < i; l += BLOCK) {
      const T ril = in_lds ? s_R[(size_t)i * (i + 1) / 2 + l] : (T)st.R[(size_t)i * ld + l];
      s_g[l] -= ril * yi;
    }
    if (threadIdx.x == 0) st.y[i] = (double)yi;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// outer (fp64) refinement kernels
// ---------------------------------------------------------------------------

// Reset the state header without hipMemsetAsync (safe inside captured graphs).
__global__ void k_init_state(State st, double rtol, int check_mode, double gamma0) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    StateHdr* hd = st.hdr;
    hd->beta = 0.0;
    hd->gamma = gamma0;
    hd->gamma_in = 0.0;
    hd->inv_h = 0.0;
    hd->stop_abs = -1.0;
    hd->rtol = rtol;
    hd->implicit = 0.0;
    hd->lsrho = 0.0;
    hd->check_mode = check_mode;
    hd->k = 0;
    hd->flags = 0;
    hd->cycle_k = 0;
    hd->cycle_flags = 0;
    for (int i = 0; i < 8; ++i) hd->spare[i] = 0u;
  }
}

// *dst = ||v||_2 in fp64 (dst is a field of the state header).
__global__ __launch_bounds__(BLOCK) void k_norm64(int n, const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double s_vals[1], s_scr[NWAVES * WAVE];
  int r0, r1;
  block_rows(n, r0, r1);
  double s = 0.0;
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) s += v[r] * v[r];
  const double bs = block_sum(s, s_scr);
  if (threadIdx.x == 0) s_vals[0] = bs;
  __syncthreads();
  store_partials(s_vals, 1, part);
}

struct ResidEpi {
  const double* b;
  double* r;
  double nrm;
  __device__ __forceinline__ void operator()(int i, double y) {
    const double v = b[i] - y;
    r[i] = v;
    nrm += v * v;
  }
};

// r = b - A x (fp64 matrix and vectors), gamma = ||r||_2 (Algorithm 2, first and last lines).
__global__ __launch_bounds__(BLOCK) void k_resid64(Csr A, const double* __restrict__ x, const double* __restrict__ b,
                                                   double* __restrict__ r, double* __restrict__ part) {
  double* prod = dyn_lds<double>();  // one entry per nonzero of the largest tile
  __shared__ double s_vals[1], s_scr[NWAVES * WAVE];
  ResidEpi epi{b, r, 0.0};
  if (A.sell) sell_rows<double>(A, XPlain<double>{x}, epi);
  else spmv_tiles<double>(A, XPlain<double>{x}, epi, prod, s_scr);
  const double bs = block_sum(epi.nrm, s_scr);
  if (threadIdx.x == 0) s_vals[0] = bs;
  __syncthreads();
  store_partials(s_vals, 1, part);
}

// Start of a cycle after the tail of a reduction gave gin = ||rhat||: reset
// the cycle state and the early-exit threshold rtol ||b|| / ||r||.
template <typename T>
__device__ __forceinline__ void cycle_start_tail(const State& st, T gin) {
  StateHdr* hd = st.hdr;
  hd->gamma_in = (double)gin;
  hd->inv_h = (double)(T(1) / gin);
  st.g[0] = (double)gin;
  hd->k = 0;
  hd->implicit = (double)gin;
  hd->flags = (isfinite(gin) && gin > T(0)) ? 0 : (F_DONE | F_NUMERIC);
  hd->stop_abs = hd->check_mode == 1 ? (double)(T)(hd->rtol * hd->beta / hd->gamma) : -1.0;
}

// gin = sqrt(sum of the partials): start of a cycle.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cycle_tail(const T* __restrict__ part, int B, State st) {
  __shared__ T s_out[1];
  reduce_partials(part, 1, B, s_out);
  if (threadIdx.x == 0) cycle_start_tail<T>(st, (T)sqrt(s_out[0]));
}

// wtmp = round_T(r / gamma) (the inner right-hand side, Algorithm 2 line 3),
// optionally also kept in rhat; gin = ||wtmp|| in inner precision.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cast(int n, const double* __restrict__ r, T* __restrict__ wtmp,
                                                T* __restrict__ rhat, State st, T* __restrict__ part) {
  __shared__ T s_vals[1], s_scr[NWAVES * WAVE];
  const double gamma = st.hdr->gamma;
  int r0, r1;
  block_rows(n, r0, r1);
  T s = T(0);
  for (int i = r0 + threadIdx.x; i < r1; i += BLOCK) {
    const T v = (T)(r[i] / gamma);
    wtmp[i] = v;
    if (rhat) rhat[i] = v;
    s += v * v;
  }
  const T bs = block_sum(s, s_scr);
  if (threadIdx.x == 0) s_vals[0] = bs;
  __syncthreads();
  store_partials(s_vals, 1, part);
}

template <typename T>
struct InnerResidEpi {
  const T* rhat;
  T* wtmp;
  T nrm;
  __device__ __forceinline__ void operator()(int i, T y) {
    const T v = rhat[i] - y;
    wtmp[i] = v;
    nrm += v * v;
  }
};

// Restart of the inner solve in its own precision: wtmp = rhat - A_in u.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_inner_resid(Csr A, const T* __restrict__ u, const T* __restrict__ rhat,
                                                       T* __restrict__ wtmp, T* __restrict__ part) {
  T* prod = dyn_lds<T>();  // one entry per nonzero of the largest tile
  __shared__ T s_vals[1], s_scr[NWAVES * WAVE];
  InnerResidEpi<T> epi{rhat, wtmp, T(0)};
  if (A.sell) sell_rows<T>(A, XPlain<T>{u}, epi);
  else spmv_tiles<T>(A, XPlain<T>{u}, epi, prod, s_scr);
  const T bs = block_sum(epi.nrm, s_scr);
  if (threadIdx.x == 0) s_vals[0] = bs;
  __syncthreads();
  store_partials(s_vals, 1, part);
}

// x += gamma * (V_k y) with V_k y accumulated in inner precision (Algorithm 2,
// line 4).  Four rows per lane; x (the caller's vector) is accessed per element.
template <typename T, typename S>
__global__ __launch_bounds__(BLOCK) void k_correct_x(int n, const S* __restrict__ V, long ldv, State st,
                                                     double* __restrict__ x) {
  __shared__ T s_y[MAX_RESTART];
  if (st.hdr->flags & F_NUMERIC) return;
  const int k = st.hdr->k;
  const double gamma = st.hdr->gamma;
  for (int c = threadIdx.x; c < k; c += BLOCK) s_y[c] = (T)st.y[c];
  __syncthreads();
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + 4 * threadIdx.x; r < r1; r += 4 * BLOCK) {
    const int nv = r1 - r < 4 ? r1 - r : 4;
    T u[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll 4
    for (int c = 0; c < k; ++c) {
      T v[4];
      Quad<S, T>::load(V + (size_t)c * ldv + r, v);
      const T yc = s_y[c];
#pragma unroll
      for (int i = 0; i < 4; ++i) u[i] += v[i] * yc;
    }
    for (int i = 0; i < nv; ++i) x[r + i] = x[r + i] + gamma * (double)u[i];
  }
}

// z = V_k y in inner precision (z is a workspace vector padded to ldv).
template <typename T, typename S>
__global__ __launch_bounds__(BLOCK) void k_vy(int n, const S* __restrict__ V, long ldv, State st, T* __restrict__ z) {
  __shared__ T s_y[MAX_RESTART];
  const int k = (st.hdr->flags & F_NUMERIC) ? 0 : st.hdr->k;
  for (int c = threadIdx.x; c < k; c += BLOCK) s_y[c] = (T)st.y[c];
  __syncthreads();
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + 4 * threadIdx.x; r < r1; r += 4 * BLOCK) {
    const int nv = r1 - r < 4 ? r1 - r : 4;
    T u[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll 4
    for (int c = 0; c < k; ++c) {
      T v[4];
      Quad<S, T>::load(V + (size_t)c * ldv + r, v);
      const T yc = s_y[c];
#pragma unroll
      for (int i = 0; i < 4; ++i) u[i] += v[i] * yc;
    }
    for (int i = 0; i < nv; ++i) z[r + i] = u[i];
  }
}

// u = z (first) or u += z, inner precision.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_accum(int n, const T* __restrict__ z, T* __restrict__ u, int first) {
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) u[r] = first ? z[r] : u[r] + z[r];
}

// x += gamma * u (fp64 update).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_axpy_x(int n, const T* __restrict__ u, State st, double* __restrict__ x) {
  const double gamma = st.hdr->gamma;
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) x[r] = x[r] + gamma * (double)u[r];
}

// fp64 inner solve with an fp32 polynomial preconditioner (an fp32 M applied
// to fp64 vectors: cast in, multiply in fp32, cast back).  Step one of an
// iteration: v_j = wtmp / ||wtmp|| is stored as basis column j (fp64) and
// rounded to fp32 as the polynomial's input.
template <typename T, typename S>
__global__ __launch_bounds__(BLOCK) void k_scale_narrow(int n, const T* __restrict__ wtmp, S* __restrict__ V, long ldv,
                                                        int j, float* __restrict__ v32, State st,
                                                        const T* __restrict__ norm_part, int nB) {
  const int flags = load_flags(st.hdr);
  const T inv = prev_inv_norm<T>(st, norm_part, nB);
  if (flags & F_DONE) return;
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) {
    const T v = Basis<S, T>::round(wtmp[r] * inv);
    Basis<S, T>::store(V + (size_t)j * ldv + r, v);
    v32[r] = (float)v;
  }
}

// y = fp32(x) (round to nearest even); check_done: no-op once the cycle stopped.
__global__ __launch_bounds__(BLOCK) void k_narrow(int n, const double* __restrict__ x, float* __restrict__ y, State st,
                                                  int check_done) {
  if (check_done && (load_flags(st.hdr) & F_DONE)) return;
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) y[r] = (float)x[r];
}

// y = fp64(x) (exact); check_done as above.
__global__ __launch_bounds__(BLOCK) void k_widen(int n, const float* __restrict__ x, double* __restrict__ y, State st,
                                                 int check_done) {
  if (check_done && (load_flags(st.hdr) & F_DONE)) return;
  int r0, r1;
  block_rows(n, r0, r1);
  for (int r = r0 + threadIdx.x; r < r1; r += BLOCK) y[r] = (double)x[r];
}

// ---------------------------------------------------------------------------
// block Jacobi preconditioner: M = blockdiag(A_11, A_22, ...), blocks of
// bs <= 64 consecutive rows/columns (the last one ragged)
// ---------------------------------------------------------------------------

constexpr int BJ_MAX = 64;

// One wave inverts G = 64 / bs consecutive diagonal blocks (lane = g * bs + i:
// row i of block g) in precision C, the precision the preconditioner is
// applied in (Section "Preconditioning": for GMRES-IR the fp32 preconditioner
// is both computed and applied in fp32; the fp64 solve keeps it in fp64).
// Each block is gathered from the CSR arrays of the matrix copy in C (for
// fp32 the round-to-nearest-even copy) into LDS next to an identity (C =
// double: 66 KB of LDS, gfx950 gives a workgroup up to 160 KB), reduced by
// Gauss-Jordan elimination with partial pivoting in C, and its inverse
// written by wave group and column: Minv[grp][c][lane] = inv(A_bb)[i][c]
// (grp = this block's index, lane = g * bs + i < W = G * bs, column stride
// W), so that for each column the lanes of the applying wave read one
// contiguous row of W entries (columns past a ragged block's size are never
// read).  The bs
// pivot steps run in lock step for all blocks of the wave (a ragged last
// block skips the steps beyond its size).  A zero or non-finite pivot writes
// NaN (the solve then reports NUMERIC).
template <typename C>
__global__ __launch_bounds__(WAVE) void k_bj_invert(int n, const int* __restrict__ rowptr,
                                                    const int* __restrict__ col, const C* __restrict__ vals,
                                                    int bs, C* __restrict__ Minv) {
  __shared__ C a[WAVE][2 * BJ_MAX + 1];
  __shared__ int s_piv[WAVE];
  const int lane = threadIdx.x;
  const int G = WAVE / bs;
  const int g = lane / bs;
  const int i = lane - g * bs;
  const long nblk = ((long)n + bs - 1) / bs;
  const long blk = (long)blockIdx.x * G + g;
  const long r0 = blk * bs;
  const int m = (g < G && blk < nblk) ? (int)((n - r0) < bs ? (n - r0) : bs) : 0;
  const int base = g * bs;  // first LDS row of this lane's block
  for (int c = 0; c < 2 * BJ_MAX; ++c) a[lane][c] = (i < m && c == m + i) ? C(1) : C(0);
  if (i < m) {
    const long r = r0 + i;
    for (int q = rowptr[r]; q < rowptr[r + 1]; ++q) {
      const long c = col[q] - r0;
      if (c >= 0 && c < m) a[lane][c] = vals[q];
    }
  }
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < bs; ++k) {
    const bool act = k < m;
    if (act && i == 0) {
      int p = k;
      C best = fabs(a[base + k][k]);
      for (int q = k + 1; q < m; ++q)
        if (fabs(a[base + q][k]) > best) best = fabs(a[base + q][k]), p = q;
      s_piv[g] = p;
    }
    __syncthreads();
    if (act) {
      const int p = s_piv[g];
      if (p != k) {
        for (int c = i; c < 2 * m; c += bs) {
          const C t = a[base + k][c];
          a[base + k][c] = a[base + p][c];
          a[base + p][c] = t;
        }
      }
    }
    __syncthreads();
    const C piv = act ? a[base + k][k] : C(1);
    if (act) bad = bad || !(fabs(piv) > C(0)) || !isfinite(piv);
    __syncthreads();
    if (act)
      for (int c = i; c < 2 * m; c += bs) a[base + k][c] = a[base + k][c] / piv;
    __syncthreads();
    if (act && i < m && i != k) {
      const C f = a[lane][k];
      for (int c = 0; c < 2 * m; ++c) a[lane][c] -= f * a[base + k][c];
    }
    __syncthreads();
  }
  const C nan = (C)__builtin_nan("");
  if (i < m) {
    const int W = G * bs;
    C* out = Minv + (size_t)blockIdx.x * bs * W + lane;
    for (int c = 0; c < m; ++c) out[(size_t)c * W] = bad ? nan : a[lane][m + c];
  }
}

// y = M^{-1} x.  A wave takes G = 64 / bs consecutive diagonal blocks at
// once (lane = g * bs + i: row i of block g; for bs = 8 all 64 lanes work),
// stages their x in LDS and each lane sums its row of the inverse over the
// block's columns in ascending order; the inverses are stored by wave group
// and column (stride W = G * bs), so each column step is one contiguous load
// of W entries for the wave (stored block by block, bs = 8 took 8 cache lines
// per load: 11.4 us per application on the 1000^2 system; a stride of 64 for
// bs = 42 left 22 of every 64 entries unused, 37.6 -> 52.0 us).
// SCALED: x is the next basis vector v_j = round(wtmp * inv), which is also
// stored as basis column j (the fused start of an iteration, as in the
// polynomial path).  check_done as in the other iteration kernels.
template <typename T, typename S, bool SCALED>
__global__ __launch_bounds__(BLOCK) void k_bj_apply(int n, int bs, const T* __restrict__ Minv,
                                                    const T* __restrict__ src, S* __restrict__ V, long ldv, int j,
                                                    T* __restrict__ y, State st, int check_done,
                                                    const T* __restrict__ norm_part, int nB) {
  __shared__ T s_x[NWAVES][WAVE];
  const int flags = check_done ? load_flags(st.hdr) : 0;
  const T inv = SCALED ? prev_inv_norm<T>(st, norm_part, nB) : T(1);
  if (flags & F_DONE) return;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int G = WAVE / bs;  // blocks per wave, >= 1 for bs <= 64
  const int g = lane / bs;
  const int i = lane - g * bs;
  const long nblk = ((long)n + bs - 1) / bs;
  const long ngrp = (nblk + G - 1) / G;
  for (long grp = (long)blockIdx.x * NWAVES + wid; grp < ngrp; grp += (long)gridDim.x * NWAVES) {
    const long blk = grp * G + g;
    const long r0 = blk * bs;
    const int m = (g < G && blk < nblk) ? (int)((n - r0) < bs ? (n - r0) : bs) : 0;
    T xv = T(0);
    if (i < m) {
      if (SCALED) {
        xv = Basis<S, T>::round(src[r0 + i] * inv);
        Basis<S, T>::store(V + (size_t)j * ldv + r0 + i, xv);
      } else {
        xv = src[r0 + i];
      }
    }
    s_x[wid][lane] = xv;
    __builtin_amdgcn_wave_barrier();
    if (i < m) {
      const int W = G * bs;
      const T* Mg = Minv + (size_t)grp * bs * W + lane;
      const T* xs = &s_x[wid][g * bs];
      T acc = T(0);
      for (int c = 0; c < m; ++c) acc += Mg[(size_t)c * W] * xs[c];
      y[r0 + i] = acc;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ void k_fill64(int n, double* __restrict__ x, double v) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) x[i] = v;
}

// ---------------------------------------------------------------------------
// polynomial preconditioner: one SpMV step of the product form of p(A)
// ---------------------------------------------------------------------------

template <typename T>
struct PolyCoef {
  T ay, aw, ax, at;  // y = ay*y + aw*W + ax*X + at*(A X)
  T bw, bx, bt;      // d = bw*W + bx*X + bt*(A X)
  int has_y, y_read, has_d, has_w;
};

template <typename T, typename S, bool SCALED>
struct PolyEpi {
  const T* src;
  T inv;
  S* V;
  long ldv;
  int j;
  int write_v;
  const T* W;
  int w_scaled;
  T* Y;
  T* D;
  PolyCoef<T> cf;
  __device__ __forceinline__ void operator()(int r, T t) {
    T xr;
    if (SCALED) {
      xr = Basis<S, T>::round(src[r] * inv);
      if (write_v) Basis<S, T>::store(V + (size_t)j * ldv + r, xr);
    } else {
      xr = src[r];
    }
    T wr = T(0);
    if (cf.has_w) wr = w_scaled ? Basis<S, T>::round(W[r] * inv) : W[r];
    if (cf.has_y) {
      T yv = cf.aw * wr + cf.ax * xr + cf.at * t;
      if (cf.y_read) yv += cf.ay * Y[r];
      Y[r] = yv;
    }
    if (cf.has_d) D[r] = cf.bw * wr + cf.bx * xr + cf.bt * t;
  }
};

template <typename T, typename S, bool SCALED>
__global__ __launch_bounds__(BLOCK) void k_poly_step(Csr A, const T* __restrict__ src, S* __restrict__ V, long ldv,
                                                     int j, int write_v, const T* __restrict__ W, int w_scaled,
                                                     T* __restrict__ Y, T* __restrict__ D, PolyCoef<T> cf, State st,
                                                     int check_done, const T* __restrict__ norm_part, int nB) {
  if (check_done && (st.hdr->flags & F_DONE)) return;
  T* prod = dyn_lds<T>();  // one entry per nonzero of the largest tile
  __shared__ T s_scr[NWAVES * WAVE];
  PolyEpi<T, S, SCALED> epi;
  epi.src = src;
  epi.inv = (SCALED || w_scaled) ? prev_inv_norm<T>(st, norm_part, nB) : T(1);
  epi.V = V;
  epi.ldv = ldv;
  epi.j = j;
  epi.write_v = write_v;
  epi.W = W;
  epi.w_scaled = w_scaled;
  epi.Y = Y;
  epi.D = D;
  epi.cf = cf;
  if (SCALED) {
    if (A.sell) sell_rows<T>(A, XScaled<T, S>{src, epi.inv}, epi);
    else spmv_tiles<T>(A, XScaled<T, S>{src, epi.inv}, epi, prod, s_scr);
  } else {
    if (A.sell) sell_rows<T>(A, XPlain<T>{src}, epi);
    else spmv_tiles<T>(A, XPlain<T>{src}, epi, prod, s_scr);
  }
}

// ---------------------------------------------------------------------------
// plain SpMV, start vector, casts, row statistics
// ---------------------------------------------------------------------------

template <typename T>
struct PlainEpi {
  T* y;
  __device__ __forceinline__ void operator()(int r, T v) { y[r] = v; }
};

template <typename T, bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_spmv(Csr A, const T* __restrict__ x, T* __restrict__ y) {
  T* prod = dyn_lds<T>();  // one entry per nonzero of the largest tile
  __shared__ T s_scr[NWAVES * WAVE];
  PlainEpi<T> epi{y};
  if (A.sell) sell_rows<T, WIDE>(A, XPlain<T>{x}, epi);
  else spmv_tiles<T>(A, XPlain<T>{x}, epi, prod, s_scr);
}

__global__ void k_cast_vals(int64_t nnz, const double* __restrict__ v64, float* __restrict__ v32) {
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * BLOCK)
    v32[i] = (float)v64[i];
}

// *flag != 0 if some entry lies more than 32767 columns from its row (then
// the sliced copy keeps 32-bit columns).  Grid-stride over the rows.
__global__ void k_col_offset_check(int n, const int* __restrict__ rowptr, const int* __restrict__ colidx, int* flag) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    bool far = false;
    for (int p = rowptr[r]; p < rowptr[r + 1]; ++p) {
      const int d = colidx[p] - r;
      far = far || d > 32767 || d < -32767;
    }
    if (far) atomicOr(flag, 1);
  }
}

// Fill the sliced ELLPACK copy (one block of 64 threads per slice, one row per
// thread); fp32 values rounded to nearest even like the CSR copy.  Columns are
// stored as 32-bit indices, or (d16) as 16-bit offsets from the row, which
// take a quarter of the SpMV's bytes off (6 instead of 8 per fp32 nonzero).
// Padding entries point at the row itself (offset 0), rows past n at row 0.
__global__ void k_build_sell(int n, const int* __restrict__ rowptr, const int* __restrict__ colidx,
                             const double* __restrict__ vals, const int* __restrict__ sptr, int* __restrict__ scol,
                             short* __restrict__ scol16, int d16, float* __restrict__ sv32,
                             double* __restrict__ sv64) {
  const int sl = blockIdx.x, lane = threadIdx.x;
  const int r = sl * SELL_C + lane;
  const int base = sptr[sl];
  const int K = (sptr[sl + 1] - base) / SELL_C;
  const int p0 = r < n ? rowptr[r] : 0;
  const int len = r < n ? rowptr[r + 1] - p0 : 0;
  const int rr = r < n ? r : 0;
  for (int k = 0; k < K; ++k) {
    const int e = base + SELL_C * k + lane;
    int c = rr;
    double v = 0.0;
    if (k < len) {
      c = colidx[p0 + k];
      v = vals[p0 + k];
    }
    if (d16) scol16[e] = (short)(c - rr);
    else scol[e] = c;
    sv64[e] = v;
    sv32[e] = (float)v;
  }
}

// Values of the shared-offset sliced copy (one block of 64 threads per
// slice, one row per thread): slot k of the row takes the CSR entry at column
// r + soff[k] if the row has one, else 0; fp32 values rounded to nearest even
// like the CSR copy.  The host has checked that every row's columns strictly
// increase and lie in its slice's offset list, so one pass with a cursor
// takes every entry.
__global__ void k_build_sell_shared(int n, const int* __restrict__ rowptr, const int* __restrict__ colidx,
                                    const double* __restrict__ vals, const int* __restrict__ sptr,
                                    const int* __restrict__ soff_all, float* __restrict__ sv32,
                                    double* __restrict__ sv64) {
  const int sl = blockIdx.x, lane = threadIdx.x;
  const int r = sl * SELL_C + lane;
  const int base = sptr[sl];
  const int K = (sptr[sl + 1] - base) / SELL_C;
  const int* soff = soff_all + base / SELL_C;
  int p = r < n ? rowptr[r] : 0;
  const int pe = r < n ? rowptr[r + 1] : 0;
  for (int k = 0; k < K; ++k) {
    double v = 0.0;
    if (p < pe && colidx[p] - r == soff[k]) v = vals[p++];
    const int e = base + SELL_C * k + lane;
    sv64[e] = v;
    sv32[e] = (float)v;
  }
}

// v[i] = 2 * (splitmix64(seed ^ i) >> 11) * 2^-53 - 1 (SplitMix64, S. Vigna).
__global__ void k_start_vector(int n, uint64_t seed, double* __restrict__ v) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    uint64_t z = (seed ^ (uint64_t)i) + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    v[i] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
  }
}

// Row statistics of the chooser features, fp64:
// out[0] sum d/(d+S)  out[1] min d/(d+S)  out[2] #rows d >= S  out[3] sum rowsum
// out[4] sum a^2      out[5] sum a_ii     out[6] sum a_ii^2    out[7] sum |U-L|/S
// out[8] max row nnz  out[9] sum |a_ii|
__device__ __forceinline__ double rowstat_combine(int c, double a, double b) {
  return (c == 1) ? fmin(a, b) : (c == 8) ? fmax(a, b) : a + b;
}

__global__ __launch_bounds__(BLOCK) void k_rowstats(Csr A, double* __restrict__ part) {
  __shared__ double s_scr[NWAVES * 10];
  __shared__ double s_vals[10];
  const double* vals = (const double*)A.vals;
  int r0, r1;
  block_rows(A.n, r0, r1);
  double acc[10] = {0, 1e300, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = r0 + threadIdx.x; i < r1; i += BLOCK) {
    double d = 0, ds = 0, S = 0, L = 0, U = 0, rs = 0, a2 = 0;
    const int q0 = A.rowptr[i], q1 = A.rowptr[i + 1];
    for (int q = q0; q < q1; ++q) {
      const int c = A.col[q];
      const double a = vals[q];
      rs += a;
      a2 += a * a;
      if (c == i) {
        d += fabs(a);
        ds += a;
      } else {
        S += fabs(a);
        if (c < i) L += a; else U += a;
      }
    }
    const double tot = d + S;
    const double frac = tot > 0 ? d / tot : 0.0;
    acc[0] += frac;
    acc[1] = fmin(acc[1], frac);
    acc[2] += (d >= S) ? 1.0 : 0.0;
    acc[3] += rs;
    acc[4] += a2;
    acc[5] += ds;
    acc[6] += ds * ds;
    acc[7] += S > 0 ? fabs(U - L) / (S + 1e-30) : 0.0;
    acc[8] = fmax(acc[8], (double)(q1 - q0));
    acc[9] += d;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
  for (int c = 0; c < 10; ++c) {
    double v = acc[c];
    for (int o = 32; o > 0; o >>= 1) v = rowstat_combine(c, v, __shfl_xor(v, o, 64));
    if (lane == 0) s_scr[wid * 10 + c] = v;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    const int c = threadIdx.x;
    double v = s_scr[c];
    for (int w = 1; w < NWAVES; ++w) v = rowstat_combine(c, v, s_scr[w * 10 + c]);
    s_vals[c] = v;
  }
  __syncthreads();
  store_partials(s_vals, 10, part);
}

__global__ __launch_bounds__(BLOCK) void k_rowstats_tail(const double* __restrict__ part, int B,
                                                         double* __restrict__ out) {
  if (threadIdx.x < 10) {
    const int c = threadIdx.x;
    double v = part[(size_t)c * MAX_BLOCKS];
    for (int b = 1; b < B; ++b) v = rowstat_combine(c, v, part[(size_t)c * MAX_BLOCKS + b]);
    out[c] = v;
  }
}

}  // namespace gir
