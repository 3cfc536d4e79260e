// Device-side building blocks of libgmresir for gfx950 (wave64, 256 CUs in
// 8 XCDs): basis storage types, wave/block reductions, the deterministic
// two-kernel grid reduction, and the shared device state of a cycle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace gir {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int NWAVES = BLOCK / WAVE;

typedef uint16_t bf16_t;

// ---------------------------------------------------------------------------
// basis storage: S is the stored element type, T the arithmetic type
// ---------------------------------------------------------------------------

template <typename S, typename T>
struct Basis;

template <>
struct Basis<double, double> {
  static __device__ __forceinline__ double load(const double* p) { return *p; }
  static __device__ __forceinline__ double round(double v) { return v; }
  static __device__ __forceinline__ void store(double* p, double v) { *p = v; }
};

template <>
struct Basis<float, float> {
  static __device__ __forceinline__ float load(const float* p) { return *p; }
  static __device__ __forceinline__ float round(float v) { return v; }
  static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
};

// bfloat16: the top half of the binary32 pattern, rounded to nearest even.
// gfx950 converts in one instruction (v_cvt_pk_bf16_f32); measured on the GPU
// against the bit arithmetic "u + 0x7fff + bit 16 of u, keep the top half;
// NaN keeps its top half with the quiet bit set" over all 2^32 fp32 patterns:
// identical, NaN payloads included.  (In the SpMV's gather every source
// element is rounded, 27 times per row on a 27-point stencil, so the
// instruction count matters there.)
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <>
struct Basis<bf16_t, float> {
  static __device__ __forceinline__ float load(const bf16_t* p) { return bf16_bits_to_f32(*p); }
  static __device__ __forceinline__ float round(float v) { return (float)(__bf16)v; }
  static __device__ __forceinline__ void store(bf16_t* p, float v) { *p = f32_to_bf16_bits(v); }
};

// Load element (row, column c) of a column-major basis: the column base is
// wave-uniform (scalar registers) and the row offset is a 32-bit byte offset
// shared by all columns, so each load costs no per-column vector address.
template <typename S, typename T>
__device__ __forceinline__ T vload(const S* V, long ldv, int c, uint32_t roff) {
  const char* base = (const char*)V + (size_t)c * (size_t)ldv * sizeof(S);
  return Basis<S, T>::load((const S*)(base + roff));
}

template <typename T>
struct Unit;
template <>
struct Unit<float> {
  static constexpr double roundoff = 5.9604644775390625e-08;  // 2^-24
};
template <>
struct Unit<double> {
  static constexpr double roundoff = 1.1102230246251565e-16;  // 2^-53
};

// ---------------------------------------------------------------------------
// device state of one solve (lives in the caller's workspace)
// ---------------------------------------------------------------------------

enum : int32_t { F_DONE = 1, F_BREAKDOWN = 2, F_NUMERIC = 4, F_STOPPED = 8 };

struct StateHdr {
  double beta;      // ||b||_2 (fp64)
  double gamma;     // ||r||_2 of the current outer residual (fp64)
  double gamma_in;  // norm of the current cycle's right-hand side (inner precision)
  double inv_h;     // 1 / norm of the vector held in wtmp: next basis vector = wtmp * inv_h
  double stop_abs;  // implicit early exit when |g_{j+1}| <= stop_abs (< 0: off)
  double rtol;
  double implicit;  // |g_{k}| of the last step (implicit residual, cycle units)
  double lsrho;     // one-reduction CGS2: norm of the vector the next update normalises
  int32_t check_mode;
  int32_t k;            // Arnoldi steps completed in the current cycle
  int32_t flags;        // F_* of the current cycle
  int32_t cycle_k;      // k and flags of the last finished cycle (kept across
  int32_t cycle_flags;  // the reset a new cycle start does)
  int32_t pad[3];
  uint32_t spare[8];
};

// The stop flags, read where the call stands: an atomic (relaxed) read is not
// sunk to its first use, so its round trip overlaps the loads that follow.
__device__ __forceinline__ int load_flags(const StateHdr* h) {
  return __hip_atomic_load(&h->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct State {
  StateHdr* hdr;
  double* h1;    // m+1   first-pass projection coefficients (even iterations j)
  double* h1x;   // m+1   the same for odd j (the Givens step of j-1 reads its h1 while h1 of j is written)
  double* h2;    // m+1   second-pass projection coefficients
  double* Hbar;  // (m+1) x m unrotated Hessenberg matrix, column-major, ld
  double* R;     // (m+1) x m rotated (triangular) columns
  double* cs;    // m     Givens cosines
  double* sn;    // m     Givens sines
  double* g;     // m+1   rotated right-hand side
  double* y;     // m     least-squares solution of the finished cycle
  double* hist;  // m     |g_{j+1}| / gamma_in per step
  double* red;   // one-reduction CGS2: column sums of the iteration's reduction (alpha, gam, a, c)
  double* dco;   // one-reduction CGS2: update coefficients d of the iteration
  int ld;        // m+1
  __host__ __device__ double* h1_of(int j) const { return (j & 1) ? h1x : h1; }
};

// CSR operand of the SpMV kernels; vals has element type MT.
struct Csr {
  int n;
  int ntiles;
  const int* rowptr;
  const int* col;
  const void* vals;
  const int* tile_row;  // ntiles+1 row boundaries
  // sliced ELLPACK copy (sell != 0): slice s holds entries sptr[s] .. sptr[s+1]
  int sell;
  int nslices;
  const int* sptr;
  const int* scol;      // column of each entry (d16 == 0)
  const short* scol16;  // column - row of each entry (d16 != 0; padding 0, rows >= n relative to row 0)
  int d16;
  // shared != 0: one list of column offsets per slice (sorted, at scol +
  // sptr[s] / 64), the same for all its rows; absent entries hold value 0
  int shared;
  const void* svals;  // element type MT, like vals
};

// Dynamic LDS of a kernel (sized at launch: the SpMV product buffer holds the
// largest tile of the matrix, the back substitution its triangle).
template <typename T>
__device__ __forceinline__ T* dyn_lds() {
  extern __shared__ __align__(16) unsigned char gir_dyn_lds[];
  return (T*)gir_dyn_lds;
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Hardware block b runs on XCD (b mod 8); map it to a logical block so that
// each XCD owns a contiguous eighth of the rows (its L2 then holds the x
// neighbourhood the SpMV gathers from).
__device__ __forceinline__ int logical_block() {
  const int b = blockIdx.x, B = gridDim.x;
  return (B % 8 == 0) ? (b % 8) * (B / 8) + b / 8 : b;
}

// Row range [r0, r1) of this block for row-parallel kernels.
__device__ __forceinline__ void block_rows(int n, int& r0, int& r1) {
  const int B = gridDim.x;
  long chunk = ((long)n + B - 1) / B;
  chunk = (chunk + 63) & ~63L;
  long a = (long)logical_block() * chunk;
  r0 = (int)(a < n ? a : n);
  long e = a + chunk;
  r1 = (int)(e < n ? e : n);
}

// Reduce acc[0..nv) over the block (fixed order: butterfly in each wave, then
// waves in order).  Result in out[0..nv) (LDS), visible to all threads.
template <typename T, int NV>
__device__ __forceinline__ void block_reduce_vec(const T (&acc)[NV], int nv, T* lds, T* out) {
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    if (c < nv) {
      T v = wave_sum(acc[c]);
      if (lane == 0) lds[wid * NV + c] = v;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nv; c += BLOCK) {
    T s = lds[c];
#pragma unroll
    for (int w = 1; w < NWAVES; ++w) s += lds[w * NV + c];
    out[c] = s;
  }
  __syncthreads();
}

// Same as block_sum for any block size up to 1024 threads.
template <typename T>
__device__ __forceinline__ T block_sum_any(T v, T* lds /* 16 */) {
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  const int nw = blockDim.x / WAVE;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  T s = lds[0];
  for (int w = 1; w < nw; ++w) s += lds[w];
  __syncthreads();
  return s;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* lds /* NWAVES */) {
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  T s = lds[0];
#pragma unroll
  for (int w = 1; w < NWAVES; ++w) s += lds[w];
  __syncthreads();
  return s;
}

// Cross-block reductions are two kernels: the producer grid stores one
// partial vector per block (column-major, part[c * MAX_BLOCKS + block]) and a
// tail kernel sums them in a fixed order after the kernel boundary has
// published them.  (A "last block" ticket inside the producer would need
// a device-scope release per block, which on gfx950 writes back the whole L2
// of the XCD every time.)
constexpr int MAX_BLOCKS = 1024;
constexpr int RED_BATCH = 4;                   // columns reduced per wave and batch
constexpr int PART_COLS = 136;                 // partial columns in the workspace (>= 129 + 1)
constexpr int NORM_SLOT = PART_COLS - 1;       // column of the ||w''||^2 partials of k_update_norm

template <typename T>
__device__ __forceinline__ void store_partials(const T* vals, int nv, T* part) {
  for (int c = threadIdx.x; c < nv; c += BLOCK) part[(size_t)c * MAX_BLOCKS + blockIdx.x] = vals[c];
}

// Lane l's share of one column of B partials: b = l + 64 i in order of i,
// NL loads all issued before the adds (branch-free: out-of-range blocks read
// a valid address and add 0).
template <int NL, typename T>
__device__ __forceinline__ T lane_share(const T* col, int B) {
  const int lane = threadIdx.x & (WAVE - 1);
  T s = T(0);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int b = lane + WAVE * i;
    const int bc = b < B ? b : B - 1;
    const T v = col[bc];
    s += (b < B) ? v : T(0);
  }
  return s;
}

// Sum of one column of partials by one wave: lane shares in order, then the
// lanes by a fixed butterfly (the order reduce_partials uses, so both give
// the same bits).  Every lane returns the sum.
template <typename T>
__device__ __forceinline__ T wave_reduce_column(const T* col, int B) {
  const T s = B <= MAX_BLOCKS / 2 ? lane_share<MAX_BLOCKS / 2 / WAVE>(col, B) : lane_share<MAX_BLOCKS / WAVE>(col, B);
  return wave_sum(s);
}

template <int NL, typename T>
__device__ __forceinline__ void reduce_batches(const T* part, int nv, int B, T* out, int wid, int nwaves) {
  const int lane = threadIdx.x & (WAVE - 1);
  for (int c0 = wid * RED_BATCH; c0 < nv; c0 += nwaves * RED_BATCH) {
    T s[RED_BATCH];
#pragma unroll
    for (int q = 0; q < RED_BATCH; ++q) s[q] = T(0);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int b = lane + WAVE * i;
      const int bc = b < B ? b : B - 1;
#pragma unroll
      for (int q = 0; q < RED_BATCH; ++q) {
        const int c = (c0 + q < nv) ? c0 + q : nv - 1;
        const T v = part[(size_t)c * MAX_BLOCKS + bc];
        s[q] += (b < B) ? v : T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < RED_BATCH; ++q) {
      const T t = wave_sum(s[q]);
      if (lane == 0 && c0 + q < nv) out[c0 + q] = t;
    }
  }
}

// out[c] = sum over the B producer blocks of part[c][b], one wave per column
// (batches of RED_BATCH columns), each as wave_reduce_column.  With
// extra != nullptr the last wave first sums one more column, out[nv] = sum of
// extra[b], b < nE, the same way.  out is LDS; ends with a barrier.
template <typename T>
__device__ __forceinline__ void reduce_partials(const T* part, int nv, int B, T* out, const T* extra = nullptr,
                                                int nE = 0) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int nwaves = blockDim.x / WAVE;
  if (extra && wid == nwaves - 1) {
    const T t = wave_reduce_column(extra, nE);
    if (lane == 0) out[nv] = t;
  }
  if (B <= MAX_BLOCKS / 2) reduce_batches<MAX_BLOCKS / 2 / WAVE>(part, nv, B, out, wid, nwaves);
  else reduce_batches<MAX_BLOCKS / WAVE>(part, nv, B, out, wid, nwaves);
  __syncthreads();
}

}  // namespace gir
