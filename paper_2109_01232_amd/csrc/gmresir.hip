// C-ABI entry points and host driver of libgmresir (see include/gmresir.h).
//
// The driver owns no device memory: every buffer is carved out of the
// caller's workspace.  One refinement step of GMRES-IR (Algorithm 2) is
// enqueued without host synchronisation -- m iterations of three kernels,
// the back substitution, the fp64 correction and the fp64 residual -- and
// the host reads the small state header once per refinement to decide on
// convergence (the paper's restart-time check).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <iterator>
#include <map>
#include <tuple>
#include <mutex>
#include <utility>
#include <vector>

#include "gmresir.h"
#include "kernels.hpp"
#include "lowsync.hpp"

using namespace gir;

struct gmresir_matrix {
  int64_t n, nnz;
  const int32_t* rowptr;
  const int32_t* colidx;
  const double* vals64;
  float* vals32;
  int32_t* tile_row;
  int ntiles;
  int lds_nnz;  // largest nonzero count of a tile that is staged in LDS (<= TILE_NNZ)
  // sliced ELLPACK copy (used by the SpMV kernels when present)
  bool sell;
  int nslices;
  int32_t* sell_ptr;
  int32_t* sell_col;  // 32-bit columns, or (sell_d16) 16-bit offsets from the row in the same region,
                      // or (sell_shared) each slice's shared offsets at sell_ptr[s] / 64
  bool sell_d16;
  bool sell_shared;
  bool sell_wide;  // shared offsets and some slice wider than 9: the kernels' wide-round instances
  float* sell_v32;
  double* sell_v64;
  int device;
};

namespace {

constexpr int MAX_GRID = 1024;  // <= MAX_BLOCKS (partials per reduction)
constexpr int64_t GRAPH_MAX_N = 1 << 18;  // cycles of smaller systems run as HIP graphs
constexpr size_t ALIGN = 256;

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return GMRESIR_ERR_HIP;                                                      \
    }                                                                              \
  } while (0)

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// ---------------------------------------------------------------------------
// launch configuration: blocks = CUs x resident blocks per CU (one wave of
// blocks), capped by the useful parallelism
// ---------------------------------------------------------------------------

int device_cus(int dev) {
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  cache[dev] = cus;
  return cus;
}

// blocks of kern resident on the whole device at once (before any cap)
int resident_blocks(const void* kern, size_t smem, int threads) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, size_t>, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find({dev, kern, smem});
    if (it != cache.end()) return it->second;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, smem) != hipSuccess || nb <= 0) nb = 1;
  const int g = device_cus(dev) * nb;
  std::lock_guard<std::mutex> lk(mu);
  cache[{dev, kern, smem}] = g;
  return g;
}

int resident_grid(const void* kern, size_t smem, int threads = BLOCK) {
  return std::min(MAX_GRID, resident_blocks(kern, smem, threads));
}

int grid_rows(const void* kern, int64_t n, int threads = BLOCK) {
  int g = resident_grid(kern, 0, threads);
  int64_t want = (n + BLOCK - 1) / BLOCK;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, want));
}

// Row-tiled CSR kernels that leave per-block partial sums run one resident
// wave of blocks (at most MAX_GRID), each over a contiguous range of tiles,
// which amortises their prologue and partial sums (measured: one tile per
// block 17 % slower on the 5-point 1000^2 system, 2048 blocks 10 % slower on
// the 27-point 128^3 system).  Kernels without partials take one tile per
// block (grid_spmv).
int grid_tiles_part(const void* kern, int ntiles, size_t smem) {
  return std::max(1, std::min(resident_grid(kern, smem), ntiles));
}

Csr csr_of(const gmresir_matrix* A, bool fp64) {
  Csr c;
  c.n = (int)A->n;
  c.ntiles = A->ntiles;
  c.rowptr = A->rowptr;
  c.col = A->colidx;
  c.vals = fp64 ? (const void*)A->vals64 : (const void*)A->vals32;
  c.tile_row = A->tile_row;
  c.sell = A->sell ? 1 : 0;
  c.nslices = A->nslices;
  c.sptr = A->sell_ptr;
  c.scol = A->sell_col;
  c.scol16 = (const short*)A->sell_col;
  c.d16 = A->sell_d16 ? 1 : 0;
  c.shared = A->sell_shared ? 1 : 0;
  c.svals = fp64 ? (const void*)A->sell_v64 : (const void*)A->sell_v32;
  return c;
}

// Grid of an SpMV kernel without partial sums: one tile per block, or four
// slices (one per wave) per block.
int grid_spmv(const gmresir_matrix* A) {
  return A->sell ? std::max(1, (A->nslices + NWAVES - 1) / NWAVES) : std::max(1, A->ntiles);
}
// Grid of an SpMV kernel leaving per-block partial sums: one resident wave of
// blocks at most.
int grid_spmv_part(const gmresir_matrix* A, const void* kern, size_t smem) {
  return std::max(1, std::min(resident_grid(kern, smem), A->sell ? (A->nslices + NWAVES - 1) / NWAVES : A->ntiles));
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

struct Layout {
  size_t V, wtmp, w1, w2, r64, rhat, u, z, py, p0, p1, p2, minv, part, hdr, arr, total;
  long ldv;
  int m;
  int sT, sS;
  int bj;  // block-Jacobi block size (0: none)
  bool multi, poly;
  bool ls;  // one-reduction CGS2 (ortho = 1)
};

bool valid_params(const gmresir_params* p, const char** why) {
  if (!p) return *why = "params is NULL", false;
  if (p->restart < 1 || p->restart > MAX_RESTART) return *why = "restart must be in [1, 512]", false;
  if (p->inner_cap < 0) return *why = "inner_cap must be >= 0", false;
  if (p->max_iters <= 0) return *why = "max_iters must be > 0", false;
  if (!(p->rtol > 0.0) || !isfinite(p->rtol)) return *why = "rtol must be finite and > 0", false;
  if (p->inner_prec != GMRESIR_FP64 && p->inner_prec != GMRESIR_FP32) return *why = "inner_prec must be FP64 or FP32", false;
  if (p->inner_prec == GMRESIR_FP64 && p->basis_prec != GMRESIR_FP64)
    return *why = "an fp64 inner solve needs an fp64 basis", false;
  if (p->inner_prec == GMRESIR_FP32 && p->basis_prec != GMRESIR_FP32 && p->basis_prec != GMRESIR_BF16)
    return *why = "an fp32 inner solve needs an FP32 or BF16 basis", false;
  if (p->poly_degree < 0 || p->poly_degree > 255) return *why = "poly_degree must be in [0, 255]", false;
  if (p->check_mode != 0 && p->check_mode != 1) return *why = "check_mode must be 0 or 1", false;
  if (p->profile != 0 && p->profile != 1) return *why = "profile must be 0 or 1", false;
  if (p->poly_prec != 0 && p->poly_prec != GMRESIR_FP32) return *why = "poly_prec must be 0 or FP32", false;
  if (p->bj_block < 0 || p->bj_block > BJ_MAX) return *why = "bj_block must be in [0, 64]", false;
  if (p->bj_block > 0 && p->poly_degree > 0) return *why = "bj_block and poly_degree exclude each other", false;
  if (p->ortho != 0 && p->ortho != 1) return *why = "ortho must be 0 or 1", false;
  if (p->ortho == 1 && p->basis_prec == GMRESIR_BF16)
    return *why = "the one-reduction CGS2 (ortho 1) keeps the basis in the inner precision (no BF16)", false;
  if (p->ortho == 1 && p->restart > LS_MAX_RESTART) return *why = "ortho 1 needs restart <= 128", false;
  return true;
}

Layout make_layout(int64_t n, const gmresir_params* p) {
  Layout L{};
  L.m = p->restart;
  L.sT = p->inner_prec == GMRESIR_FP64 ? 8 : 4;
  L.sS = p->basis_prec == GMRESIR_FP64 ? 8 : p->basis_prec == GMRESIR_FP32 ? 4 : 2;
  int cap = p->inner_cap == 0 ? p->restart : p->inner_cap;
  L.multi = cap > p->restart;
  L.poly = p->poly_degree > 0;
  L.bj = p->bj_block;
  L.ls = p->ortho == 1;
  L.ldv = (long)((n + 127) / 128 * 128);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  // every internal vector is padded to ldv rows (vector loads of 2-4 rows)
  size_t vecT = (size_t)L.ldv * L.sT;
  L.V = take((size_t)L.ldv * (L.m + 1) * L.sS);
  L.wtmp = take(vecT);
  L.w1 = take(vecT);
  L.w2 = take(vecT);
  L.r64 = take((size_t)L.ldv * 8);
  bool need_uz = L.multi || L.poly || L.bj > 0;
  L.rhat = L.multi ? take(vecT) : 0;
  L.u = L.multi ? take(vecT) : 0;
  L.z = need_uz ? take(vecT) : 0;
  L.py = (L.poly || L.bj > 0) ? take(vecT) : 0;
  // block-Jacobi inverses by wave group (G = 64 / bs blocks) and column: G * bs entries per column
  L.minv = L.bj > 0 ? take((size_t)((((n + L.bj - 1) / L.bj) + WAVE / L.bj - 1) / (WAVE / L.bj)) * L.bj *
                           (WAVE / L.bj * L.bj) * L.sT)
                    : 0;
  L.p0 = L.poly ? take(vecT) : 0;
  L.p1 = L.poly ? take(vecT) : 0;
  L.p2 = L.poly ? take(vecT) : 0;
  L.part = take((size_t)MAX_BLOCKS * (L.ls ? std::max(PART_COLS, LS_PART_COLS) : PART_COLS) * 8);
  L.hdr = take(sizeof(StateHdr));
  size_t m = L.m;
  size_t arr = (3 * (m + 2) + 2 * (m + 1) * m + 2 * m + (m + 2) + 2 * m + LS_PART_COLS + (m + 2)) * sizeof(double);
  L.arr = take(arr);
  L.total = o;
  return L;
}

State state_of(char* ws, const Layout& L) {
  State st;
  st.hdr = (StateHdr*)(ws + L.hdr);
  double* a = (double*)(ws + L.arr);
  size_t m = L.m;
  st.ld = (int)(m + 1);
  st.h1 = a;
  a += m + 2;
  st.h1x = a;
  a += m + 2;
  st.h2 = a;
  a += m + 2;
  st.Hbar = a;
  a += (m + 1) * m;
  st.R = a;
  a += (m + 1) * m;
  st.cs = a;
  a += m;
  st.sn = a;
  a += m;
  st.g = a;
  a += m + 2;
  st.y = a;
  a += m;
  st.hist = a;
  a += m;
  st.red = a;
  a += LS_PART_COLS;
  st.dco = a;
  return st;
}

// ---------------------------------------------------------------------------
// profiling (start/end events of every launch) and algorithmic byte counts
// ---------------------------------------------------------------------------

struct Prof {
  bool on = false;
  hipStream_t stream = nullptr;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  double t[GMRESIR_NCAT] = {0};
  double bytes[GMRESIR_NCAT] = {0};
  int64_t launches[GMRESIR_NCAT] = {0};
  // Launches since the last commit.  Kernels of iteration j (tag = j) after
  // the step where a cycle stopped exit at once without work; they are not
  // booked.  "early" kernels of an iteration (polynomial steps, SpMV +
  // projection, the h1/Givens tail) still run in the iteration right after
  // the stop, because the stop is decided by that tail.
  struct Entry {
    int cat;
    double b;
    int tag;
    bool early;
    hipEvent_t e0, e1;
  };
  std::vector<Entry> pend;
  int tag = -1;
  bool early = false;
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  // Graph recording (rec != nullptr): launches become kernel nodes chained
  // after `last`, and their bookings are kept in `recorded`.
  hipGraph_t rec = nullptr;
  hipGraphNode_t last = nullptr;
  bool rec_failed = false;
  std::vector<Entry> recorded;

  template <typename Tup, size_t... I>
  static void arg_ptrs(Tup& t, void** p, std::index_sequence<I...>) {
    ((p[I] = (void*)&std::get<I>(t)), ...);
  }

  // Launch kern on strm and book it under category cat with b algorithmic
  // bytes; when profiling, the kernel's own start and end are recorded
  // (hipExtLaunchKernel events, no extra packets between kernels).
  template <typename... P, typename... Args>
  void launch(int cat, double b, void (*kern)(P...), dim3 grid, dim3 block, size_t smem, hipStream_t strm,
              Args... args) {
    Entry e{cat, b, tag, early, nullptr, nullptr};
    if (rec) {
      // node arguments converted to the kernel's own parameter types
      std::tuple<std::remove_cv_t<std::remove_reference_t<P>>...> t(args...);
      void* ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
      arg_ptrs(t, ptrs, std::index_sequence_for<P...>{});
      hipKernelNodeParams kp{};
      kp.func = (void*)kern;
      kp.gridDim = grid;
      kp.blockDim = block;
      kp.sharedMemBytes = (unsigned)smem;
      kp.kernelParams = ptrs;
      kp.extra = nullptr;
      hipGraphNode_t node = nullptr;
      if (hipGraphAddKernelNode(&node, rec, last ? &last : nullptr, last ? 1 : 0, &kp) != hipSuccess)
        rec_failed = true;
      else
        last = node;
      recorded.push_back(e);
      return;
    }
    if (!on) {
      hipLaunchKernelGGL(kern, grid, block, smem, strm, args...);
    } else {
      e.e0 = take();
      e.e1 = take();
      hipExtLaunchKernelGGL(kern, grid, block, (std::uint32_t)smem, strm, e.e0, e.e1, 0u, args...);
    }
    pend.push_back(e);
  }
  // After a stream synchronisation: book the pending launches; k = steps the
  // cycle among them completed.
  void commit(int k) {
    for (const Entry& e : pend) {
      const bool ran = e.tag < 0 || e.tag < k || (e.tag == k && e.early);
      if (!ran) continue;
      bytes[e.cat] += e.b;
      launches[e.cat] += 1;
      float ms = 0.f;
      if (e.e0 && e.e1 && hipEventElapsedTime(&ms, e.e0, e.e1) == hipSuccess) t[e.cat] += ms * 1e-3;
    }
    pend.clear();
    used = 0;
  }
  ~Prof() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// ---------------------------------------------------------------------------
// polynomial program: the product form of p(A) as a list of SpMV steps
// ---------------------------------------------------------------------------

enum PBuf { PB_SRC = 0, PB_P0, PB_P1, PB_P2, PB_NONE };

struct PStep {
  int x, w, d;  // gathered source, own-row auxiliary vector, output vector (PB_*)
  bool has_y, y_read;
  double ay, aw, ax, at, bw, bx, bt;
};

// roots: nr (re, im) pairs in application order, conjugate pairs adjacent.
// y accumulates p(A) src; see the oracle-independent derivation in the
// Python package's documentation of the product form.
bool build_poly_program(int nr, const double* roots, std::vector<PStep>& prog, const char** why) {
  prog.clear();
  if (nr < 2) return *why = "a polynomial preconditioner needs at least 2 roots", false;
  int cur = PB_SRC;
  auto other = [](int b) { return b == PB_P0 ? PB_P1 : PB_P0; };
  bool y_has = false;
  int i = 0;
  while (i < nr) {
    const double re = roots[2 * i], im = roots[2 * i + 1];
    if (im == 0.0) {
      if (re == 0.0 || !isfinite(re)) return *why = "polynomial root is zero or not finite", false;
      if (i == nr - 1) {
        // last root: y += d_prev / theta, folded into the previous step
        PStep& p = prog.back();
        const double inv = 1.0 / re;
        if (!p.has_y) {
          p.has_y = true;
          p.y_read = y_has;
          p.ay = 1.0;
          p.aw = p.ax = p.at = 0.0;
        }
        p.aw += p.bw * inv;
        p.ax += p.bx * inv;
        p.at += p.bt * inv;
        p.d = PB_NONE;
        i += 1;
      } else {
        PStep s{};
        s.x = cur;
        s.w = PB_NONE;
        s.has_y = true;
        s.y_read = y_has;
        s.ay = 1.0;
        s.ax = 1.0 / re;
        s.d = other(cur);
        s.bx = 1.0;
        s.bt = -1.0 / re;
        prog.push_back(s);
        cur = s.d;
        y_has = true;
        i += 1;
      }
    } else {
      if (i + 1 >= nr || roots[2 * (i + 1)] != re || roots[2 * (i + 1) + 1] != -im)
        return *why = "complex roots must come in adjacent conjugate pairs", false;
      const double mu = re * re + im * im;
      const bool last = (i + 2 == nr);
      PStep a{};
      a.x = cur;
      a.w = PB_NONE;
      a.has_y = true;
      a.y_read = y_has;
      a.ay = 1.0;
      a.ax = 2.0 * re / mu;
      a.at = -1.0 / mu;
      a.d = last ? PB_NONE : PB_P2;
      a.bt = 1.0;
      prog.push_back(a);
      y_has = true;
      if (!last) {
        PStep b{};
        b.x = PB_P2;
        b.w = cur;
        b.has_y = false;
        b.d = other(cur);
        b.bw = 1.0;
        b.bx = -2.0 * re / mu;
        b.bt = 1.0 / mu;
        prog.push_back(b);
        cur = b.d;
      }
      i += 2;
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// the solver context
// ---------------------------------------------------------------------------

template <typename T, typename S>
struct Ctx {
  const gmresir_matrix* A;
  hipStream_t stream;
  Layout L;
  char* ws;
  State st;
  S* V;
  T *wtmp, *w1, *w2, *rhat, *u, *z, *py, *p0, *p1, *p2;
  double* r64;
  T* part;
  int n;
  Csr Ain;  // matrix in inner precision
  Csr A64;
  Prof* prof;
  std::vector<PStep> prog;
  bool poly_on = false;  // inner operator is A p(A)
  T* minv = nullptr;  // block-Jacobi inverses in inner precision (L.bj > 0): inner operator A M^{-1}
  // fp32 polynomial inside an fp64 inner solve: its buffers are carved from
  // the fp64 polynomial buffers (ldv fp32 entries each; two per buffer)
  bool poly32 = false;
  Csr A32;
  float *q32[3] = {nullptr, nullptr, nullptr}, *s32 = nullptr, *y32 = nullptr;


  Ctx(const gmresir_matrix* A_, char* ws_, const Layout& L_, hipStream_t s, Prof* pr) : A(A_), stream(s), L(L_), ws(ws_), prof(pr) {
    st = state_of(ws, L);
    V = (S*)(ws + L.V);
    wtmp = (T*)(ws + L.wtmp);
    w1 = (T*)(ws + L.w1);
    w2 = (T*)(ws + L.w2);
    r64 = (double*)(ws + L.r64);
    rhat = L.multi ? (T*)(ws + L.rhat) : nullptr;
    u = L.multi ? (T*)(ws + L.u) : nullptr;
    z = (L.multi || L.poly || L.bj > 0) ? (T*)(ws + L.z) : nullptr;
    py = (L.poly || L.bj > 0) ? (T*)(ws + L.py) : nullptr;
    minv = L.bj > 0 ? (T*)(ws + L.minv) : nullptr;
    p0 = L.poly ? (T*)(ws + L.p0) : nullptr;
    p1 = L.poly ? (T*)(ws + L.p1) : nullptr;
    p2 = L.poly ? (T*)(ws + L.p2) : nullptr;
    part = (T*)(ws + L.part);
    n = (int)A->n;
    Ain = csr_of(A, sizeof(T) == 8);
    A64 = csr_of(A, true);
    A32 = csr_of(A, false);
    if (L.poly && sizeof(T) == 8) {
      q32[0] = (float*)p0;
      q32[1] = (float*)p1;
      q32[2] = (float*)p2;
      s32 = (float*)p0 + L.ldv;
      y32 = (float*)p1 + L.ldv;
    }
  }

  // LDS of the tiled SpMV products (none for the sliced ELLPACK kernels)
  size_t lds_tiled() const { return (size_t)A->lds_nnz * sizeof(T); }
  size_t lds_in() const { return A->sell ? 0 : lds_tiled(); }
  size_t lds_64() const { return A->sell ? 0 : (size_t)A->lds_nnz * sizeof(double); }
  double sT() const { return (double)sizeof(T); }
  double sS() const { return (double)sizeof(S); }
  // algorithmic bytes of the CSR arrays: values + 4-byte column indices +
  // row pointers (what the CSR SpMV must read once; the sliced copy's 16-bit
  // column offsets read less, which the counter traffic shows)
  double spmv_bytes(bool sell_path = true) const {
    (void)sell_path;
    return (sT() + 4.0) * A->nnz + 4.0 * (A->n + 1);
  }

  T* buf(int b, T* src) {
    switch (b) {
      case PB_SRC: return src;
      case PB_P0: return p0;
      case PB_P1: return p1;
      case PB_P2: return p2;
      default: return nullptr;
    }
  }

  // y_out = p(A) src; scaled: src holds the unnormalised next basis vector
  // (wtmp, scaled by inv_h and rounded to the basis type, written into V[:, j]).
  void run_poly(T* src, bool scaled, int j, T* y_out, int check_done, int cat, int nB = 0) {
    for (size_t s = 0; s < prog.size(); ++s) {
      const PStep& ps = prog[s];
      PolyCoef<T> cf;
      cf.ay = (T)ps.ay;
      cf.aw = (T)ps.aw;
      cf.ax = (T)ps.ax;
      cf.at = (T)ps.at;
      cf.bw = (T)ps.bw;
      cf.bx = (T)ps.bx;
      cf.bt = (T)ps.bt;
      cf.has_y = ps.has_y;
      cf.y_read = ps.y_read;
      cf.has_d = ps.d != PB_NONE;
      cf.has_w = ps.w != PB_NONE;
      T* X = buf(ps.x, src);
      T* W = buf(ps.w, src);
      T* D = buf(ps.d, src);
      const int w_scaled = (scaled && ps.w == PB_SRC) ? 1 : 0;
      const int write_v = (scaled && s == 0) ? 1 : 0;
      double b = spmv_bytes() + sT() * n * (1 + (ps.has_y ? 1 : 0) + (ps.y_read ? 1 : 0) + (cf.has_w ? 1 : 0) +
                                            (cf.has_d ? 1 : 0)) +
                 (write_v ? sS() * n : 0.0);
      if (scaled && ps.x == PB_SRC) {
        auto kern = k_poly_step<T, S, true>;
        int g = grid_spmv(A);
        prof->launch(cat, b, kern, dim3(g), dim3(BLOCK), lds_in(), stream, Ain, X, V, L.ldv, j, write_v, W, w_scaled, y_out, D, cf, st, check_done, (const T*)norm_part(), nB);
      } else {
        auto kern = k_poly_step<T, S, false>;
        int g = grid_spmv(A);
        prof->launch(cat, b, kern, dim3(g), dim3(BLOCK), lds_in(), stream, Ain, X, V, L.ldv, j, 0, W, w_scaled, y_out, D, cf, st, check_done, (const T*)norm_part(), nB);
      }
    }
  }

  // y_out = p(A) src with the fp32 copy of A and fp32 vectors (poly32); the
  // same product-form program as run_poly, never scaled.
  void run_poly32(float* src, float* y_out, int check_done, int cat) {
    auto pick = [&](int b) -> float* {
      switch (b) {
        case PB_SRC: return src;
        case PB_P0: return q32[0];
        case PB_P1: return q32[1];
        case PB_P2: return q32[2];
        default: return nullptr;
      }
    };
    const size_t lds = A->sell ? 0 : (size_t)A->lds_nnz * sizeof(float);
    const double idx = 4.0;  // algorithmic: 4-byte column indices
    for (size_t s = 0; s < prog.size(); ++s) {
      const PStep& ps = prog[s];
      PolyCoef<float> cf;
      cf.ay = (float)ps.ay;
      cf.aw = (float)ps.aw;
      cf.ax = (float)ps.ax;
      cf.at = (float)ps.at;
      cf.bw = (float)ps.bw;
      cf.bx = (float)ps.bx;
      cf.bt = (float)ps.bt;
      cf.has_y = ps.has_y;
      cf.y_read = ps.y_read;
      cf.has_d = ps.d != PB_NONE;
      cf.has_w = ps.w != PB_NONE;
      float* X = pick(ps.x);
      float* W = pick(ps.w);
      float* D = pick(ps.d);
      double b = (4.0 + idx) * A->nnz + 4.0 * (A->n + 1) +
                 4.0 * n * (1 + (ps.has_y ? 1 : 0) + (ps.y_read ? 1 : 0) + (cf.has_w ? 1 : 0) + (cf.has_d ? 1 : 0));
      auto kern = k_poly_step<float, float, false>;
      int g = grid_spmv(A);
      prof->launch(cat, b, kern, dim3(g), dim3(BLOCK), lds, stream, A32, (const float*)X, (float*)nullptr, L.ldv, 0, 0,
                   (const float*)W, 0, y_out, D, cf, st, check_done, (const float*)nullptr, 0);
    }
  }

  // block-Jacobi inverses computed in inner precision from that precision's
  // copy of the CSR values (once per solve)
  void bj_setup() {
    const long nblk = ((long)n + L.bj - 1) / L.bj;
    const long per_wave = WAVE / L.bj;  // blocks a wave inverts together
    const long grid = (nblk + per_wave - 1) / per_wave;
    const double b = (sT() + 4.0) * A->nnz + 4.0 * (n + 1) + sT() * nblk * L.bj * L.bj;
    const T* vals = sizeof(T) == 8 ? (const T*)A->vals64 : (const T*)A->vals32;
    prof->launch(GMRESIR_CAT_OTHER, b, k_bj_invert<T>, dim3((unsigned)grid), dim3(WAVE), 0, stream, n,
                 (const int*)A->rowptr, (const int*)A->colidx, vals, L.bj, minv);
  }

  int bj_grid() const {
    const long nblk = ((long)n + L.bj - 1) / L.bj;
    const long per_wave = WAVE / L.bj;  // blocks a wave takes at once
    const long ngrp = (nblk + per_wave - 1) / per_wave;
    const long g = (ngrp + NWAVES - 1) / NWAVES;
    return (int)std::min<long>(g, 1L << 20);
  }

  // y = M^{-1} src; scaled: src is wtmp, v_j = round(wtmp * inv) also goes into V[:, j]
  void bj_apply(const T* src, bool scaled, int j, T* y_out, int check_done, int cat, int nB = 0) {
    const double b = sT() * n * L.bj + sT() * n * 2 + (scaled ? sS() * n : 0.0);
    if (scaled) {
      auto kern = k_bj_apply<T, S, true>;
      prof->launch(cat, b, kern, dim3(bj_grid()), dim3(BLOCK), 0, stream, n, L.bj, (const T*)minv, src, V, L.ldv,
                   j, y_out, st, check_done, (const T*)norm_part(), nB);
    } else {
      auto kern = k_bj_apply<T, S, false>;
      prof->launch(cat, b, kern, dim3(bj_grid()), dim3(BLOCK), 0, stream, n, L.bj, (const T*)minv, src, V, L.ldv,
                   j, y_out, st, check_done, (const T*)norm_part(), 0);
    }
  }

  void narrow(const double* x64, float* y, int check_done, int cat) {
    auto kern = k_narrow;
    int g = grid_rows((const void*)kern, n);
    prof->launch(cat, 12.0 * n, kern, dim3(g), dim3(BLOCK), 0, stream, n, x64, y, st, check_done);
  }

  void widen(const float* x, double* y64, int check_done, int cat) {
    auto kern = k_widen;
    int g = grid_rows((const void*)kern, n);
    prof->launch(cat, 12.0 * n, kern, dim3(g), dim3(BLOCK), 0, stream, n, x, y64, st, check_done);
  }

  // partials of ||w''||^2 written by k_update_norm (their own column, so
  // they survive the projections of the next iteration)
  T* norm_part() const { return part + (size_t)NORM_SLOT * MAX_BLOCKS; }
  int norm_grid() const { return grid_rows((const void*)k_update_norm<T, S, 2 * BLOCK>, n, 2 * BLOCK); }

  // nB: producer blocks of the previous iteration's norm partials (0 at a
  // cycle start); the tail also makes the Givens step of iteration j - 1.
  template <int SLOTS, bool SCALED>
  void launch_spmv_proj(const T* src, int j, int kmax, int nB) {
    constexpr int KMAX = NWAVES * SLOTS;
    const int C = std::min(j + 1, KMAX);
    // basis columns read from memory: all handled columns but the new one (SCALED)
    const int nread = SCALED ? std::min(j, C) : C;
    // small systems (under 64 K rows) keep the tiled kernel, whose 512-row
    // tiles give more blocks than the 1024-row stages
    const bool sell_path = A->sell && A->nslices >= 1024;
    double b = spmv_bytes(sell_path) + sT() * n * 2 + sS() * n * nread + (SCALED ? sS() * n : 0.0);
    int g;
    if (sell_path) {
      // up to 32 columns: eight waves per block with half the column slots
      // each (same KMAX), twice the loads in flight per CU at the same number
      // of partial sums (measured on the 1000^2 system: 18.8 -> 16.4 us at
      // k <= 16, 27.2 -> 25.0 us at k <= 32).  Up to 64 columns eight waves
      // pay only for rows of more than 6 nonzeros, where the SpMV part needs
      // the loads in flight (27-point 128^3: 138 -> 122 us; 5-point 1000^2:
      // 37.2 -> 41.1 us, so short rows keep four waves there).
      constexpr int NW = KMAX <= 32 ? 2 * NWAVES : NWAVES;
      constexpr int SPS = (sizeof(T) == 8 ? TILE_ROWS : 2 * TILE_ROWS) / SELL_C;  // slices per stage
      bool done = false;
      if constexpr (KMAX == 64 || KMAX == 128) {
        if (A->nnz > 6 * A->n) {
          auto kern = A->sell_wide ? k_spmv_proj_sell<T, S, KMAX / (2 * NWAVES), SCALED, 2 * NWAVES, true>
                                   : k_spmv_proj_sell<T, S, KMAX / (2 * NWAVES), SCALED, 2 * NWAVES, false>;
          g = std::max(1, std::min(resident_grid((const void*)kern, 0, 2 * NWAVES * WAVE), (A->nslices + SPS - 1) / SPS));
          prof->launch(GMRESIR_CAT_SPMV_PROJ, b, kern, dim3(g), dim3(2 * NWAVES * WAVE), 0, stream, Ain, src, V, L.ldv,
                       j, w1, st, part, (const T*)norm_part(), nB);
          done = true;
        }
      }
      if (!done) {
        auto kern = A->sell_wide ? k_spmv_proj_sell<T, S, KMAX / NW, SCALED, NW, true>
                                 : k_spmv_proj_sell<T, S, KMAX / NW, SCALED, NW, false>;
        g = std::max(1, std::min(resident_grid((const void*)kern, 0, NW * WAVE), (A->nslices + SPS - 1) / SPS));
        prof->launch(GMRESIR_CAT_SPMV_PROJ, b, kern, dim3(g), dim3(NW * WAVE), 0, stream, Ain, src, V, L.ldv, j, w1,
                     st, part, (const T*)norm_part(), nB);
      }
    } else {
      auto kern = k_spmv_proj<T, S, SLOTS, SCALED>;
      g = grid_tiles_part((const void*)kern, Ain.ntiles, lds_tiled());
      prof->launch(GMRESIR_CAT_SPMV_PROJ, b, kern, dim3(g), dim3(BLOCK), lds_tiled(), stream, Ain, src, V, L.ldv, j,
                   w1, st, part, (const T*)norm_part(), nB);
    }
    auto tail = k_reduce_h1_givens<T>;
    const int tg = (C + NWAVES - 1) / NWAVES + (j > 0 ? 1 : 0);
    prof->launch(GMRESIR_CAT_TAIL, 0.0, tail, dim3(tg), dim3(BLOCK), 0, stream, (const T*)part, C, g, (const T*)norm_part(), nB, st, j - 1, kmax);
  }

  void reduce_h(int cat, int producer_grid, int nv, double* h) {
    auto kern = k_reduce_cols<T>;
    const int tg = (nv + NWAVES - 1) / NWAVES;
    prof->launch(cat == GMRESIR_CAT_OTHER ? cat : GMRESIR_CAT_TAIL, 0.0, kern, dim3(tg), dim3(BLOCK), 0, stream, (const T*)part, nv, producer_grid, h);
  }

  template <bool SCALED>
  void spmv_proj_dispatch(const T* src, int j, int kmax, int nB) {
    const int k = j + 1;
    if (k <= 16) launch_spmv_proj<4, SCALED>(src, j, kmax, nB);
    else if (k <= 32) launch_spmv_proj<8, SCALED>(src, j, kmax, nB);
    else if (k <= 64) launch_spmv_proj<16, SCALED>(src, j, kmax, nB);
    else launch_spmv_proj<32, SCALED>(src, j, kmax, nB);
    // columns beyond the fused limit (V[:, j] is in memory by now); they
    // skip when the tail has just stopped the cycle
    prof->early = false;
    for (int c0 = 128; c0 < k; c0 += 64) dots(c0, std::min(64, k - c0), w1, st.h1_of(j), GMRESIR_CAT_OTHER);
  }

  void dots(int c0, int nc, const T* w, double* h, int cat) {
    auto kern = k_dots<T, S>;
    int g = grid_rows((const void*)kern, n);
    prof->launch(cat, sS() * n * nc + sT() * n, kern, dim3(g), dim3(BLOCK), 0, stream, n, V, L.ldv, c0, nc, w, st, 1, part);
    reduce_h(cat, g, nc, h + c0);
  }

  template <int SLOTS, int R, int WV>
  void launch_update_proj(int k) {
    auto kern = k_update_proj<T, S, SLOTS, R, WV>;
    int g = grid_rows((const void*)kern, n, WV * WAVE);
    prof->launch(GMRESIR_CAT_UPDATE_PROJ, sT() * n * 2 + sS() * n * k, kern, dim3(g), dim3(WV * WAVE), 0, stream, n, w1,
                 w2, V, L.ldv, k, st, part);
    reduce_h(GMRESIR_CAT_UPDATE_PROJ, g, k, st.h2);
  }

  void update_proj_dispatch(int k) {
    // rows per lane: 16-byte loads of fp64 (2) and fp32 (4), 8-byte loads
    // of bf16 (4: the pipelined steps hold two register sets)
    constexpr int R = sizeof(S) == 2 ? 4 : 16 / sizeof(S);
    // an fp32 basis of 33..64 columns: eight waves (the grid is capped at
    // MAX_BLOCKS blocks; 27-point 128^3: 47.4 -> 45.3 us per launch); a bf16
    // basis keeps four (eight measured slower: 34.5 -> 45.0 us)
    constexpr bool W8 = sizeof(S) == 4 && sizeof(T) == 4;
    if (k <= 16) launch_update_proj<4, R, 4>(k);
    else if (k <= 32) launch_update_proj<8, R, 4>(k);
    else if (k <= 48) launch_update_proj<W8 ? 6 : 12, R, W8 ? 8 : 4>(k);
    else if (k <= 64) launch_update_proj<W8 ? 8 : 16, R, W8 ? 8 : 4>(k);
    // widest bases: fp32 / bf16 split the columns over eight waves (4.4 vs
    // 3.7 TB/s measured at m = 100); fp64 keeps four waves, one row per lane
    else if (k <= 128) {
      if constexpr (sizeof(T) == 8) {
        if (k <= 96) launch_update_proj<24, 1, 4>(k);
        else launch_update_proj<32, 1, 4>(k);
      } else {
        if (k <= 96) launch_update_proj<12, R, 8>(k);
        else launch_update_proj<16, R, 8>(k);
      }
    } else {
      auto kern = k_update<T, S>;
      int g = grid_rows((const void*)kern, n);
      prof->launch(GMRESIR_CAT_OTHER, sT() * n * 2 + sS() * n * k, kern, dim3(g), dim3(BLOCK), 0, stream, n, w1, w2, V,
                   L.ldv, k, (const double*)st.h1_of(k - 1), st);
      for (int c0 = 0; c0 < k; c0 += 64) dots(c0, std::min(64, k - c0), w2, st.h2, GMRESIR_CAT_OTHER);
    }
  }

  static constexpr int NORM_NT = 2 * BLOCK;
  void update_norm(int j) {
    auto kern = k_update_norm<T, S, NORM_NT>;
    prof->launch(GMRESIR_CAT_UPDATE_NORM, sT() * n * 2 + sS() * n * (j + 1), kern, dim3(norm_grid()), dim3(NORM_NT), 0,
                 stream, n, w2, wtmp, V, L.ldv, j, st, norm_part());
  }

  // Givens step of the last iteration of a cycle (the others run in the
  // tail after the next iteration's SpMV)
  void norm_givens(int j, int kmax) {
    auto tail = k_norm_givens<T>;
    prof->launch(GMRESIR_CAT_TAIL, 0.0, tail, dim3(1), dim3(BLOCK), 0, stream, (const T*)norm_part(), norm_grid(), st, j, kmax);
  }

  // one inner iteration j of a cycle of at most kmax steps
  void iteration(int j, int kmax) {
    const int nB = j > 0 ? norm_grid() : 0;
    prof->tag = j;
    prof->early = true;
    if (L.bj > 0) {
      bj_apply(wtmp, true, j, z, 1, GMRESIR_CAT_POLY, nB);
      spmv_proj_dispatch<false>(z, j, kmax, nB);
    } else if (poly_on && poly32) {
      auto kern = k_scale_narrow<T, S>;
      int g = grid_rows((const void*)kern, n);
      prof->launch(GMRESIR_CAT_POLY, sT() * n + sS() * n + 4.0 * n, kern, dim3(g), dim3(BLOCK), 0, stream, n,
                   (const T*)wtmp, V, L.ldv, j, s32, st, (const T*)norm_part(), nB);
      run_poly32(s32, y32, 1, GMRESIR_CAT_POLY);
      widen(y32, (double*)z, 1, GMRESIR_CAT_POLY);
      spmv_proj_dispatch<false>(z, j, kmax, nB);
    } else if (poly_on) {
      run_poly(wtmp, true, j, z, 1, GMRESIR_CAT_POLY, nB);
      spmv_proj_dispatch<false>(z, j, kmax, nB);
    } else {
      spmv_proj_dispatch<true>(wtmp, j, kmax, nB);
    }
    prof->early = false;
    update_proj_dispatch(j + 1);
    update_norm(j);
  }

  // -------------------------------------------------------------------------
  // one-reduction CGS2 (ortho = 1): per iteration the SpMV with the partial
  // sums of the one reduction, the column sums, the dense step and the update
  // sweep; p = A M^{-1} q lives in w1, the once-orthogonalised q in w2
  // -------------------------------------------------------------------------

  T* q_ls() const { return w2; }
  T* p_ls() const { return w1; }
  static int ls_ncols(int j, bool has_p) { return LS_A + (has_p ? 2 * j : j); }

  void ls_reduce(int ncols, int producer_grid) {
    auto kern = k_reduce_cols<T>;
    prof->launch(GMRESIR_CAT_TAIL, 0.0, kern, dim3((ncols + NWAVES - 1) / NWAVES), dim3(BLOCK), 0, stream,
                 (const T*)part, ncols, producer_grid, st.red);
  }

  template <int SLOTS, int NW, bool SCALED>
  void ls_spmv_dots_sell_launch(const T* gsrc, const T* own, int j, bool own_read) {
    auto kern = A->sell_wide ? k_ls_spmv_dots_sell<T, S, SLOTS, SCALED, NW, true>
                             : k_ls_spmv_dots_sell<T, S, SLOTS, SCALED, NW, false>;
    constexpr int SPS = (sizeof(T) == 8 ? TILE_ROWS : 2 * TILE_ROWS) / SELL_C;  // slices per stage
    const int g = std::max(1, std::min(resident_grid((const void*)kern, 0, NW * WAVE), (A->nslices + SPS - 1) / SPS));
    const double b = spmv_bytes() + 2.0 * sT() * n + sS() * n * j + (SCALED ? sS() * n : own_read ? sT() * n : 0.0);
    prof->launch(GMRESIR_CAT_SPMV_PROJ, b, kern, dim3(g), dim3(NW * WAVE), 0, stream, Ain, gsrc, own, V, L.ldv, j,
                 p_ls(), st, part);
    ls_reduce(ls_ncols(j, true), g);
  }

  template <bool SCALED>
  void ls_spmv_dots_sell(const T* gsrc, const T* own, int j, bool own_read) {
    if (j <= 16) ls_spmv_dots_sell_launch<2, 8, SCALED>(gsrc, own, j, own_read);
    else if (j <= 32) ls_spmv_dots_sell_launch<4, 8, SCALED>(gsrc, own, j, own_read);
    else if (j <= 64) ls_spmv_dots_sell_launch<8, 8, SCALED>(gsrc, own, j, own_read);
    else ls_spmv_dots_sell_launch<16, 8, SCALED>(gsrc, own, j, own_read);
  }

  template <int SLOTS, bool HAS_P>
  void ls_dots_launch(const T* q, int j) {
    constexpr int WV = NWAVES;
    auto kern = k_ls_dots<T, S, SLOTS, HAS_P, WV>;
    const int g = grid_rows((const void*)kern, n, WV * WAVE);
    const double b = sS() * n * j + sT() * n * (HAS_P ? 2 : 1);
    prof->launch(GMRESIR_CAT_SPMV_PROJ, b, kern, dim3(g), dim3(WV * WAVE), 0, stream, n, q, (const T*)p_ls(),
                 (const S*)V, L.ldv, j, st, part);
    ls_reduce(ls_ncols(j, HAS_P), g);
  }

  template <bool HAS_P>
  void ls_dots(const T* q, int j) {
    if (j <= 16) ls_dots_launch<4, HAS_P>(q, j);
    else if (j <= 32) ls_dots_launch<8, HAS_P>(q, j);
    else if (j <= 64) ls_dots_launch<16, HAS_P>(q, j);
    else ls_dots_launch<32, HAS_P>(q, j);
  }

  // plain SpMV p = A src that skips a stopped cycle (matrices without a fused sliced kernel)
  void ls_spmv(const T* src) {
    auto kern = k_ls_spmv<T>;
    prof->launch(GMRESIR_CAT_SPMV_PROJ, spmv_bytes() + 2.0 * sT() * n, kern, dim3(grid_spmv(A)), dim3(BLOCK), lds_in(),
                 stream, Ain, src, p_ls(), st);
  }

  void ls_dense(int j, int kmax) {
    // dynamic LDS: the Hessenberg columns 0..j-1, rows 0..j, in inner precision
    const size_t smem = (size_t)(j + 1) * j * sizeof(T);
    prof->launch(GMRESIR_CAT_TAIL, 0.0, k_ls_dense<T>, dim3(1), dim3(BLOCK), smem, stream, st, (const double*)st.red,
                 st.dco, j, kmax);
  }

  void ls_update(int j) {
    auto kern = k_ls_update<T, S, 2 * BLOCK>;
    const int g = grid_rows((const void*)kern, n, 2 * BLOCK);
    const double b = sS() * n * (j + 1) + sT() * n * (j > 0 ? 3 : 2);
    prof->launch(GMRESIR_CAT_UPDATE_NORM, b, kern, dim3(g), dim3(2 * BLOCK), 0, stream, n, (const T*)p_ls(), q_ls(), V,
                 L.ldv, j, st, (const double*)st.dco);
  }

  // iteration j: p = A M^{-1} q_j (j = 0: A M^{-1} v_0) with the one
  // reduction, the dense step (completes column j-1), the update sweep
  void ls_iteration(int j, int kmax) {
    prof->tag = j;
    prof->early = true;
    const bool precond = L.bj > 0 || poly_on;
    const bool fused = A->sell && A->nslices >= 1024;
    T* q = q_ls();
    T* v0 = (T*)V;  // S == T on this path
    const T* gsrc = q;
    const T* own = q;
    if (precond) {
      // the preconditioner's first kernel forms v_0 into V[:, 0] at j = 0
      const T* src = j == 0 ? (const T*)wtmp : (const T*)q;
      if (L.bj > 0) {
        bj_apply(src, j == 0, 0, z, 1, GMRESIR_CAT_POLY, 0);
      } else if (poly32) {
        if (j == 0) {
          auto kern = k_scale_narrow<T, S>;
          const int g = grid_rows((const void*)kern, n);
          prof->launch(GMRESIR_CAT_POLY, sT() * n + sS() * n + 4.0 * n, kern, dim3(g), dim3(BLOCK), 0, stream, n,
                       (const T*)wtmp, V, L.ldv, 0, s32, st, (const T*)norm_part(), 0);
        } else {
          narrow((const double*)q, s32, 1, GMRESIR_CAT_POLY);
        }
        run_poly32(s32, y32, 1, GMRESIR_CAT_POLY);
        widen(y32, (double*)z, 1, GMRESIR_CAT_POLY);
      } else {
        run_poly((T*)src, j == 0, 0, z, 1, GMRESIR_CAT_POLY, 0);
      }
      gsrc = z;
      own = j == 0 ? v0 : q;
    } else if (j == 0 && !fused) {
      auto kern = k_ls_form_v0<T, S>;
      prof->launch(GMRESIR_CAT_SPMV_PROJ, sT() * n + sS() * n, kern, dim3(grid_rows((const void*)kern, n)),
                   dim3(BLOCK), 0, stream, n, (const T*)wtmp, V, st);
      gsrc = own = v0;
    }
    if (fused) {
      if (j == 0 && !precond) ls_spmv_dots_sell<true>(wtmp, nullptr, 0, false);
      else ls_spmv_dots_sell<false>(gsrc, own, j, precond);
    } else {
      ls_spmv(gsrc);
      ls_dots<true>(own, j);
    }
    ls_dense(j, kmax);
    prof->early = false;
    ls_update(j);
  }

  // the cycle's last column: the reduction without an SpMV, then its Givens step
  void ls_cycle(int kmax) {
    for (int j = 0; j < kmax; ++j) ls_iteration(j, kmax);
    prof->tag = kmax;
    prof->early = true;
    ls_dots<false>(q_ls(), kmax);
    ls_dense(kmax, kmax);
    prof->tag = -1;
    prof->early = false;
  }

  // Small systems are bound by the host's launch rate (~5 kernels of a few
  // microseconds per step): their cycles run as one HIP graph, recorded on
  // first use and replayed for every later cycle of the same length (all
  // kernel arguments are fixed per position in the cycle; the per-cycle state
  // lives in the workspace).
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_kmax = -1;
  bool graph_ok = false;
  std::vector<typename Prof::Entry> graph_entries;

  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
    graph_kmax = -1;
  }
  ~Ctx() { drop_graph(); }

  void run_cycle(int kmax) {
    if (!graph_ok) {
      cycle(kmax);
      return;
    }
    if (graph_kmax != kmax) {
      drop_graph();
      bool ok = hipGraphCreate(&graph, 0) == hipSuccess;
      if (ok) {
        prof->rec = graph;
        prof->last = nullptr;
        prof->rec_failed = false;
        prof->recorded.clear();
        cycle(kmax);
        prof->rec = nullptr;
        ok = !prof->rec_failed && hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0) == hipSuccess;
      }
      if (!ok) {
        // fall back to direct launches for the rest of the solve
        (void)hipGetLastError();
        drop_graph();
        graph_ok = false;
        cycle(kmax);
        return;
      }
      graph_kmax = kmax;
      graph_entries = prof->recorded;
    }
    (void)hipGraphLaunch(graph_exec, stream);
    prof->pend.insert(prof->pend.end(), graph_entries.begin(), graph_entries.end());
  }

  // the Arnoldi steps of one cycle, ending with its last Givens step
  void cycle(int kmax) {
    if constexpr (sizeof(S) == sizeof(T)) {
      if (L.ls) {  // (the parameter check keeps bf16 bases off this path)
        ls_cycle(kmax);
        return;
      }
    }
    for (int j = 0; j < kmax; ++j) iteration(j, kmax);
    prof->tag = kmax - 1;
    prof->early = false;
    norm_givens(kmax - 1, kmax);
    prof->tag = -1;
  }

  void backsolve(int kmax) {
    auto kern = k_backsolve<T>;
    size_t tri = (size_t)kmax * (kmax + 1) / 2 * sizeof(T);
    size_t smem = (size_t)(((kmax + 1) & ~1) + 2) * sizeof(T) + std::min<size_t>(40960, tri);
    prof->launch(GMRESIR_CAT_REFINE, 0.0, kern, dim3(1), dim3(BLOCK), smem, stream, st);
  }

  void init(double rtol, int check_mode, double gamma0) {
    prof->launch(GMRESIR_CAT_REFINE, 0.0, k_init_state, dim3(1), dim3(64), 0, stream, st, rtol, check_mode, gamma0);
  }

  void norm64(const double* v, double* dst) {
    auto kern = k_norm64;
    int g = grid_rows((const void*)kern, n);
    prof->launch(GMRESIR_CAT_REFINE, 8.0 * n, kern, dim3(g), dim3(BLOCK), 0, stream, n, v, (double*)part);
    sqrt_tail(g, dst);
  }

  void sqrt_tail(int producer_grid, double* dst) {
    prof->launch(GMRESIR_CAT_REFINE, 0.0, k_sqrt_tail, dim3(1), dim3(BLOCK), 0, stream, (const double*)part, producer_grid, dst);
  }

  void cycle_tail(int producer_grid) {
    auto kern = k_cycle_tail<T>;
    prof->launch(GMRESIR_CAT_REFINE, 0.0, kern, dim3(1), dim3(BLOCK), 0, stream, (const T*)part, producer_grid, st);
  }

  void resid64(const double* x, const double* b) {
    auto kern = k_resid64;
    int g = grid_spmv_part(A, (const void*)kern, lds_64());
    prof->launch(GMRESIR_CAT_REFINE, 12.0 * A->nnz + 4.0 * (A->n + 1) + 8.0 * n * 3, kern, dim3(g), dim3(BLOCK), lds_64(), stream, A64, x, b, r64, (double*)part);
    sqrt_tail(g, &st.hdr->gamma);
  }

  void cast(const double* r) {
    auto kern = k_cast<T>;
    int g = grid_rows((const void*)kern, n);
    prof->launch(GMRESIR_CAT_REFINE, 8.0 * n + sT() * n * (rhat ? 2 : 1), kern, dim3(g), dim3(BLOCK), 0, stream, n, r, wtmp, rhat, st, part);
    cycle_tail(g);
  }

  void correct_x(double* x, int kmax) {
    auto kern = k_correct_x<T, S>;
    int g = grid_rows((const void*)kern, n);
    prof->launch(GMRESIR_CAT_REFINE, sS() * n * kmax + 16.0 * n, kern, dim3(g), dim3(BLOCK), 0, stream, n, V, L.ldv, st, x);
  }

  void vy(T* out, int kmax) {
    auto kern = k_vy<T, S>;
    int g = grid_rows((const void*)kern, n);
    prof->launch(GMRESIR_CAT_REFINE, sS() * n * kmax + sT() * n, kern, dim3(g), dim3(BLOCK), 0, stream, n, V, L.ldv, st, out);
  }

  void accum(const T* zz, T* uu, int first) {
    auto kern = k_accum<T>;
    int g = grid_rows((const void*)kern, n);
    prof->launch(GMRESIR_CAT_REFINE, sT() * n * (first ? 2 : 3), kern, dim3(g), dim3(BLOCK), 0, stream, n, zz, uu, first);
  }

  void axpy_x(const T* uu, double* x) {
    auto kern = k_axpy_x<T>;
    int g = grid_rows((const void*)kern, n);
    prof->launch(GMRESIR_CAT_REFINE, sT() * n + 16.0 * n, kern, dim3(g), dim3(BLOCK), 0, stream, n, uu, st, x);
  }

  void inner_resid() {
    auto kern = k_inner_resid<T>;
    int g = grid_spmv_part(A, (const void*)kern, lds_in());
    prof->launch(GMRESIR_CAT_REFINE, spmv_bytes() + sT() * n * 3, kern, dim3(g), dim3(BLOCK), lds_in(), stream, Ain, (const T*)u, (const T*)rhat, wtmp, part);
    cycle_tail(g);
  }

  // Copies of the cycle history ride along with the header (one stream
  // synchronisation for both); hist_stage holds the last finished cycle's
  // per-step values after read_hdr(.., true).
  std::vector<double> hist_stage;

  int read_hdr(StateHdr* h, bool with_hist = false) {
    HIP_TRY(hipMemcpyAsync(h, st.hdr, sizeof(StateHdr), hipMemcpyDeviceToHost, stream));
    if (with_hist) {
      hist_stage.resize((size_t)L.m);
      HIP_TRY(hipMemcpyAsync(hist_stage.data(), st.hist, (size_t)L.m * sizeof(double), hipMemcpyDeviceToHost, stream));
    }
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipGetLastError());
    prof->commit(h->cycle_k);
    return 0;
  }
};

// --------------------------------------------------------------------------
// the refinement loop (Algorithm 2; with an fp64 inner solve and one cycle
// per refinement it is restarted GMRES(m), Algorithm 1)
// --------------------------------------------------------------------------

template <typename T, typename S>
int solve_impl(const gmresir_matrix* A, const double* b, double* x, const gmresir_params* p,
               const double* roots, char* ws, const Layout& L, gmresir_result* res, double* hist, int64_t hist_cap,
               hipStream_t stream, int max_refinements = 0, bool allow_graph = true) {
  Prof prof;
  prof.on = p->profile == 1;
  prof.stream = stream;
  Ctx<T, S> c(A, ws, L, stream, &prof);
  c.graph_ok = allow_graph && !prof.on && A->n <= GRAPH_MAX_N;
  if (L.poly) {
    const char* why = "";
    if (!build_poly_program(p->poly_degree + 1, roots, c.prog, &why)) {
      set_error("%s", why);
      return GMRESIR_ERR_INVALID_ARG;
    }
    c.poly_on = true;
    c.poly32 = sizeof(T) == 8 && p->poly_prec == GMRESIR_FP32;
  }
  const int m = p->restart;
  const int cap = p->inner_cap == 0 ? m : p->inner_cap;
  const bool single = cap <= m;
  int64_t hist_n = 0;

  if (L.bj > 0 && (!c.z || !c.py || !c.minv)) {
    set_error("internal: block-Jacobi buffers missing from the workspace layout");
    return GMRESIR_ERR_INVALID_ARG;
  }
  c.init(p->rtol, p->check_mode, 0.0);
  if (L.bj > 0) c.bj_setup();
  c.norm64(b, &c.st.hdr->beta);
  c.resid64(x, b);
  c.cast(c.r64);
  StateHdr H;
  if (int e = c.read_hdr(&H)) return e;
  const double beta = H.beta;
  double gamma = H.gamma;
  int status = GMRESIR_OK;
  if (!isfinite(beta)) {
    set_error("||b|| is not finite");
    status = GMRESIR_ERR_NUMERIC;
  }
  if (status == GMRESIR_OK && beta == 0.0) {
    int g = grid_rows((const void*)k_fill64, c.n);
    hipLaunchKernelGGL(k_fill64, dim3(g), dim3(BLOCK), 0, stream, c.n, x, 0.0);
    HIP_TRY(hipStreamSynchronize(stream));
    res->rel_resid_true = 0.0;
    res->rel_resid_implicit = 0.0;
    return GMRESIR_OK;
  }
  double best = gamma;
  int stall = 0;
  double implicit_rel = gamma / beta;
  while (status == GMRESIR_OK) {
    const double rel = gamma / beta;
    if (!isfinite(rel)) {
      set_error("non-finite residual after %d refinements: ||r|| = %g, ||b|| = %g", res->refinements, gamma, beta);
      status = GMRESIR_ERR_NUMERIC;
      break;
    }
    if (rel <= p->rtol) break;
    if (res->iters >= p->max_iters || (max_refinements > 0 && res->refinements >= max_refinements)) {
      status = GMRESIR_NOT_CONVERGED;
      break;
    }
    const int64_t budget = std::min<int64_t>(cap, p->max_iters - res->iters);
    int64_t used = 0;
    bool numeric = false;
    int first = 1;
    while (used < budget) {
      const int kmax = (int)std::min<int64_t>(m, budget - used);
      c.run_cycle(kmax);
      c.backsolve(kmax);
      if (single && !L.poly && L.bj == 0) {
        c.correct_x(x, kmax);
      } else {
        c.vy(c.z, kmax);
        T* upart = c.z;
        if (L.bj > 0) {
          c.bj_apply(c.z, false, 0, c.py, 0, GMRESIR_CAT_REFINE);
          upart = c.py;
        } else if (L.poly && c.poly32) {
          c.narrow((const double*)c.z, c.s32, 0, GMRESIR_CAT_REFINE);
          c.run_poly32(c.s32, c.y32, 0, GMRESIR_CAT_REFINE);
          c.widen(c.y32, (double*)c.py, 0, GMRESIR_CAT_REFINE);
          upart = c.py;
        } else if (L.poly) {
          c.run_poly(c.z, false, 0, c.py, 0, GMRESIR_CAT_REFINE);
          upart = c.py;
        }
        if (single) c.axpy_x(upart, x);
        else c.accum(upart, c.u, first);
      }
      if (single) {
        used = -1;  // read after the residual
        break;
      }
      if (int e = c.read_hdr(&H, hist && hist_n < hist_cap)) return e;
      res->cycles += 1;
      const int kc = H.cycle_k;
      if (hist && hist_n < hist_cap && kc > 0) {
        int64_t cnt = std::min<int64_t>(kc, hist_cap - hist_n);
        memcpy(hist + hist_n, c.hist_stage.data(), cnt * sizeof(double));
        hist_n += cnt;
      }
      used += kc;
      if (H.cycle_flags & F_NUMERIC) {
        set_error("NaN/Inf in inner cycle %lld: k=%d flags=%d gamma_in=%.3e", (long long)res->cycles, kc,
                  H.cycle_flags, H.gamma_in);
        numeric = true;
        break;
      }
      implicit_rel = H.implicit * gamma / beta;
      if ((H.cycle_flags & (F_STOPPED | F_BREAKDOWN)) || kc == 0 || used >= budget) break;
      c.inner_resid();
      first = 0;
    }
    if (numeric) {
      status = GMRESIR_ERR_NUMERIC;
      break;
    }
    if (!single) c.axpy_x(c.u, x);
    c.resid64(x, b);
    c.cast(c.r64);
    const double gamma_old = gamma;
    if (int e = c.read_hdr(&H, single && hist && hist_n < hist_cap)) return e;
    if (single) {
      res->cycles += 1;
      const int kc = H.cycle_k;
      if (hist && hist_n < hist_cap && kc > 0) {
        int64_t cnt = std::min<int64_t>(kc, hist_cap - hist_n);
        memcpy(hist + hist_n, c.hist_stage.data(), cnt * sizeof(double));
        hist_n += cnt;
      }
      used = kc;
      if (H.cycle_flags & F_NUMERIC) {
        set_error("NaN/Inf in inner cycle %lld (refinement %d): cycle k=%d flags=%d gamma=%.3e gamma_in=%.3e",
                  (long long)res->cycles, res->refinements, kc, H.cycle_flags, gamma_old, H.gamma_in);
        status = GMRESIR_ERR_NUMERIC;
        res->iters += used;
        break;
      }
      implicit_rel = H.implicit * gamma_old / beta;
    }
    res->iters += used;
    res->refinements += 1;
    gamma = H.gamma;
    if (gamma < best) {
      best = gamma;
      stall = 0;
    } else if (++stall >= 3) {
      status = GMRESIR_STAGNATED;
      break;
    }
  }
  res->rel_resid_true = gamma / beta;
  res->rel_resid_implicit = implicit_rel;
  for (int i = 0; i < GMRESIR_NCAT; ++i) {
    res->cat_time_s[i] = prof.t[i];
    res->cat_bytes[i] = prof.bytes[i];
    res->cat_launches[i] = prof.launches[i];
  }
  return status;
}

// fp32 Arnoldi process of `steps` steps from the fp64 vector src (scaled to
// unit norm in fp32); fills the header and the unrotated Hessenberg matrix.
int arnoldi32(const gmresir_matrix* A, const double* src, int steps, char* ws, const Layout& L, hipStream_t stream,
              StateHdr* H, std::vector<double>* hbar, std::vector<double>* hist) {
  Prof prof;
  prof.stream = stream;
  Ctx<float, float> c(A, ws, L, stream, &prof);
  c.init(0.0, 0, 1.0);
  c.cast(src);
  c.cycle(steps);
  // the Hessenberg matrix and the history are copied on the stream before
  // the one synchronisation of read_hdr
  if (hbar) {
    hbar->assign((size_t)(steps + 1) * c.st.ld, 0.0);
    HIP_TRY(hipMemcpyAsync(hbar->data(), c.st.Hbar, (size_t)steps * c.st.ld * sizeof(double), hipMemcpyDeviceToHost,
                           stream));
  }
  if (hist) {
    hist->assign(steps, 0.0);
    HIP_TRY(hipMemcpyAsync(hist->data(), c.st.hist, steps * sizeof(double), hipMemcpyDeviceToHost, stream));
  }
  if (int e = c.read_hdr(H)) return e;
  return 0;
}

Layout arnoldi_layout(int64_t n, int steps, bool poly) {
  gmresir_params q{};
  q.restart = std::max(steps, 1);
  q.inner_cap = 0;
  q.max_iters = 1;
  q.rtol = 1.0;
  q.inner_prec = GMRESIR_FP32;
  q.basis_prec = GMRESIR_FP32;
  q.poly_degree = poly ? 1 : 0;
  return make_layout(n, &q);
}

bool ws_ok(const void* ws, size_t have, size_t need) {
  if (!ws) return set_error("workspace is NULL"), false;
  if (((uintptr_t)ws) % ALIGN) return set_error("workspace must be 256-byte aligned"), false;
  if (have < need) return set_error("workspace has %zu bytes, %zu needed", have, need), false;
  return true;
}

// GMRES-FD (Section "Mixed Precision GMRES-FD"): the two phases are ordinary
// solves.  Phase one is one refinement whose inner solve is fp32 GMRES(m),
// restarted in fp32 for `switch_iters` iterations (its right-hand side is
// b / ||b|| rounded to fp32, its solution is scaled back by ||b|| in fp64);
// phase two is fp64 GMRES(m) from that solution.
bool fd_params(const gmresir_params* p, int64_t switch_iters, gmresir_params* q32, gmresir_params* q64,
               const char** why) {
  if (!valid_params(p, why)) return false;
  if (p->inner_prec != GMRESIR_FP32) return *why = "GMRES-FD needs inner_prec FP32 (its first phase)", false;
  if (p->inner_cap != 0) return *why = "GMRES-FD needs inner_cap 0 (the switch point sets phase one)", false;
  if (p->poly_degree != 0 || p->bj_block != 0) return *why = "GMRES-FD takes no preconditioner", false;
  if (switch_iters < 0 || switch_iters > INT32_MAX) return *why = "switch_iters must be in [0, 2^31)", false;
  *q32 = *p;
  q32->inner_cap = (int32_t)std::max<int64_t>(switch_iters, 1);
  q32->max_iters = std::max<int64_t>(std::min<int64_t>(switch_iters, p->max_iters), 1);
  q32->check_mode = 0;  // phase one runs its full length
  *q64 = *p;
  q64->inner_prec = GMRESIR_FP64;
  q64->basis_prec = GMRESIR_FP64;
  return true;
}

void add_result(gmresir_result* acc, const gmresir_result& r) {
  acc->status = r.status;
  acc->refinements += r.refinements;
  acc->iters += r.iters;
  acc->cycles += r.cycles;
  acc->rel_resid_true = r.rel_resid_true;
  acc->rel_resid_implicit = r.rel_resid_implicit;
  for (int i = 0; i < GMRESIR_NCAT; ++i) {
    acc->cat_time_s[i] += r.cat_time_s[i];
    acc->cat_bytes[i] += r.cat_bytes[i];
    acc->cat_launches[i] += r.cat_launches[i];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// scratch memory of gmresir_solve_noalloc: a file-scope device array; every
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel (in host code it is a
// host-side stand-in): it looks the device address up once per device.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[GMRESIR_NOALLOC_MAX_BYTES];

namespace {

// Device address of the current device's copy of `scratch` (dev must be the
// current device), looked up on the first call per device and kept.
int scratch_ptr(int dev, char** out) {
  static std::mutex mu;
  static std::map<int, char*> addr;
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) {
    *out = it->second;
    return GMRESIR_OK;
  }
  void* ptr = nullptr;
  HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr || ((uintptr_t)ptr) % ALIGN) {
    set_error("scratch array of device %d is not 256-byte aligned", dev);
    return GMRESIR_ERR_HIP;
  }
  addr[dev] = (char*)ptr;
  *out = (char*)ptr;
  return GMRESIR_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int32_t gmresir_abi_version(void) { return 4; }

const char* gmresir_last_error(void) { return gir::last_error(); }

const char* gmresir_status_string(int status) {
  switch (status) {
    case GMRESIR_OK: return "ok";
    case GMRESIR_NOT_CONVERGED: return "not converged (max_iters reached)";
    case GMRESIR_STAGNATED: return "stagnated (residual did not decrease over 3 restarts)";
    case GMRESIR_BREAKDOWN: return "Arnoldi breakdown before the requested number of steps";
    case GMRESIR_ERR_INVALID_ARG: return "invalid argument";
    case GMRESIR_ERR_HIP: return "HIP runtime error";
    case GMRESIR_ERR_WORKSPACE: return "workspace too small or misaligned";
    case GMRESIR_ERR_NUMERIC: return "NaN or Inf encountered";
    case GMRESIR_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

// storage: fp32 CSR values | tile table | SELL slice pointers | SELL columns |
// SELL fp32 values | SELL fp64 values (the SELL part sized for its bound)
size_t gmresir_matrix_storage_bytes(int64_t n, int64_t nnz) {
  if (n < 1 || nnz < 0 || nnz >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31)) return 0;
  const size_t E = (size_t)sell_max_entries(n, nnz);
  const size_t ns = (size_t)((n + SELL_C - 1) / SELL_C);
  return align_up((size_t)nnz * 4) + align_up((size_t)(max_tiles(n, nnz) + 1) * 4) + align_up((ns + 1) * 4) +
         align_up(E * 4) + align_up(E * 4) + align_up(E * 8);
}

int gmresir_matrix_create(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                          void* storage, size_t storage_bytes, void* stream, gmresir_matrix** out) {
  if (!out || !rowptr || (nnz > 0 && (!colidx || !vals)) || !storage) {
    set_error("gmresir_matrix_create: NULL pointer argument");
    return GMRESIR_ERR_INVALID_ARG;
  }
  size_t need = gmresir_matrix_storage_bytes(n, nnz);
  if (need == 0) {
    set_error("gmresir_matrix_create: invalid sizes n=%lld nnz=%lld", (long long)n, (long long)nnz);
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (!ws_ok(storage, storage_bytes, need)) return GMRESIR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> rp(n + 1);
  HIP_TRY(hipMemcpyAsync(rp.data(), rowptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (rp[0] != 0 || rp[n] != nnz) {
    set_error("gmresir_matrix_create: rowptr[0] must be 0 and rowptr[n] == nnz");
    return GMRESIR_ERR_INVALID_ARG;
  }
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) {
      set_error("gmresir_matrix_create: rowptr decreases at row %lld", (long long)i);
      return GMRESIR_ERR_INVALID_ARG;
    }
  // greedy cut into tiles of <= TILE_ROWS rows and <= TILE_NNZ nonzeros
  std::vector<int32_t> tiles;
  tiles.push_back(0);
  int64_t r0 = 0;
  while (r0 < n) {
    int64_t r = r0;
    while (r < n && r - r0 < TILE_ROWS && (int64_t)rp[r + 1] - rp[r0] <= TILE_NNZ) ++r;
    if (r == r0) {
      r = r0 + 1;  // one row longer than a tile
    } else if (r < n && (r & 7) && (r & ~(int64_t)7) > r0) {
      r &= ~(int64_t)7;  // end tiles on a multiple of 8 rows (16-byte loads of 4 fp32 / 8 bf16 basis rows)
    }
    tiles.push_back((int32_t)r);
    r0 = r;
  }
  const int ntiles = (int)tiles.size() - 1;
  int lds_nnz = 1;
  for (int t = 0; t < ntiles; ++t) {
    const int len = rp[tiles[t + 1]] - rp[tiles[t]];
    if (len <= TILE_NNZ) lds_nnz = std::max(lds_nnz, len);
  }
  if (ntiles > max_tiles(n, nnz)) {
    set_error("internal: tile bound exceeded");
    return GMRESIR_ERR_INVALID_ARG;
  }
  char* st = (char*)storage;
  float* v32 = (float*)st;
  int32_t* tr = (int32_t*)(st + align_up((size_t)nnz * 4));
  HIP_TRY(hipMemcpyAsync(tr, tiles.data(), tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (nnz > 0) {
    int g = (int)std::min<int64_t>(4096, (nnz + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_cast_vals, dim3(g), dim3(BLOCK), 0, s, nnz, vals, v32);
    HIP_TRY(hipGetLastError());
  }
  // sliced ELLPACK copy, if compact
  const int64_t ns = (n + SELL_C - 1) / SELL_C;
  std::vector<int32_t> sptr(ns + 1, 0);
  bool sell = nnz > 0;
  for (int64_t sl = 0; sl < ns && sell; ++sl) {
    int64_t K = 0;
    for (int64_t r = sl * SELL_C; r < std::min<int64_t>(n, (sl + 1) * SELL_C); ++r) K = std::max<int64_t>(K, rp[r + 1] - rp[r]);
    if (K > SELL_MAX_ROW) sell = false;
    const int64_t next = (int64_t)sptr[sl] + SELL_C * K;
    if (next > sell_max_entries(n, nnz)) sell = false;
    else sptr[sl + 1] = (int32_t)next;
  }
  const size_t E = (size_t)sell_max_entries(n, nnz);
  // shared offsets: per slice the sorted union of its rows' offsets c - r,
  // taken when every row's columns strictly increase and the slots grow by
  // at most SHARED_MAX_GROWTH over the per-row copy (rows mostly repeat the
  // previous row's offsets, so the union is merged only on a change)
  bool shared = false;
  std::vector<int32_t> sptr3, soff;
  if (sell) {
    // the column indices come to the host in windows of at most SHARED_SCAN_WINDOW
    // entries, 16 MB (a slice's entries, <= 64 * SELL_MAX_ROW, always fit one
    // window; the 27-point 128^3 matrix takes 14 windows)
    constexpr int64_t SHARED_SCAN_WINDOW = (int64_t)1 << 22;
    std::vector<int32_t> ci;
    int64_t w0 = 0, w1 = 0;  // entries [w0, w1) held in ci
    sptr3.assign(ns + 1, 0);
    std::vector<int32_t> U, row, prev, merged;
    bool ok = true;
    for (int64_t sl = 0; sl < ns && ok; ++sl) {
      const int64_t ra = sl * SELL_C, rb = std::min<int64_t>(n, (sl + 1) * SELL_C);
      if (rp[rb] > w1) {
        w0 = rp[ra];
        w1 = std::min<int64_t>(nnz, std::max<int64_t>(w0 + SHARED_SCAN_WINDOW, rp[rb]));
        ci.resize(w1 - w0);
        HIP_TRY(hipMemcpyAsync(ci.data(), colidx + w0, (w1 - w0) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
      }
      U.clear();
      prev.clear();
      for (int64_t r = ra; r < rb && ok; ++r) {
        row.clear();
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
          const int32_t d = ci[p - w0] - (int32_t)r;
          if (!row.empty() && d <= row.back()) {
            ok = false;
            break;
          }
          row.push_back(d);
        }
        if (!ok || row == prev) continue;
        merged.clear();
        std::set_union(U.begin(), U.end(), row.begin(), row.end(), std::back_inserter(merged));
        U.swap(merged);
        prev = row;
      }
      if ((int64_t)U.size() > SELL_MAX_ROW) ok = false;
      if (!ok) break;
      soff.insert(soff.end(), U.begin(), U.end());
      sptr3[sl + 1] = sptr3[sl] + SELL_C * (int32_t)U.size();
    }
    shared = ok && (size_t)sptr3[ns] <= E && (double)sptr3[ns] <= SHARED_MAX_GROWTH * (double)sptr[ns];
  }
  bool wide = false;
  if (shared)
    for (int64_t sl = 0; sl < ns && !wide; ++sl) wide = sptr3[sl + 1] - sptr3[sl] > 9 * SELL_C;
  char* sbase = st + align_up((size_t)nnz * 4) + align_up((size_t)(max_tiles(n, nnz) + 1) * 4);
  int32_t* d_sptr = (int32_t*)sbase;
  int32_t* d_scol = (int32_t*)(sbase + align_up((ns + 1) * 4));
  float* d_sv32 = (float*)((char*)d_scol + align_up(E * 4));
  double* d_sv64 = (double*)((char*)d_sv32 + align_up(E * 4));
  bool d16 = false;
  if (shared) {
    HIP_TRY(hipMemcpyAsync(d_sptr, sptr3.data(), (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_scol, soff.data(), soff.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_build_sell_shared, dim3((unsigned)ns), dim3(SELL_C), 0, s, (int)n, rowptr, colidx, vals,
                       d_sptr, d_scol, d_sv32, d_sv64);
    HIP_TRY(hipGetLastError());
  } else if (sell) {
    // 16-bit column offsets if every entry is within 32767 columns of its row
    // (the check's flag sits in the column region until the copy is built)
    int far = 1;
    HIP_TRY(hipMemsetAsync(d_scol, 0, sizeof(int), s));
    const int gc = (int)std::min<int64_t>(4096, (n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_col_offset_check, dim3(gc), dim3(BLOCK), 0, s, (int)n, rowptr, colidx, (int*)d_scol);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&far, d_scol, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    d16 = far == 0;
    HIP_TRY(hipMemcpyAsync(d_sptr, sptr.data(), (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_build_sell, dim3((unsigned)ns), dim3(SELL_C), 0, s, (int)n, rowptr, colidx, vals, d_sptr,
                       d_scol, (short*)d_scol, d16 ? 1 : 0, d_sv32, d_sv64);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(s));
  gmresir_matrix* A = new gmresir_matrix;
  A->sell = sell;
  A->nslices = (int)ns;
  A->sell_ptr = d_sptr;
  A->sell_col = d_scol;
  A->sell_d16 = d16;
  A->sell_shared = shared;
  A->sell_wide = wide;
  A->sell_v32 = d_sv32;
  A->sell_v64 = d_sv64;
  A->n = n;
  A->nnz = nnz;
  A->rowptr = rowptr;
  A->colidx = colidx;
  A->vals64 = vals;
  A->vals32 = v32;
  A->tile_row = tr;
  A->ntiles = ntiles;
  A->lds_nnz = lds_nnz;
  A->device = 0;
  (void)hipGetDevice(&A->device);
  *out = A;
  return GMRESIR_OK;
}

int gmresir_matrix_destroy(gmresir_matrix* A) {
  delete A;
  return GMRESIR_OK;
}

int64_t gmresir_matrix_n(const gmresir_matrix* A) { return A ? A->n : -1; }
int64_t gmresir_matrix_nnz(const gmresir_matrix* A) { return A ? A->nnz : -1; }
int64_t gmresir_matrix_tiles(const gmresir_matrix* A) { return A ? A->ntiles : -1; }
int32_t gmresir_matrix_layout(const gmresir_matrix* A) {
  return A ? (A->sell ? (A->sell_shared ? 3 : A->sell_d16 ? 2 : 1) : 0) : -1;
}

int gmresir_spmv(const gmresir_matrix* A, int32_t prec, const void* x, void* y, void* stream) {
  if (!A || !x || !y) {
    set_error("gmresir_spmv: NULL argument");
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (x == y) {
    set_error("gmresir_spmv: x and y must not overlap");
    return GMRESIR_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  if (prec == GMRESIR_FP64) {
    auto kern = A->sell_wide ? k_spmv<double, true> : k_spmv<double, false>;
    const size_t smem = A->sell ? 0 : (size_t)A->lds_nnz * sizeof(double);
    int g = grid_spmv(A);
    hipLaunchKernelGGL(kern, dim3(g), dim3(BLOCK), smem, s, csr_of(A, true), (const double*)x, (double*)y);
  } else if (prec == GMRESIR_FP32) {
    auto kern = A->sell_wide ? k_spmv<float, true> : k_spmv<float, false>;
    const size_t smem = A->sell ? 0 : (size_t)A->lds_nnz * sizeof(float);
    int g = grid_spmv(A);
    hipLaunchKernelGGL(kern, dim3(g), dim3(BLOCK), smem, s, csr_of(A, false), (const float*)x, (float*)y);
  } else {
    set_error("gmresir_spmv: prec must be FP64 or FP32");
    return GMRESIR_ERR_INVALID_ARG;
  }
  HIP_TRY(hipGetLastError());
  return GMRESIR_OK;
}

size_t gmresir_workspace_bytes(const gmresir_matrix* A, const gmresir_params* p) {
  const char* why = "";
  if (!A || !valid_params(p, &why)) return 0;
  return make_layout(A->n, p).total;
}

int gmresir_solve(const gmresir_matrix* A, const double* b, double* x, const gmresir_params* p,
                  const double* poly_roots, void* ws, size_t ws_bytes, gmresir_result* res, double* hist,
                  int64_t hist_cap, void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  const char* why = "";
  if (!A || !b || !x || !res) {
    set_error("gmresir_solve: NULL argument");
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (!valid_params(p, &why)) {
    set_error("gmresir_solve: %s", why);
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (p->poly_degree > 0 && !poly_roots) {
    set_error("gmresir_solve: poly_degree > 0 needs poly_roots_host");
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (hist_cap < 0 || (hist_cap > 0 && !hist)) {
    set_error("gmresir_solve: bad history buffer");
    return GMRESIR_ERR_INVALID_ARG;
  }
  Layout L = make_layout(A->n, p);
  if (!ws_ok(ws, ws_bytes, L.total)) return GMRESIR_ERR_WORKSPACE;
  memset(res, 0, sizeof(*res));
  hipStream_t s = (hipStream_t)stream;
  int st;
  if (p->inner_prec == GMRESIR_FP64)
    st = solve_impl<double, double>(A, b, x, p, poly_roots, (char*)ws, L, res, hist, hist_cap, s);
  else if (p->basis_prec == GMRESIR_FP32)
    st = solve_impl<float, float>(A, b, x, p, poly_roots, (char*)ws, L, res, hist, hist_cap, s);
  else
    st = solve_impl<float, bf16_t>(A, b, x, p, poly_roots, (char*)ws, L, res, hist, hist_cap, s);
  res->status = st;
  res->solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

int gmresir_solve_noalloc(const gmresir_matrix* A, const double* b, double* x, const gmresir_params* p,
                          const double* poly_roots, gmresir_result* res, double* hist, int64_t hist_cap,
                          void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  const char* why = "";
  if (!A || !b || !x || !res) {
    set_error("gmresir_solve_noalloc: NULL argument");
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (!valid_params(p, &why)) {
    set_error("gmresir_solve_noalloc: %s", why);
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (p->profile != 0) {
    set_error("gmresir_solve_noalloc: profile must be 0 (per-kernel timing creates HIP events)");
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (p->poly_degree > 0 && !poly_roots) {
    set_error("gmresir_solve_noalloc: poly_degree > 0 needs poly_roots_host");
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (hist_cap < 0 || (hist_cap > 0 && !hist)) {
    set_error("gmresir_solve_noalloc: bad history buffer");
    return GMRESIR_ERR_INVALID_ARG;
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != A->device) {
    set_error("gmresir_solve_noalloc: device %d is current, the matrix lives on device %d", dev, A->device);
    return GMRESIR_ERR_INVALID_ARG;
  }
  const Layout L = make_layout(A->n, p);
  if (L.total > GMRESIR_NOALLOC_MAX_BYTES) {
    set_error("gmresir_solve_noalloc: this solve needs %zu bytes of scratch, the static array holds %zu", L.total,
              (size_t)GMRESIR_NOALLOC_MAX_BYTES);
    return GMRESIR_ERR_WORKSPACE;
  }
  char* ws = nullptr;
  if (int e = scratch_ptr(dev, &ws)) return e;
  memset(res, 0, sizeof(*res));
  hipStream_t s = (hipStream_t)stream;
  int st;
  // direct launches only: recording a HIP graph would allocate
  if (p->inner_prec == GMRESIR_FP64)
    st = solve_impl<double, double>(A, b, x, p, poly_roots, ws, L, res, hist, hist_cap, s, 0, false);
  else if (p->basis_prec == GMRESIR_FP32)
    st = solve_impl<float, float>(A, b, x, p, poly_roots, ws, L, res, hist, hist_cap, s, 0, false);
  else
    st = solve_impl<float, bf16_t>(A, b, x, p, poly_roots, ws, L, res, hist, hist_cap, s, 0, false);
  res->status = st;
  res->solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

size_t gmresir_fd_workspace_bytes(const gmresir_matrix* A, const gmresir_params* p, int64_t switch_iters) {
  const char* why = "";
  gmresir_params q32, q64;
  if (!A || !fd_params(p, switch_iters, &q32, &q64, &why)) return 0;
  return std::max(make_layout(A->n, &q32).total, make_layout(A->n, &q64).total);
}

int gmresir_solve_fd(const gmresir_matrix* A, const double* b, double* x, const gmresir_params* p,
                     int64_t switch_iters, void* ws, size_t ws_bytes, gmresir_result* res, double* hist,
                     int64_t hist_cap, void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  const char* why = "";
  gmresir_params q32, q64;
  if (!A || !b || !x || !res) {
    set_error("gmresir_solve_fd: NULL argument");
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (!fd_params(p, switch_iters, &q32, &q64, &why)) {
    set_error("gmresir_solve_fd: %s", why);
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (hist_cap < 0 || (hist_cap > 0 && !hist)) {
    set_error("gmresir_solve_fd: bad history buffer");
    return GMRESIR_ERR_INVALID_ARG;
  }
  const size_t need = std::max(make_layout(A->n, &q32).total, make_layout(A->n, &q64).total);
  if (!ws_ok(ws, ws_bytes, need)) return GMRESIR_ERR_WORKSPACE;
  memset(res, 0, sizeof(*res));
  hipStream_t s = (hipStream_t)stream;
  int st = GMRESIR_NOT_CONVERGED;
  int64_t hist_used = 0;
  if (switch_iters > 0) {
    gmresir_result r1{};
    const Layout L1 = make_layout(A->n, &q32);
    if (q32.basis_prec == GMRESIR_FP32)
      st = solve_impl<float, float>(A, b, x, &q32, nullptr, (char*)ws, L1, &r1, hist, hist_cap, s, 1);
    else
      st = solve_impl<float, bf16_t>(A, b, x, &q32, nullptr, (char*)ws, L1, &r1, hist, hist_cap, s, 1);
    r1.status = st;
    add_result(res, r1);
    hist_used = std::min<int64_t>(hist_cap, r1.iters);
  }
  // phase two unless phase one converged or failed
  if (st == GMRESIR_NOT_CONVERGED && res->iters < p->max_iters) {
    q64.max_iters = p->max_iters - res->iters;
    gmresir_result r2{};
    const Layout L2 = make_layout(A->n, &q64);
    st = solve_impl<double, double>(A, b, x, &q64, nullptr, (char*)ws, L2, &r2, hist ? hist + hist_used : nullptr,
                                    hist_cap - hist_used, s);
    r2.status = st;
    add_result(res, r2);
  }
  res->status = st;
  res->solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

size_t gmresir_poly_workspace_bytes(const gmresir_matrix* A, int32_t max_degree) {
  if (!A || max_degree < 0 || max_degree > 255) return 0;
  return arnoldi_layout(A->n, std::max(max_degree + 1, 10), true).total;
}

int gmresir_poly_setup(const gmresir_matrix* A, int32_t degree, const double* start, uint64_t seed, void* ws,
                       size_t ws_bytes, double* roots, double* hbar_host, void* stream) {
  if (!A || !roots || degree < 1 || degree > 255) {
    set_error("gmresir_poly_setup: NULL argument or degree outside [1, 255]");
    return GMRESIR_ERR_INVALID_ARG;
  }
  const int steps = degree + 1;
  Layout L = arnoldi_layout(A->n, std::max(steps, 10), true);
  if (!ws_ok(ws, ws_bytes, L.total)) return GMRESIR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const double* src = start;
  if (!src) {
    double* r64 = (double*)((char*)ws + L.r64);
    int g = (int)std::min<int64_t>(4096, (A->n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_start_vector, dim3(g), dim3(BLOCK), 0, s, (int)A->n, seed, r64);
    HIP_TRY(hipGetLastError());
    src = r64;
  }
  StateHdr H;
  std::vector<double> hb;
  if (int e = arnoldi32(A, src, steps, (char*)ws, L, s, &H, &hb, nullptr)) return e;
  if (H.flags & F_NUMERIC) {
    set_error("gmresir_poly_setup: NaN/Inf in the Arnoldi process");
    return GMRESIR_ERR_NUMERIC;
  }
  const int ld = L.m + 1;
  if (hbar_host)
    for (int jj = 0; jj < steps; ++jj)
      for (int i = 0; i < steps + 1; ++i) hbar_host[(size_t)jj * (steps + 1) + i] = hb[(size_t)jj * ld + i];
  if (H.k < steps) {
    set_error("gmresir_poly_setup: Arnoldi breakdown after %d of %d steps", H.k, steps);
    return GMRESIR_BREAKDOWN;
  }
  if (harmonic_ritz_leja(steps, hb.data(), ld, roots) != 0) {
    set_error("gmresir_poly_setup: harmonic Ritz computation failed (singular H or no QR convergence)");
    return GMRESIR_ERR_NUMERIC;
  }
  return GMRESIR_OK;
}

int gmresir_poly_apply(const gmresir_matrix* A, int32_t degree, const double* roots, const float* v, float* y,
                       void* ws, size_t ws_bytes, void* stream) {
  if (!A || !roots || !v || !y || degree < 1 || degree > 255 || (const void*)v == (void*)y) {
    set_error("gmresir_poly_apply: bad arguments");
    return GMRESIR_ERR_INVALID_ARG;
  }
  Layout L = arnoldi_layout(A->n, std::max(degree + 1, 10), true);
  if (!ws_ok(ws, ws_bytes, L.total)) return GMRESIR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Prof prof;
  Ctx<float, float> c(A, (char*)ws, L, s, &prof);
  const char* why = "";
  if (!build_poly_program(degree + 1, roots, c.prog, &why)) {
    set_error("gmresir_poly_apply: %s", why);
    return GMRESIR_ERR_INVALID_ARG;
  }
  c.init(0.0, 0, 1.0);
  c.run_poly((float*)v, false, 0, y, 0, GMRESIR_CAT_POLY);
  HIP_TRY(hipGetLastError());
  return GMRESIR_OK;
}

int gmresir_features(const gmresir_matrix* A, const double* b, void* ws, size_t ws_bytes, float* feat, void* stream) {
  if (!A || !b || !feat) {
    set_error("gmresir_features: NULL argument");
    return GMRESIR_ERR_INVALID_ARG;
  }
  const int steps = 10;
  Layout L = arnoldi_layout(A->n, steps, true);
  if (!ws_ok(ws, ws_bytes, L.total)) return GMRESIR_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  State st = state_of((char*)ws, L);
  // row statistics (the r64 buffer holds the 10 results)
  double* out = (double*)((char*)ws + L.r64);
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, 0.0, 0, 1.0);
  {
    auto kern = k_rowstats;
    int g = grid_rows((const void*)kern, A->n);
    double* part = (double*)((char*)ws + L.part);
    hipLaunchKernelGGL(kern, dim3(g), dim3(BLOCK), 0, s, csr_of(A, true), part);
    hipLaunchKernelGGL(k_rowstats_tail, dim3(1), dim3(BLOCK), 0, s, (const double*)part, g, out);
  }
  HIP_TRY(hipGetLastError());
  double rs[10];
  HIP_TRY(hipMemcpyAsync(rs, out, sizeof(rs), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  StateHdr H;
  std::vector<double> hb, hist;
  if (int e = arnoldi32(A, b, steps, (char*)ws, L, s, &H, &hb, &hist)) return e;
  const double n = (double)A->n;
  const double TINY = 1e-30;
  auto lg = [&](double v) { return log10(std::max(v, TINY)); };
  const double D = rs[9] / n;
  double f[16] = {0};
  f[0] = log10(n);
  f[1] = (double)A->nnz / n;
  f[2] = rs[8];
  f[3] = rs[0] / n;
  f[4] = rs[1];
  f[5] = rs[2] / n;
  f[6] = (rs[3] / n) / std::max(D, TINY);
  f[7] = lg(sqrt(rs[4]) / sqrt(n));
  const double mean = rs[5] / n;
  f[8] = sqrt(std::max(0.0, rs[6] / n - mean * mean)) / std::max(D, TINY);
  f[9] = rs[7] / n;
  const int k = (H.flags & F_NUMERIC) ? 0 : H.k;
  if (k > 0) {
    f[10] = lg(hist[std::min(5, k) - 1]);
    f[11] = lg(hist[k - 1]);
    const int ld = L.m + 1;
    std::vector<double> a((size_t)k * k);
    for (int i = 0; i < k; ++i)
      for (int jj = 0; jj < k; ++jj) a[(size_t)i * k + jj] = (i > jj + 1) ? 0.0 : hb[(size_t)jj * ld + i];
    std::vector<double> wr(k), wi(k);
    if (hessenberg_eigvals(k, a, wr.data(), wi.data()) == 0) {
      double amax = 0, amin = INFINITY, imax = 0, remin = INFINITY;
      for (int i = 0; i < k; ++i) {
        const double mod = hypot(wr[i], wi[i]);
        amax = std::max(amax, mod);
        amin = std::min(amin, mod);
        imax = std::max(imax, fabs(wi[i]));
        remin = std::min(remin, wr[i]);
      }
      f[12] = lg(amax / std::max(amin, TINY));
      f[13] = imax / std::max(amax, TINY);
      f[14] = remin / std::max(amax, TINY);
      f[15] = lg(amax / std::max(D, TINY));
    }
  }
  for (int i = 0; i < 16; ++i) feat[i] = (float)f[i];
  return GMRESIR_OK;
}

int gmresir_host_hessenberg_eigvals(int32_t n, const double* H, int32_t ld, double* wr, double* wi) {
  if (n < 1 || n > 512 || !H || !wr || !wi || ld < n) {
    set_error("gmresir_host_hessenberg_eigvals: bad arguments");
    return GMRESIR_ERR_INVALID_ARG;
  }
  std::vector<double> a((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[(size_t)i * n + j] = (i > j + 1) ? 0.0 : H[(size_t)j * ld + i];
  if (hessenberg_eigvals(n, a, wr, wi) != 0) {
    set_error("gmresir_host_hessenberg_eigvals: QR iteration did not converge");
    return GMRESIR_ERR_NUMERIC;
  }
  return GMRESIR_OK;
}

int gmresir_host_harmonic_ritz_leja(int32_t k, const double* Hbar, int32_t ld, double* roots) {
  if (k < 1 || k > 512 || !Hbar || !roots || ld < k + 1) {
    set_error("gmresir_host_harmonic_ritz_leja: bad arguments");
    return GMRESIR_ERR_INVALID_ARG;
  }
  if (harmonic_ritz_leja(k, Hbar, ld, roots) != 0) {
    set_error("gmresir_host_harmonic_ritz_leja: singular H or no QR convergence");
    return GMRESIR_ERR_NUMERIC;
  }
  return GMRESIR_OK;
}

}  // extern "C"
