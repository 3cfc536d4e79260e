// Declarations shared by the translation units of libgmresir (not installed).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace gir {

// host_linalg.cpp
int hessenberg_eigvals(int n, std::vector<double>& a_rowmajor, double* wr, double* wi);
void leja_order(int k, const double* wr, const double* wi, double* out_re_im);
int harmonic_ritz_leja(int k, const double* Hbar_colmajor, int ld, double* roots_re_im);

// errors.cpp
void set_error(const char* fmt, ...);
const char* last_error();

// Row tiles of the SpMV kernels: at most this many rows / nonzeros per tile
// (2560 nonzeros: 512 rows of a 5-point stencil, ~95 rows of a 27-point one;
// the LDS product buffer then allows 8 blocks per CU).
constexpr int TILE_ROWS = 512;
constexpr int TILE_NNZ = 2560;
constexpr int SPMV_UNROLL = 5;  // nonzeros per thread whose loads are issued together

// Sliced ELLPACK copy of the matrix used by the SpMV kernels when it stays
// compact: slices of SELL_C = 64 rows (one wave, one row per lane), entry k
// of row 64 s + l at sell_ptr[s] + 64 k + l; padding entries point at the row
// itself with value 0 and are skipped by the row length.  Built when no row
// is longer than SELL_MAX_ROW and the padded size fits sell_max_entries;
// otherwise the row-tiled CSR kernels run.  When the rows of each slice share
// their column offsets (stencils: the union of a slice's offsets is hardly
// wider than its longest row), slot k of slice s holds offset
// sell_col[sell_ptr[s] / 64 + k] for all 64 rows, absent entries value 0: no
// column index and no row length is read per entry (SHARED_MAX_GROWTH bounds
// the extra slots against the per-row copy).
constexpr int SELL_C = 64;
constexpr int SELL_MAX_ROW = 512;
inline int64_t sell_max_entries(int64_t n, int64_t nnz) { return nnz + nnz / 4 + (n < 4096 ? n : 4096) * 4; }
constexpr double SHARED_MAX_GROWTH = 1.25;

// Upper bound of the number of tiles (every tile holds at least one row).
inline int64_t max_tiles(int64_t n, int64_t nnz) {
  (void)nnz;
  return n;
}

}  // namespace gir
