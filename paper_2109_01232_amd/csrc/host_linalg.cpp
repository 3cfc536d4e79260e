// Host-side dense helpers of the polynomial preconditioner and the chooser
// features: eigenvalues of a small real upper Hessenberg matrix (Francis
// double-shift QR, Golub & Van Loan "Matrix Computations" Sec. 7.5), harmonic
// Ritz values (the roots of the GMRES residual polynomial) and modified Leja
// ordering of those roots.  Sizes are at most a few hundred, so plain loops.
#include "internal.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <complex>
#include <vector>

namespace gir {

namespace {

// Eigenvalues of the real 2x2 block [[a, b], [c, d]]; complex pairs with the
// positive imaginary part first.
void eig2x2(double a, double b, double c, double d, double* wr, double* wi) {
  double p = 0.5 * (a - d);
  double bc = b * c;
  double disc = p * p + bc;
  if (disc >= 0.0) {
    double mu = p + std::copysign(std::sqrt(disc), p);
    wr[0] = d + mu;
    wr[1] = (mu != 0.0) ? d - bc / mu : d;
    wi[0] = wi[1] = 0.0;
  } else {
    double re = d + p;
    double im = std::sqrt(-disc);
    wr[0] = wr[1] = re;
    wi[0] = im;
    wi[1] = -im;
  }
}

// Householder vector v (v[0] implicit scaling) with (I - beta v v^T) x = alpha e1.
int house(int len, const double* x, double* v, double* beta) {
  double nrm2 = 0.0;
  for (int i = 0; i < len; ++i) nrm2 += x[i] * x[i];
  double nrm = std::sqrt(nrm2);
  if (nrm == 0.0) {
    *beta = 0.0;
    for (int i = 0; i < len; ++i) v[i] = 0.0;
    return 0;
  }
  double alpha = (x[0] >= 0.0) ? -nrm : nrm;
  v[0] = x[0] - alpha;
  for (int i = 1; i < len; ++i) v[i] = x[i];
  double vv = 0.0;
  for (int i = 0; i < len; ++i) vv += v[i] * v[i];
  *beta = (vv > 0.0) ? 2.0 / vv : 0.0;
  return 0;
}

}  // namespace

// a: n x n row-major working copy (destroyed).
int hessenberg_eigvals(int n, std::vector<double>& a, double* wr, double* wi) {
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  double anorm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = std::max(0, i - 1); j < n; ++j) anorm = std::max(anorm, std::fabs(A(i, j)));
  int hi = n - 1;
  int iter = 0;
  while (hi >= 0) {
    // locate the start l of the unreduced active block ending at hi
    int l = hi;
    while (l > 0) {
      double s = std::fabs(A(l - 1, l - 1)) + std::fabs(A(l, l));
      if (s == 0.0) s = anorm;
      if (std::fabs(A(l, l - 1)) <= DBL_EPSILON * s) {
        A(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {
      wr[hi] = A(hi, hi);
      wi[hi] = 0.0;
      hi -= 1;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {
      eig2x2(A(hi - 1, hi - 1), A(hi - 1, hi), A(hi, hi - 1), A(hi, hi), wr + hi - 1, wi + hi - 1);
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++iter > 100) return -1;
    // double shift: trace s and determinant t of the trailing 2x2 block
    double s, t;
    if (iter % 10 == 0) {
      double w = std::fabs(A(hi, hi - 1)) + std::fabs(A(hi - 1, hi - 2));
      s = 1.5 * w;
      t = -0.4375 * w * w;
    } else {
      s = A(hi - 1, hi - 1) + A(hi, hi);
      t = A(hi - 1, hi - 1) * A(hi, hi) - A(hi - 1, hi) * A(hi, hi - 1);
    }
    // first column of (H - s1 I)(H - s2 I) restricted to the active block
    double xyz[3];
    xyz[0] = A(l, l) * A(l, l) + A(l, l + 1) * A(l + 1, l) - s * A(l, l) + t;
    xyz[1] = A(l + 1, l) * (A(l, l) + A(l + 1, l + 1) - s);
    xyz[2] = A(l + 1, l) * A(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      double v[3], beta;
      house(3, xyz, v, &beta);
      if (beta != 0.0) {
        int c0 = std::max(l, k - 1);
        for (int j = c0; j <= hi; ++j) {
          double d = v[0] * A(k, j) + v[1] * A(k + 1, j) + v[2] * A(k + 2, j);
          d *= beta;
          A(k, j) -= d * v[0];
          A(k + 1, j) -= d * v[1];
          A(k + 2, j) -= d * v[2];
        }
        int r1 = std::min(k + 3, hi);
        for (int i = l; i <= r1; ++i) {
          double d = A(i, k) * v[0] + A(i, k + 1) * v[1] + A(i, k + 2) * v[2];
          d *= beta;
          A(i, k) -= d * v[0];
          A(i, k + 1) -= d * v[1];
          A(i, k + 2) -= d * v[2];
        }
      }
      xyz[0] = A(k + 1, k);
      xyz[1] = A(k + 2, k);
      if (k < hi - 2) xyz[2] = A(k + 3, k);
    }
    {
      double v[2], beta;
      house(2, xyz, v, &beta);
      if (beta != 0.0) {
        for (int j = hi - 2; j <= hi; ++j) {
          double d = beta * (v[0] * A(hi - 1, j) + v[1] * A(hi, j));
          A(hi - 1, j) -= d * v[0];
          A(hi, j) -= d * v[1];
        }
        for (int i = l; i <= hi; ++i) {
          double d = beta * (A(i, hi - 1) * v[0] + A(i, hi) * v[1]);
          A(i, hi - 1) -= d * v[0];
          A(i, hi) -= d * v[1];
        }
      }
    }
  }
  return 0;
}

// Solve M^T f = e_last for a k x k matrix M (row-major) by Gaussian elimination
// with partial pivoting.  Returns -1 if M is singular.
static int solve_transposed_last(int k, const std::vector<double>& M, std::vector<double>& f) {
  std::vector<double> T((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) T[(size_t)i * k + j] = M[(size_t)j * k + i];  // T = M^T
  f.assign(k, 0.0);
  f[k - 1] = 1.0;
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(T[(size_t)r * k + c]) > std::fabs(T[(size_t)piv * k + c])) piv = r;
    if (T[(size_t)piv * k + c] == 0.0) return -1;
    if (piv != c) {
      for (int j = 0; j < k; ++j) std::swap(T[(size_t)c * k + j], T[(size_t)piv * k + j]);
      std::swap(f[c], f[piv]);
    }
    for (int r = c + 1; r < k; ++r) {
      double m = T[(size_t)r * k + c] / T[(size_t)c * k + c];
      if (m == 0.0) continue;
      for (int j = c; j < k; ++j) T[(size_t)r * k + j] -= m * T[(size_t)c * k + j];
      f[r] -= m * f[c];
    }
  }
  for (int i = k - 1; i >= 0; --i) {
    double s = f[i];
    for (int j = i + 1; j < k; ++j) s -= T[(size_t)i * k + j] * f[j];
    f[i] = s / T[(size_t)i * k + i];
  }
  return 0;
}

void leja_order(int k, const double* wr, const double* wi, double* out) {
  std::vector<std::complex<double>> rest(k), chosen;
  for (int i = 0; i < k; ++i) rest[i] = {wr[i], wi[i]};
  while (!rest.empty()) {
    size_t pick = 0;
    if (chosen.empty()) {
      for (size_t i = 1; i < rest.size(); ++i)
        if (std::abs(rest[i]) > std::abs(rest[pick])) pick = i;
    } else {
      double best = -INFINITY;
      bool first = true;
      for (size_t i = 0; i < rest.size(); ++i) {
        double sc = 0.0;
        for (auto& c : chosen) {
          double d = std::abs(rest[i] - c);
          if (d == 0.0) {
            sc = -INFINITY;
            break;
          }
          sc += std::log(d);
        }
        if (first || sc > best) {
          best = sc;
          pick = i;
          first = false;
        }
      }
    }
    std::complex<double> t = rest[pick];
    rest.erase(rest.begin() + pick);
    if (t.imag() != 0.0) {
      size_t j = 0;
      for (size_t i = 1; i < rest.size(); ++i)
        if (std::abs(rest[i] - std::conj(t)) < std::abs(rest[j] - std::conj(t))) j = i;
      if (!rest.empty()) rest.erase(rest.begin() + j);
      std::complex<double> hi = (t.imag() > 0.0) ? t : std::conj(t);
      chosen.push_back(hi);
      chosen.push_back(std::conj(hi));
    } else {
      chosen.push_back(t);
    }
  }
  for (size_t i = 0; i < chosen.size(); ++i) {
    out[2 * i] = chosen[i].real();
    out[2 * i + 1] = chosen[i].imag();
  }
}

// Hbar: (k+1) x k column-major with leading dimension ld.
int harmonic_ritz_leja(int k, const double* Hbar, int ld, double* roots) {
  std::vector<double> H((size_t)k * k);  // row-major square top; entries below the subdiagonal are 0
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) H[(size_t)i * k + j] = (i > j + 1) ? 0.0 : Hbar[(size_t)j * ld + i];
  double hk = Hbar[(size_t)(k - 1) * ld + k];
  std::vector<double> f;
  if (solve_transposed_last(k, H, f) != 0) return -1;
  for (int i = 0; i < k; ++i) H[(size_t)i * k + (k - 1)] += hk * hk * f[i];
  std::vector<double> wr(k), wi(k);
  if (hessenberg_eigvals(k, H, wr.data(), wi.data()) != 0) return -1;
  leja_order(k, wr.data(), wi.data(), roots);
  return 0;
}

}  // namespace gir
