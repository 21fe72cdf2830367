// Host dense real Schur decomposition and reordering for the Krylov-Schur
// restart (Stewart's method, used in Sec. 6.1 of arXiv 2104.01253).
//
// Written from the textbook algorithms:
//   * Householder reduction to upper Hessenberg form and the implicit Francis
//     double-shift QR step with bulge chasing (Golub & Van Loan, "Matrix
//     Computations", Alg. 7.4.2 / 7.5.1), with the ad hoc exceptional shift of
//     the EISPACK hqr routine after 10 and 20 stagnant iterations;
//   * standardisation of 2x2 diagonal blocks (real eigenvalues -> triangular,
//     complex pair -> equal diagonal entries) by a rotation found from the
//     double-angle form of 2x2 similarity (derived at std2x2);
//   * swapping adjacent diagonal blocks through the Sylvester equation
//     T11 X - X T22 = T12 and a QR factorisation of [-X; I] (Bai & Demmel, 1993).
// The matrices are tiny (p <= DCGS2_MAX_N), so clarity wins over blocking.
#include "schur.h"
#include "std2x2.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace dcgs2 {
namespace {

constexpr double EPS = 2.220446049250313e-16;

struct Mat {
  double* a;
  int ld;
  double& operator()(int i, int j) const { return a[(size_t)j * ld + i]; }
};

// Householder vector for x[0..n): returns tau with (I - tau v v^T) x = mu e_1,
// v[0] = 1.  tau = 0 when x[1..n) is already zero.
double make_house(const double* x, int n, double* v) {
  double sigma = 0.0;
  for (int i = 1; i < n; ++i) sigma += x[i] * x[i];
  v[0] = 1.0;
  for (int i = 1; i < n; ++i) v[i] = x[i];
  if (sigma == 0.0) return 0.0;
  const double mu = std::sqrt(x[0] * x[0] + sigma);
  const double v0 = (x[0] <= 0.0) ? x[0] - mu : -sigma / (x[0] + mu);
  const double tau = 2.0 * v0 * v0 / (sigma + v0 * v0);
  for (int i = 1; i < n; ++i) v[i] /= v0;
  return tau;
}

// rows r0..r0+n-1, columns c0..c1:  A <- (I - tau v v^T) A
void house_left(const Mat& A, const double* v, int n, double tau, int r0, int c0, int c1) {
  for (int j = c0; j <= c1; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += v[i] * A(r0 + i, j);
    s *= tau;
    for (int i = 0; i < n; ++i) A(r0 + i, j) -= s * v[i];
  }
}

// columns c0..c0+n-1, rows r0..r1:  A <- A (I - tau v v^T)
void house_right(const Mat& A, const double* v, int n, double tau, int c0, int r0, int r1) {
  for (int i = r0; i <= r1; ++i) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += A(i, c0 + k) * v[k];
    s *= tau;
    for (int k = 0; k < n; ++k) A(i, c0 + k) -= s * v[k];
  }
}

// Plane rotation G = [cs -sn; sn cs]:  rows (i, i+1) <- G^T rows, columns c0..c1.
void rot_rows(const Mat& A, int i, int c0, int c1, double cs, double sn) {
  for (int j = c0; j <= c1; ++j) {
    const double x = A(i, j), y = A(i + 1, j);
    A(i, j) = cs * x + sn * y;
    A(i + 1, j) = -sn * x + cs * y;
  }
}

// columns (i, i+1) <- columns G, rows r0..r1.
void rot_cols(const Mat& A, int i, int r0, int r1, double cs, double sn) {
  for (int r = r0; r <= r1; ++r) {
    const double x = A(r, i), y = A(r, i + 1);
    A(r, i) = cs * x + sn * y;
    A(r, i + 1) = -sn * x + cs * y;
  }
}

// Standardise the 2x2 block at (i, i) of the full p x p Schur form and Z.
void standardize_block(int p, const Mat& T, const Mat& Z, int i) {
  double a = T(i, i), b = T(i, i + 1), c = T(i + 1, i), d = T(i + 1, i + 1), cs, sn;
  std2x2(a, b, c, d, cs, sn);
  if (i + 2 <= p - 1) rot_rows(T, i, i + 2, p - 1, cs, sn);
  if (i >= 1) rot_cols(T, i, 0, i - 1, cs, sn);
  rot_cols(Z, i, 0, p - 1, cs, sn);
  T(i, i) = a; T(i, i + 1) = b; T(i + 1, i) = c; T(i + 1, i + 1) = d;
}

int block_size(const Mat& T, int p, int i) { return (i + 1 < p && T(i + 1, i) != 0.0) ? 2 : 1; }

double block_mag(const Mat& T, int i, int sz) {
  if (sz == 1) return std::fabs(T(i, i));
  // standard complex block: eigenvalues a +- i sqrt(|b c|)
  return std::sqrt(T(i, i) * T(i, i) + std::fabs(T(i, i + 1) * T(i + 1, i)));
}

// Gaussian elimination with partial pivoting for N <= 4.
bool small_solve(int N, double* M, double* rhs) {
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int i = k + 1; i < N; ++i)
      if (std::fabs(M[k * N + i]) > std::fabs(M[k * N + piv])) piv = i;
    if (M[k * N + piv] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < N; ++j) std::swap(M[j * N + k], M[j * N + piv]);
      std::swap(rhs[k], rhs[piv]);
    }
    for (int i = k + 1; i < N; ++i) {
      const double f = M[k * N + i] / M[k * N + k];
      for (int j = k; j < N; ++j) M[j * N + i] -= f * M[j * N + k];
      rhs[i] -= f * rhs[k];
    }
  }
  for (int i = N - 1; i >= 0; --i) {
    double s = rhs[i];
    for (int j = i + 1; j < N; ++j) s -= M[j * N + i] * rhs[j];
    rhs[i] = s / M[i * N + i];
  }
  return true;
}

// Swap the adjacent diagonal blocks T11 (n1 x n1 at j) and T22 (n2 x n2 at j+n1).
int swap_blocks(int p, const Mat& T, const Mat& Z, int j, int n1, int n2) {
  if (n1 == 1 && n2 == 1) {
    const double t11 = T(j, j), t22 = T(j + 1, j + 1), t12 = T(j, j + 1);
    const double f = t12, g = t22 - t11;
    const double r = std::hypot(f, g);
    if (r == 0.0) return 0;
    const double cs = f / r, sn = g / r;   // first column: eigenvector of t22
    rot_rows(T, j, j, p - 1, cs, sn);
    rot_cols(T, j, 0, j + 1, cs, sn);
    rot_cols(Z, j, 0, p - 1, cs, sn);
    T(j, j) = t22;
    T(j + 1, j + 1) = t11;
    T(j + 1, j) = 0.0;
    return 0;
  }
  const int n = n1 + n2;
  // Sylvester equation T11 X - X T22 = T12, X is n1 x n2, unknowns vec(X)
  const int N = n1 * n2;
  double M[16] = {0}, x[4];
  for (int jj = 0; jj < n2; ++jj)
    for (int ii = 0; ii < n1; ++ii) {
      const int row = ii + jj * n1;
      for (int k = 0; k < n1; ++k) M[(k + jj * n1) * N + row] += T(j + ii, j + k);
      for (int k = 0; k < n2; ++k) M[(ii + k * n1) * N + row] -= T(j + n1 + k, j + n1 + jj);
      x[row] = T(j + ii, j + n1 + jj);
    }
  if (!small_solve(N, M, x)) return 1;
  // QR of [-X; I_{n2}] (n x n2) by Householder reflectors; Qh = H_0 ... H_{n2-1}
  double W[16] = {0};
  for (int jj = 0; jj < n2; ++jj) {
    for (int ii = 0; ii < n1; ++ii) W[jj * n + ii] = -x[ii + jj * n1];
    W[jj * n + n1 + jj] = 1.0;
  }
  double Qh[16] = {0};
  for (int i = 0; i < n; ++i) Qh[i * n + i] = 1.0;
  for (int c = 0; c < n2; ++c) {
    double v[4], col[4];
    const int len = n - c;
    for (int i = 0; i < len; ++i) col[i] = W[c * n + c + i];
    const double tau = make_house(col, len, v);
    if (tau == 0.0) continue;
    const Mat Wm{W, n}, Qm{Qh, n};
    house_left(Wm, v, len, tau, c, c, n2 - 1);
    house_right(Qm, v, len, tau, c, 0, n - 1);
  }
  // T <- Qh^T T Qh on the affected rows/columns, Z <- Z Qh
  std::vector<double> buf((size_t)std::max(p, 1) * n);
  for (int col = j; col < p; ++col) {                 // rows j..j+n-1
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += Qh[i * n + k] * T(j + k, col);
      buf[(size_t)col * n + i] = s;
    }
  }
  for (int col = j; col < p; ++col)
    for (int i = 0; i < n; ++i) T(j + i, col) = buf[(size_t)col * n + i];
  auto right = [&](const Mat& A, int r1) {
    for (int r = 0; r <= r1; ++r) {
      double tmp[4];
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += A(r, j + k) * Qh[i * n + k];
        tmp[i] = s;
      }
      for (int i = 0; i < n; ++i) A(r, j + i) = tmp[i];
    }
  };
  right(T, j + n - 1);
  right(Z, p - 1);
  for (int cc = 0; cc < n2; ++cc)
    for (int rr = n2; rr < n; ++rr) T(j + rr, j + cc) = 0.0;
  if (n2 == 2) standardize_block(p, T, Z, j);
  else T(j + 1, j) = 0.0;
  if (n1 == 2) standardize_block(p, T, Z, j + n2);
  return 0;
}

}  // namespace

int real_schur(int p, double* Ap, int lda, double* Zp, int ldz) {
  const Mat A{Ap, lda}, Z{Zp, ldz};
  for (int j = 0; j < p; ++j)
    for (int i = 0; i < p; ++i) Z(i, j) = (i == j) ? 1.0 : 0.0;
  if (p <= 1) return 0;
  std::vector<double> x(p), v(p);
  // Hessenberg reduction
  for (int k = 0; k + 2 < p; ++k) {
    const int n = p - k - 1;
    for (int i = 0; i < n; ++i) x[i] = A(k + 1 + i, k);
    const double tau = make_house(x.data(), n, v.data());
    if (tau != 0.0) {
      house_left(A, v.data(), n, tau, k + 1, k, p - 1);
      house_right(A, v.data(), n, tau, k + 1, 0, p - 1);
      house_right(Z, v.data(), n, tau, k + 1, 0, p - 1);
    }
    for (int i = k + 2; i < p; ++i) A(i, k) = 0.0;
  }
  double anorm = 0.0;
  for (int j = 0; j < p; ++j)
    for (int i = 0; i <= std::min(j + 1, p - 1); ++i) anorm = std::max(anorm, std::fabs(A(i, j)));
  // Francis double-shift QR iteration on the active window [l, hi]
  int hi = p - 1, its = 0, total = 0;
  const int max_total = 60 * p + 100;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = std::fabs(A(l - 1, l - 1)) + std::fabs(A(l, l));
      if (s == 0.0) s = anorm;
      if (std::fabs(A(l, l - 1)) <= EPS * s) {
        A(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) { hi -= 1; its = 0; continue; }
    if (l == hi - 1) {
      standardize_block(p, A, Z, hi - 1);
      hi -= 2;
      its = 0;
      continue;
    }
    if (++total > max_total) return 1;
    ++its;
    double s, t;
    if (its == 10 || its == 20) {
      const double ex = std::fabs(A(hi, hi - 1)) + std::fabs(A(hi - 1, hi - 2));
      s = 1.5 * ex;
      t = ex * ex;
    } else {
      s = A(hi - 1, hi - 1) + A(hi, hi);
      t = A(hi - 1, hi - 1) * A(hi, hi) - A(hi - 1, hi) * A(hi, hi - 1);
    }
    double xx = A(l, l) * A(l, l) + A(l, l + 1) * A(l + 1, l) - s * A(l, l) + t;
    double yy = A(l + 1, l) * (A(l, l) + A(l + 1, l + 1) - s);
    double zz = A(l + 1, l) * A(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      const double xv[3] = {xx, yy, zz};
      double hv[3];
      const double tau = make_house(xv, 3, hv);
      if (tau != 0.0) {
        house_left(A, hv, 3, tau, k, std::max(l, k - 1), p - 1);
        house_right(A, hv, 3, tau, k, 0, std::min(k + 3, hi));
        house_right(Z, hv, 3, tau, k, 0, p - 1);
      }
      if (k > l) { A(k + 1, k - 1) = 0.0; A(k + 2, k - 1) = 0.0; }
      xx = A(k + 1, k);
      yy = A(k + 2, k);
      if (k < hi - 2) zz = A(k + 3, k);
    }
    const double xv[2] = {xx, yy};
    double hv[2];
    const double tau = make_house(xv, 2, hv);
    if (tau != 0.0) {
      house_left(A, hv, 2, tau, hi - 1, hi - 2, p - 1);
      house_right(A, hv, 2, tau, hi - 1, 0, hi);
      house_right(Z, hv, 2, tau, hi - 1, 0, p - 1);
    }
    A(hi, hi - 2) = 0.0;
  }
  return 0;
}

void schur_eigenvalues(int p, const double* Tp, int ldt, double* re, double* im) {
  const Mat T{const_cast<double*>(Tp), ldt};
  for (int i = 0; i < p;) {
    if (block_size(T, p, i) == 2) {
      const double a = 0.5 * (T(i, i) + T(i + 1, i + 1));
      const double w = std::sqrt(std::fabs(T(i, i + 1))) * std::sqrt(std::fabs(T(i + 1, i)));
      re[i] = a; im[i] = w;
      re[i + 1] = a; im[i + 1] = -w;
      i += 2;
    } else {
      re[i] = T(i, i); im[i] = 0.0;
      i += 1;
    }
  }
}

int reorder_schur_by_magnitude(int p, double* Tp, int ldt, double* Zp, int ldz, int count,
                               double cut_gap) {
  const Mat T{Tp, ldt}, Z{Zp, ldz};
  if (count >= p) count = p;
  std::vector<double> re(p), im(p), mags(p);
  schur_eigenvalues(p, Tp, ldt, re.data(), im.data());
  for (int i = 0; i < p; ++i) mags[i] = std::hypot(re[i], im[i]);
  std::sort(mags.begin(), mags.end(), [](double a, double b) { return a > b; });
  int cnt = std::max(count, 1);
  while (cnt < p && mags[cnt - 1] - mags[cnt] <= cut_gap * mags[0]) ++cnt;
  int filled = 0, guard = 0;
  while (filled < cnt) {
    if (++guard > 4 * p + 4) return -1;
    int best = -1;
    double bmag = -1.0;
    for (int i = filled; i < p;) {
      const int sz = block_size(T, p, i);
      const double mg = block_mag(T, i, sz);
      if (mg > bmag) { bmag = mg; best = i; }
      i += sz;
    }
    int pos = best;
    while (pos > filled) {
      int i = filled, prev = filled;
      while (i < pos) { prev = i; i += block_size(T, p, i); }
      if (i != pos) return -1;
      const int above = pos - prev;
      const int cur = block_size(T, p, pos);
      if (swap_blocks(p, T, Z, prev, above, cur) != 0) return -1;
      pos = prev;
    }
    filled += block_size(T, p, filled);
  }
  return filled;
}

}  // namespace dcgs2
