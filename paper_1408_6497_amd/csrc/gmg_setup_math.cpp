// Host-side setup arithmetic: LGL basis and quadrature (Section 2.3.2), the
// banded 1D operator rows and element matrices used by the apply kernel, the
// Jacobi diagonal by node class (Section 2.3, Setup), transfer taps from
// P(i, j) = phi_j^{coarse}(p_i) (eq. 2.2), the dense coarsest pseudo-inverse,
// the SplitMix64 stream of the Lanczos start vectors, and the largest
// eigenvalue of a symmetric tridiagonal matrix (Sturm bisection).
#include "gmg_setup_math.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

namespace gmg {

namespace {

// Legendre P_m(x) and P_m'(x) by the three-term recurrence.
void legendre(int m, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x;
  if (m == 0) {
    *p = 1.0;
    *dp = 0.0;
    return;
  }
  for (int k = 2; k <= m; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  // (1 - x^2) P_m' = m (P_{m-1} - x P_m)
  *dp = (std::fabs(1.0 - x * x) > 0.0) ? m * (p0 - x * p1) / (1.0 - x * x) : 0.0;
}

}  // namespace

std::vector<double> lgl_nodes01(int q) {
  // interior nodes: roots of P_q'(x); Newton on P_q' with the identity
  // (1 - x^2) P_q'' = 2 x P_q' - q (q+1) P_q.
  std::vector<double> x(q + 1);
  x[0] = -1.0;
  x[q] = 1.0;
  for (int j = 1; j < q; ++j) {
    double t = -std::cos(M_PI * j / q);  // Chebyshev-Gauss-Lobatto start, increasing
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(q, t, &p, &dp);
      const double d2p = (2.0 * t * dp - q * (q + 1.0) * p) / (1.0 - t * t);
      const double step = dp / d2p;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[j] = t;
  }
  for (auto& v : x) v = 0.5 * (v + 1.0);
  return x;
}

void gauss01(int m, std::vector<double>* pts, std::vector<double>* wts) {
  pts->assign(m, 0.0);
  wts->assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    double p = 0.0, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre(m, t, &p, &dp);
      const double step = p / dp;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    legendre(m, t, &p, &dp);
    (*pts)[m - 1 - i] = 0.5 * (t + 1.0);
    (*wts)[m - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2/((1-t^2)P'^2), halved for [0,1]
  }
}

double lagrange_at(const std::vector<double>& xi, int a, double t) {
  double v = 1.0;
  for (size_t b = 0; b < xi.size(); ++b)
    if (static_cast<int>(b) != a) v *= (t - xi[b]) / (xi[a] - xi[b]);
  return v;
}

double lagrange_deriv_at(const std::vector<double>& xi, int a, double t) {
  double s = 0.0;
  for (size_t k = 0; k < xi.size(); ++k) {
    if (static_cast<int>(k) == a) continue;
    double term = 1.0 / (xi[a] - xi[k]);
    for (size_t b = 0; b < xi.size(); ++b)
      if (static_cast<int>(b) != a && b != k) term *= (t - xi[b]) / (xi[a] - xi[b]);
    s += term;
  }
  return s;
}

void reference_matrices(int q, std::vector<double>* khat, std::vector<double>* mhat) {
  const std::vector<double> xi = lgl_nodes01(q);
  std::vector<double> t, w;
  gauss01(q + 1, &t, &w);
  khat->assign((q + 1) * (q + 1), 0.0);
  mhat->assign((q + 1) * (q + 1), 0.0);
  for (int a = 0; a <= q; ++a)
    for (int b = 0; b <= q; ++b) {
      double ks = 0.0, ms = 0.0;
      for (int p = 0; p <= q; ++p) {
        ks += w[p] * lagrange_deriv_at(xi, a, t[p]) * lagrange_deriv_at(xi, b, t[p]);
        ms += w[p] * lagrange_at(xi, a, t[p]) * lagrange_at(xi, b, t[p]);
      }
      (*khat)[a * (q + 1) + b] = ks;
      (*mhat)[a * (q + 1) + b] = ms;
    }
}

// Rows of the assembled periodic 1D matrices for node class c (offsets -q..q).
// A vertex (c = 0) is local node q of the element on its left and local node 0
// of the element on its right; an interior node c belongs to one element.
static void assembled_rows(int q, const std::vector<double>& ehat, double scale, double rows[][2 * kMaxQ + 1]) {
  for (int c = 0; c < q; ++c)
    for (int o = 0; o < 2 * kMaxQ + 1; ++o) rows[c][o] = 0.0;
  for (int b = 0; b <= q; ++b) {
    rows[0][(b - q) + q] += ehat[q * (q + 1) + b] * scale;  // left element
    rows[0][b + q] += ehat[0 * (q + 1) + b] * scale;        // right element
  }
  for (int c = 1; c < q; ++c)
    for (int b = 0; b <= q; ++b) rows[c][(b - c) + q] = ehat[c * (q + 1) + b] * scale;
}

LevelTables make_level_tables(int q, int n) {
  LevelTables L{};
  const double h = 1.0 / n;
  std::vector<double> khat, mhat;
  reference_matrices(q, &khat, &mhat);
  OpTab& A = L.stiff;
  A.q = q;
  assembled_rows(q, khat, 1.0 / h, A.krow);
  assembled_rows(q, mhat, h, A.mrow);
  assembled_rows(q, khat, 1.0 / h, A.zkrow);
  assembled_rows(q, mhat, h, A.zmrow);
  for (int a = 0; a <= q; ++a)
    for (int b = 0; b <= q; ++b) {
      A.zk[a][b] = khat[a * (q + 1) + b] / h;
      A.zm[a][b] = mhat[a * (q + 1) + b] * h;
    }
  double kd[kMaxQ], md[kMaxQ], msum[kMaxQ];
  for (int c = 0; c < q; ++c) {
    kd[c] = A.krow[c][q];
    md[c] = A.mrow[c][q];
    msum[c] = 0.0;
    for (int o = 0; o < 2 * q + 1; ++o) msum[c] += A.mrow[c][o];
  }
  for (int cz = 0; cz < q; ++cz)
    for (int cy = 0; cy < q; ++cy)
      for (int cx = 0; cx < q; ++cx) {
        const int i = cx + q * (cy + q * cz);
        const double d = kd[cx] * md[cy] * md[cz] + md[cx] * kd[cy] * md[cz] + md[cx] * md[cy] * kd[cz];
        L.diag[i] = d;
        L.stiff.dinv[i] = 1.0 / d;
        L.dinv_sqrt[i] = 1.0 / std::sqrt(d);
        L.dsqrt[i] = std::sqrt(d);
        L.wint[i] = msum[cx] * msum[cy] * msum[cz];
      }
  // mass M (x) M (x) M through the same kernel: g-path off (krow = 0), h-path
  // h = Mx My x, and the z element matrix of the h-path set to the mass.
  OpTab& M = L.mass;
  M = A;
  for (int c = 0; c < q; ++c)
    for (int o = 0; o < 2 * kMaxQ + 1; ++o) {
      M.krow[c][o] = 0.0;
      M.zkrow[c][o] = A.mrow[c][o];
      M.zmrow[c][o] = 0.0;
    }
  for (int a = 0; a <= q; ++a)
    for (int b = 0; b <= q; ++b) {
      M.zk[a][b] = A.zm[a][b];
      M.zm[a][b] = 0.0;
    }
  return L;
}

// Reference coordinate, inside the coarse element, of child node b = 0 .. 2q.
static double child_coord(const std::vector<double>& xi, int q, int b) {
  if (b == 2 * q) return 1.0;
  const int e = b / q, a = b % q;
  return (e + xi[a]) / 2.0;
}

void make_transfer_table(int q, TransferTab* tab) {
  const std::vector<double> xi = lgl_nodes01(q);
  std::memset(tab, 0, sizeof(TransferTab));
  tab->q = q;
  for (int b = 0; b < 2 * q; ++b)
    for (int a = 0; a <= q; ++a) tab->p[b][a] = lagrange_at(xi, a, child_coord(xi, q, b));
  // coarse node qE + a gathers fine 2qE + (t - 2q): for t >= 2q the children of
  // element E (child node t - 2q, value phi_a there); for t < 2q the children of
  // element E-1, reached only by the vertex a = 0 (coarse local node q of E-1).
  for (int a = 0; a < q; ++a)
    for (int t = 0; t <= 4 * q; ++t) {
      double w = 0.0;
      if (t >= 2 * q) w = lagrange_at(xi, a, child_coord(xi, q, t - 2 * q));
      else if (a == 0) w = lagrange_at(xi, q, child_coord(xi, q, t));
      tab->r[a][t] = (std::fabs(w) < 1e-15) ? 0.0 : w;
    }
}

// Rows of the assembled periodic 1D matrix, any order: row c (node class), tap o + q.
static std::vector<double> generic_rows(int q, const std::vector<double>& ehat, double scale) {
  const int w = 2 * q + 1;
  std::vector<double> rows(static_cast<size_t>(q) * w, 0.0);
  for (int b = 0; b <= q; ++b) {
    rows[(b - q) + q] += ehat[q * (q + 1) + b] * scale;  // vertex: left element (local node q)
    rows[b + q] += ehat[0 * (q + 1) + b] * scale;        // vertex: right element (local node 0)
  }
  for (int c = 1; c < q; ++c)
    for (int b = 0; b <= q; ++b) rows[c * w + (b - c) + q] = ehat[c * (q + 1) + b] * scale;
  return rows;
}

GenTables make_generic_tables(int q, int n) {
  GenTables T;
  T.q = q;
  const double h = 1.0 / n;
  const int w = 2 * q + 1, blk = q * w;
  std::vector<double> khat, mhat;
  reference_matrices(q, &khat, &mhat);
  const std::vector<double> K = generic_rows(q, khat, 1.0 / h), M = generic_rows(q, mhat, h);
  const std::vector<double> Z(blk, 0.0);
  // stiffness: z (K, M), y (K, M), x (K, M); mass: z (0, M), y (0, M), x (M, M)
  for (const auto* part : {&K, &M, &K, &M, &K, &M}) T.stiff_rows.insert(T.stiff_rows.end(), part->begin(), part->end());
  for (const auto* part : {&Z, &M, &Z, &M, &M, &M}) T.mass_rows.insert(T.mass_rows.end(), part->begin(), part->end());
  // diagonal entries: the taps landing on the node itself (offset 0, and +-q on a single
  // periodic element, where both ends of the element are the node)
  const int N = q * n;
  std::vector<double> kd(q, 0.0), md(q, 0.0), msum(q, 0.0);
  for (int c = 0; c < q; ++c)
    for (int o = -q; o <= q; ++o) {
      if (o % N == 0) {
        kd[c] += K[c * w + o + q];
        md[c] += M[c * w + o + q];
      }
      msum[c] += M[c * w + o + q];
    }
  const int nc = q * q * q;
  T.diag.resize(nc);
  T.dinv.resize(nc);
  T.dsqrt.resize(nc);
  T.dinv_sqrt.resize(nc);
  T.wint.resize(nc);
  for (int cz = 0; cz < q; ++cz)
    for (int cy = 0; cy < q; ++cy)
      for (int cx = 0; cx < q; ++cx) {
        const int i = cx + q * (cy + q * cz);
        const double d = kd[cx] * md[cy] * md[cz] + md[cx] * kd[cy] * md[cz] + md[cx] * md[cy] * kd[cz];
        T.diag[i] = d;
        T.dinv[i] = 1.0 / d;
        T.dinv_sqrt[i] = 1.0 / std::sqrt(d);
        T.dsqrt[i] = std::sqrt(d);
        T.wint[i] = msum[cx] * msum[cy] * msum[cz];
      }
  return T;
}

void make_generic_transfer(int q, std::vector<double>* p, std::vector<double>* r) {
  const std::vector<double> xi = lgl_nodes01(q);
  p->assign(static_cast<size_t>(2 * q) * (q + 1), 0.0);
  r->assign(static_cast<size_t>(q) * (4 * q + 1), 0.0);
  for (int b = 0; b < 2 * q; ++b)
    for (int a = 0; a <= q; ++a) (*p)[b * (q + 1) + a] = lagrange_at(xi, a, child_coord(xi, q, b));
  for (int a = 0; a < q; ++a)
    for (int t = 0; t <= 4 * q; ++t) {
      double w = 0.0;
      if (t >= 2 * q) w = lagrange_at(xi, a, child_coord(xi, q, t - 2 * q));
      else if (a == 0) w = lagrange_at(xi, q, child_coord(xi, q, t));
      (*r)[a * (4 * q + 1) + t] = (std::fabs(w) < 1e-15) ? 0.0 : w;
    }
}

// Dense periodic 1D matrices of order q on n elements (N = q n).
static void dense_1d(int q, int n, std::vector<double>* K, std::vector<double>* M) {
  const int N = q * n;
  const double h = 1.0 / n;
  std::vector<double> khat, mhat;
  reference_matrices(q, &khat, &mhat);
  K->assign(static_cast<size_t>(N) * N, 0.0);
  M->assign(static_cast<size_t>(N) * N, 0.0);
  for (int e = 0; e < n; ++e)
    for (int a = 0; a <= q; ++a)
      for (int b = 0; b <= q; ++b) {
        const int i = (q * e + a) % N, j = (q * e + b) % N;
        (*K)[static_cast<size_t>(i) * N + j] += khat[a * (q + 1) + b] / h;
        (*M)[static_cast<size_t>(i) * N + j] += mhat[a * (q + 1) + b] * h;
      }
}

// Generalized symmetric eigenpairs of the 1D pair (K, M), M positive definite:
// V^T M V = I and V^T K V = diag(lam), V column-wise (V[i N + a] = component i of
// eigenvector a).  M = L L^T (Cholesky), C = L^-1 K L^-T diagonalised by cyclic Jacobi
// rotations, V = L^-T U.  N is one element's worth of nodes here (q <= 16).
static void generalized_eigen_1d(int N, const std::vector<double>& K, const std::vector<double>& M,
                                 std::vector<double>* V, std::vector<double>* lam) {
  std::vector<double> L(static_cast<size_t>(N) * N, 0.0);
  for (int j = 0; j < N; ++j) {
    double d = M[j * N + j];
    for (int k = 0; k < j; ++k) d -= L[j * N + k] * L[j * N + k];
    if (!(d > 0.0)) throw std::runtime_error("1D mass matrix is not positive definite");
    L[j * N + j] = std::sqrt(d);
    for (int i = j + 1; i < N; ++i) {
      double t = M[i * N + j];
      for (int k = 0; k < j; ++k) t -= L[i * N + k] * L[j * N + k];
      L[i * N + j] = t / L[j * N + j];
    }
  }
  // X = L^-1 K (forward substitution per column), C = L^-1 X^T = L^-1 K L^-T
  auto lower_solve = [&](const std::vector<double>& B, std::vector<double>* X) {
    X->assign(static_cast<size_t>(N) * N, 0.0);
    for (int c = 0; c < N; ++c)
      for (int i = 0; i < N; ++i) {
        double t = B[i * N + c];
        for (int k = 0; k < i; ++k) t -= L[i * N + k] * (*X)[k * N + c];
        (*X)[i * N + c] = t / L[i * N + i];
      }
  };
  std::vector<double> X, Xt(static_cast<size_t>(N) * N), C;
  lower_solve(K, &X);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) Xt[i * N + j] = X[j * N + i];
  lower_solve(Xt, &C);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < i; ++j) C[i * N + j] = C[j * N + i] = 0.5 * (C[i * N + j] + C[j * N + i]);
  std::vector<double> U(static_cast<size_t>(N) * N, 0.0);
  for (int i = 0; i < N; ++i) U[i * N + i] = 1.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        tot += C[i * N + j] * C[i * N + j];
        if (i != j) off += C[i * N + j] * C[i * N + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < N - 1; ++p)
      for (int r = p + 1; r < N; ++r) {
        const double apr = C[p * N + r];
        if (apr == 0.0) continue;
        // the rotation that zeroes C[p][r]: tan(2 theta) = 2 apr / (arr - app)
        const double theta = 0.5 * std::atan2(2.0 * apr, C[r * N + r] - C[p * N + p]);
        const double cs = std::cos(theta), sn = std::sin(theta);
        for (int k = 0; k < N; ++k) {  // columns p, r
          const double ckp = C[k * N + p], ckr = C[k * N + r];
          C[k * N + p] = cs * ckp - sn * ckr;
          C[k * N + r] = sn * ckp + cs * ckr;
        }
        for (int k = 0; k < N; ++k) {  // rows p, r
          const double cpk = C[p * N + k], crk = C[r * N + k];
          C[p * N + k] = cs * cpk - sn * crk;
          C[r * N + k] = sn * cpk + cs * crk;
        }
        for (int k = 0; k < N; ++k) {
          const double ukp = U[k * N + p], ukr = U[k * N + r];
          U[k * N + p] = cs * ukp - sn * ukr;
          U[k * N + r] = sn * ukp + cs * ukr;
        }
      }
  }
  lam->assign(N, 0.0);
  for (int a = 0; a < N; ++a) (*lam)[a] = C[a * N + a];
  // V = L^-T U (back substitution per column)
  V->assign(static_cast<size_t>(N) * N, 0.0);
  for (int c = 0; c < N; ++c)
    for (int i = N - 1; i >= 0; --i) {
      double t = U[i * N + c];
      for (int k = i + 1; k < N; ++k) t -= L[k * N + i] * (*V)[k * N + c];
      (*V)[i * N + c] = t / L[i * N + i];
    }
}

// (A_0 + 1 1^T / n0)^-1 from the eigenpairs of the 1D pair instead of a dense
// factorisation (n0 up to 4096: one periodic element of order 16).  With W = V (x) V (x) V,
// W^T A_0 W = D = lam (+) lam (+) lam, so for r orthogonal to the constants
// e = W D^+ W^T r solves A_0 e = r (D^+ drops the one zero eigenvalue, the constants);
// removing its mean gives A_0^+ r, and the matrix is A_0^+ + 1 1^T / n0.  Column c:
// W^T (e_c - 1/n0) is the outer product of three rows of V less W^T 1 / n0, then three
// 1D mode products with V.
static std::vector<double> kron_pseudo_inverse(int q, int n) {
  const int N = q * n;
  const int n0 = N * N * N;
  std::vector<double> K, M, V, lam;
  dense_1d(q, n, &K, &M);
  generalized_eigen_1d(N, K, M, &V, &lam);
  int a0 = 0;
  for (int a = 1; a < N; ++a)
    if (std::abs(lam[a]) < std::abs(lam[a0])) a0 = a;
  std::vector<double> dplus(n0), u(N, 0.0);
  for (int c = 0; c < N; ++c)
    for (int b = 0; b < N; ++b)
      for (int a = 0; a < N; ++a) {
        const double d = lam[a] + lam[b] + lam[c];
        dplus[a + N * (b + N * c)] = (a == a0 && b == a0 && c == a0) ? 0.0 : 1.0 / d;
      }
  for (int a = 0; a < N; ++a)
    for (int i = 0; i < N; ++i) u[a] += V[i * N + a];
  std::vector<double> inv(static_cast<size_t>(n0) * n0);
  std::vector<double> t(n0), w(n0);
  const double inv_n0 = 1.0 / n0;
  for (int col = 0; col < n0; ++col) {
    const int i = col % N, j = (col / N) % N, k = col / (N * N);
    for (int c = 0; c < N; ++c)
      for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a) {
          const int idx = a + N * (b + N * c);
          t[idx] = (V[i * N + a] * V[j * N + b] * V[k * N + c] - inv_n0 * u[a] * u[b] * u[c]) * dplus[idx];
        }
    // y = W t: a mode product along each axis
    for (int c = 0; c < N; ++c)
      for (int b = 0; b < N; ++b)
        for (int x = 0; x < N; ++x) {
          double s = 0.0;
          for (int a = 0; a < N; ++a) s += V[x * N + a] * t[a + N * (b + N * c)];
          w[x + N * (b + N * c)] = s;
        }
    for (int c = 0; c < N; ++c)
      for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
          double s = 0.0;
          for (int b = 0; b < N; ++b) s += V[y * N + b] * w[x + N * (b + N * c)];
          t[x + N * (y + N * c)] = s;
        }
    double mean = 0.0;
    for (int z = 0; z < N; ++z)
      for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
          double s = 0.0;
          for (int c = 0; c < N; ++c) s += V[z * N + c] * t[x + N * (y + N * c)];
          w[x + N * (y + N * z)] = s;
          mean += s;
        }
    mean *= inv_n0;
    for (int r = 0; r < n0; ++r) inv[static_cast<size_t>(r) * n0 + col] = w[r] - mean + inv_n0;
  }
  return inv;
}

std::vector<double> coarse_pseudo_inverse(int q, int n) {
  const int N = q * n;
  const int n0 = N * N * N;
  if (n0 > 512) return kron_pseudo_inverse(q, n);
  std::vector<double> K, M;
  dense_1d(q, n, &K, &M);
  // A_0 = K (x) M (x) M + M (x) K (x) M + M (x) M (x) K
  std::vector<double> A(static_cast<size_t>(n0) * n0);
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        const int r = i + N * (j + N * k);
        for (int kk = 0; kk < N; ++kk)
          for (int jj = 0; jj < N; ++jj)
            for (int ii = 0; ii < N; ++ii) {
              const int c = ii + N * (jj + N * kk);
              A[static_cast<size_t>(r) * n0 + c] = K[i * N + ii] * M[j * N + jj] * M[k * N + kk] +
                                                   M[i * N + ii] * K[j * N + jj] * M[k * N + kk] +
                                                   M[i * N + ii] * M[j * N + jj] * K[k * N + kk];
            }
      }
  return dense_pseudo_inverse(std::move(A), n0);
}

std::vector<double> dense_pseudo_inverse(std::vector<double> B, int n0) {
  // B = A_0 + 1 1^T / n0
  for (auto& v : B) v += 1.0 / n0;
  // Cholesky B = L L^T (lower triangle in place)
  for (int j = 0; j < n0; ++j) {
    double d = B[static_cast<size_t>(j) * n0 + j];
    for (int k = 0; k < j; ++k) d -= B[static_cast<size_t>(j) * n0 + k] * B[static_cast<size_t>(j) * n0 + k];
    if (!(d > 0.0)) throw std::runtime_error("coarse matrix is not positive definite");
    const double ljj = std::sqrt(d);
    B[static_cast<size_t>(j) * n0 + j] = ljj;
    for (int i = j + 1; i < n0; ++i) {
      double s = B[static_cast<size_t>(i) * n0 + j];
      for (int k = 0; k < j; ++k) s -= B[static_cast<size_t>(i) * n0 + k] * B[static_cast<size_t>(j) * n0 + k];
      B[static_cast<size_t>(i) * n0 + j] = s / ljj;
    }
  }
  // inverse column by column: solve L y = e_c, L^T x = y
  std::vector<double> inv(static_cast<size_t>(n0) * n0);
  std::vector<double> y(n0);
  for (int c = 0; c < n0; ++c) {
    for (int i = 0; i < n0; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= B[static_cast<size_t>(i) * n0 + k] * y[k];
      y[i] = s / B[static_cast<size_t>(i) * n0 + i];
    }
    for (int i = n0 - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < n0; ++k) s -= B[static_cast<size_t>(k) * n0 + i] * inv[static_cast<size_t>(k) * n0 + c];
      inv[static_cast<size_t>(i) * n0 + c] = s / B[static_cast<size_t>(i) * n0 + i];
    }
  }
  // symmetrize (the kernel reads it column-major = row-major)
  for (int i = 0; i < n0; ++i)
    for (int j = i + 1; j < n0; ++j) {
      const double v = 0.5 * (inv[static_cast<size_t>(i) * n0 + j] + inv[static_cast<size_t>(j) * n0 + i]);
      inv[static_cast<size_t>(i) * n0 + j] = v;
      inv[static_cast<size_t>(j) * n0 + i] = v;
    }
  return inv;
}

uint64_t splitmix64_at(uint64_t key, uint64_t i) {
  uint64_t z = key + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void lanczos_start_vector(uint64_t seed, int level, int64_t count, double* out) {
  const uint64_t key = seed + static_cast<uint64_t>(level);
  for (int64_t i = 0; i < count; ++i)
    out[i] = 2.0 * static_cast<double>(splitmix64_at(key, static_cast<uint64_t>(i)) >> 11) * 0x1.0p-53 - 1.0;
}

double tridiag_max_eig(const std::vector<double>& alpha, const std::vector<double>& beta) {
  const int m = static_cast<int>(alpha.size());
  if (m == 0) return 0.0;
  // Gershgorin bounds
  double lo = alpha[0], hi = alpha[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(beta[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(beta[i]) : 0.0);
    lo = std::min(lo, alpha[i] - r);
    hi = std::max(hi, alpha[i] + r);
  }
  // count of eigenvalues < x via the Sturm sequence of the LDL^T pivots
  auto count_below = [&](double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      const double b2 = i > 0 ? beta[i - 1] * beta[i - 1] : 0.0;
      d = (alpha[i] - x) - (i > 0 ? b2 / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_below(mid) == m) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace gmg
