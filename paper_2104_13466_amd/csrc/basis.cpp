// Host construction of the one-dimensional bases of Section 2 (construction of
// high-order bases), FP64.  Own implementation: Gauss rules by the
// Golub-Welsch eigenvalue method, a cyclic Jacobi symmetric eigensolver, and
// Cholesky solves for the minimum-energy coefficients.
#include <cmath>
#include <cstring>
#include <vector>

#include "sdme.h"
#include "sdme_internal.h"

namespace sdme {

// Cyclic Jacobi rotations for a symmetric n x n matrix A (row-major, destroyed).
// On return ev[i] are the eigenvalues (ascending) and column i of V the
// corresponding unit eigenvector.
static bool sym_eig(int n, std::vector<double> &A, std::vector<double> &ev,
                    std::vector<double> &V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; i++) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0, diag = 0;
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) (i == j ? diag : off) += A[i * n + j] * A[i * n + j];
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; p++)
      for (int q = p + 1; q < n; q++) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; k++) {  // A <- A J
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; k++) {  // A <- J^T A
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; k++) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  ev.resize(n);
  for (int i = 0; i < n; i++) ev[i] = A[i * n + i];
  // sort ascending (selection sort, permuting columns of V)
  for (int i = 0; i < n; i++) {
    int m = i;
    for (int j = i + 1; j < n; j++)
      if (ev[j] < ev[m]) m = j;
    if (m != i) {
      std::swap(ev[i], ev[m]);
      for (int k = 0; k < n; k++) std::swap(V[k * n + i], V[k * n + m]);
    }
  }
  for (int i = 0; i < n; i++)
    if (!std::isfinite(ev[i])) return false;
  return true;
}

// Orthonormal Legendre recurrence: Gauss-Legendre rule by Golub-Welsch
// (eigenvalues of the symmetric tridiagonal Jacobi matrix, weights from the
// first eigenvector components), polished by Newton steps on P_Q.
static void legendre(int n, double x, double *p, double *dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int k = 2; k <= n; k++) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double d2 = d0 + (2.0 * k - 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *p = p1;
  *dp = d1;
}

bool gauss_legendre(int Q, double *x, double *w) {
  std::vector<double> J(Q * Q, 0.0), ev, V;
  for (int k = 1; k < Q; k++) {
    double b = k / std::sqrt(4.0 * k * k - 1.0);
    J[(k - 1) * Q + k] = J[k * Q + k - 1] = b;
  }
  if (!sym_eig(Q, J, ev, V)) return false;
  for (int i = 0; i < Q; i++) {
    double xi = ev[i];
    for (int it = 0; it < 3; it++) {
      double p, dp;
      legendre(Q, xi, &p, &dp);
      xi -= p / dp;
    }
    double p, dp;
    legendre(Q, xi, &p, &dp);
    x[i] = xi;
    w[i] = 2.0 / ((1.0 - xi * xi) * dp * dp);  // standard closed form, consistent with 2 v0^2
  }
  return true;
}

// Jacobi polynomial P_n^{a,b}(x) by its three-term recurrence.
static double jacobi_p(int n, double a, double b, double x) {
  if (n == 0) return 1.0;
  double pm = 1.0, p = 0.5 * (a - b + (a + b + 2.0) * x);
  for (int m = 1; m < n; m++) {
    double c = 2.0 * m + a + b;
    double num = (c + 1.0) * (c * (c + 2.0) * x + a * a - b * b) * p -
                 2.0 * (m + a) * (m + b) * (c + 2.0) * pm;
    double den = 2.0 * (m + 1.0) * (m + a + b + 1.0) * c;
    pm = p;
    p = num / den;
  }
  return p;
}

// Modal starting basis (Eq. BasePadrao1D, alpha = beta = 1), index order
// 0 = (1-x)/2, 1 = (1+x)/2, p >= 2 bubbles.
static void modal_eval(int P, double x, double *v, double *d) {
  v[0] = 0.5 * (1.0 - x); d[0] = -0.5;
  v[1] = 0.5 * (1.0 + x); d[1] = 0.5;
  for (int p = 2; p <= P; p++) {
    double j = jacobi_p(p - 2, 1.0, 1.0, x);
    double dj = (p - 2 == 0) ? 0.0 : 0.5 * (p - 2 + 3.0) * jacobi_p(p - 3, 2.0, 2.0, x);
    double bub = 0.25 * (1.0 - x * x);
    v[p] = bub * j;
    d[p] = -0.5 * x * j + bub * dj;
  }
}

// GLL points: the P-1 interior points are the roots of P_P', i.e. of
// P_{P-1}^{(1,1)}; Golub-Welsch on the Jacobi(1,1) recurrence.
static bool gll_points(int P, double *z) {
  z[0] = -1.0;
  z[P] = 1.0;
  int m = P - 1;
  if (m <= 0) return true;
  std::vector<double> J(m * m, 0.0), ev, V;
  for (int k = 1; k < m; k++) {
    // monic Jacobi(1,1): beta_k = k (k+2) / ((2k+1)(2k+3))
    double b = std::sqrt(k * (k + 2.0) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)));
    J[(k - 1) * m + k] = J[k * m + k - 1] = b;
  }
  if (!sym_eig(m, J, ev, V)) return false;
  for (int i = 0; i < m; i++) z[i + 1] = ev[i];
  return true;
}

// Gauss-Lobatto-Legendre rule of Q points (exact to degree 2Q - 3): the GLL
// points of order Q - 1 with weights 2 / (Q (Q - 1) L_{Q-1}(x)^2).
bool gll_rule(int Q, double *x, double *w) {
  if (Q < 2 || !gll_points(Q - 1, x)) return false;
  for (int i = 0; i < Q; i++) {
    double p, dp;
    legendre(Q - 1, x[i], &p, &dp);
    w[i] = 2.0 / (Q * (Q - 1.0) * p * p);
  }
  return true;
}

static void nodal_eval(int P, const double *z, double x, double *v, double *d) {
  int n = P + 1;
  for (int a = 0; a < n; a++) {
    double val = 1.0, der = 0.0;
    for (int b = 0; b < n; b++) {
      if (b == a) continue;
      double f = 1.0 / (z[a] - z[b]);
      der = der * (x - z[b]) * f + val * f;  // product rule, running
      val *= (x - z[b]) * f;
    }
    v[a] = val;
    d[a] = der;
  }
}

bool Basis::build(int P_, int kind_, double k_, double lam_) {
  P = P_; kind = kind_; k = k_; lam = lam_;
  int n = P + 1;
  nodal = (kind == SDME_BASIS_NODAL);
  z.assign(n, 0.0);
  if (nodal && !gll_points(P, z.data())) return false;
  // starting-basis vertex/internal index sets
  std::vector<int> vi, ii;
  if (nodal) { vi = {0, P}; for (int p = 1; p < P; p++) ii.push_back(p); }
  else { vi = {0, 1}; for (int p = 2; p <= P; p++) ii.push_back(p); }
  // 1D mass and stiffness of the starting basis (Eqs. Matrizesmassa,
  // Matrizesrigidez), exact with P+2 Gauss points
  int nq = P + 2;
  std::vector<double> xq(nq), wq(nq), v(n), d(n);
  if (!gauss_legendre(nq, xq.data(), wq.data())) return false;
  std::vector<double> M(n * n, 0.0), K(n * n, 0.0);
  for (int q = 0; q < nq; q++) {
    start_eval(xq[q], v.data(), d.data());
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) {
        M[i * n + j] += wq[q] * v[i] * v[j];
        K[i * n + j] += wq[q] * d[i] * d[j];
      }
  }
  T.assign(n * n, 0.0);
  lambda_s.assign(P > 1 ? P - 1 : 0, 0.0);
  bool sdme = (kind == SDME_BASIS_SDME_M || kind == SDME_BASIS_SDME_K || kind == SDME_BASIS_SDME_H);
  if (!sdme || P < 2) {
    T[0 * n + vi[0]] = 1.0;
    T[P * n + vi[1]] = 1.0;
    for (int s = 1; s < P; s++) T[s * n + ii[s - 1]] = 1.0;
  } else {
    int m = P - 1;
    std::vector<double> Mii(m * m), Kii(m * m), ev, X, Lm, lz, Z;
    for (int i = 0; i < m; i++)
      for (int j = 0; j < m; j++) {
        Mii[i * m + j] = M[ii[i] * n + ii[j]];
        Kii[i * m + j] = K[ii[i] * n + ii[j]];
      }
    // Eq. diagMassa: X^T M_ii X = Lambda_M
    std::vector<double> Mc = Mii;
    if (!sym_eig(m, Mc, ev, X)) return false;
    std::vector<double> Xs(m * m);  // X Lambda_M^{-1/2}
    for (int i = 0; i < m; i++)
      for (int j = 0; j < m; j++) {
        if (ev[j] <= 0) return false;
        Xs[i * m + j] = X[i * m + j] / std::sqrt(ev[j]);
      }
    // Eq. L: L = Xs^T K_ii Xs ; Eq. diagL: Z^T L Z = Lambda_S
    Lm.assign(m * m, 0.0);
    for (int i = 0; i < m; i++)
      for (int j = 0; j < m; j++) {
        double s = 0;
        for (int a = 0; a < m; a++)
          for (int b = 0; b < m; b++) s += Xs[a * m + i] * Kii[a * m + b] * Xs[b * m + j];
        Lm[i * m + j] = s;
      }
    for (int i = 0; i < m; i++)
      for (int j = i + 1; j < m; j++) Lm[i * m + j] = Lm[j * m + i] = 0.5 * (Lm[i * m + j] + Lm[j * m + i]);
    if (!sym_eig(m, Lm, lz, Z)) return false;
    for (int i = 0; i < m; i++) {
      if (lz[i] <= 0) return false;
      lambda_s[i] = lz[i];
    }
    // Eq. Y: Y = (Xs Z Lambda_S^{-k/2})^T; internal slot r = row r of Y
    std::vector<double> Tint(m * n, 0.0);
    for (int r = 0; r < m; r++)
      for (int i = 0; i < m; i++) {
        double s = 0;
        for (int a = 0; a < m; a++) s += Xs[i * m + a] * Z[a * m + r];
        Tint[r * n + ii[i]] = s * std::pow(lz[r], -0.5 * k);
      }
    // sign: derivative at -1 positive
    start_eval(-1.0, v.data(), d.data());
    for (int r = 0; r < m; r++) {
      double dm1 = 0;
      for (int j = 0; j < n; j++) dm1 += Tint[r * n + j] * d[j];
      if (dm1 < 0)
        for (int j = 0; j < n; j++) Tint[r * n + j] = -Tint[r * n + j];
    }
    // ME: A = M, K or K + lam M; alpha = A'_vi A'_ii^{-1} (Eqs. alphaMassa,
    // alphaRigidez, alphaKN) on the SD internal modes
    std::vector<double> A(n * n);
    for (int i = 0; i < n * n; i++)
      A[i] = (kind == SDME_BASIS_SDME_M) ? M[i] : (kind == SDME_BASIS_SDME_K) ? K[i] : K[i] + lam * M[i];
    std::vector<double> Aii(m * m, 0.0), Avi(2 * m, 0.0);
    for (int r = 0; r < m; r++) {
      for (int s = 0; s < m; s++) {
        double acc = 0;
        for (int a = 0; a < n; a++)
          for (int b = 0; b < n; b++) acc += Tint[r * n + a] * A[a * n + b] * Tint[s * n + b];
        Aii[r * m + s] = acc;
      }
      for (int vv = 0; vv < 2; vv++) {
        double acc = 0;
        for (int b = 0; b < n; b++) acc += A[vi[vv] * n + b] * Tint[r * n + b];
        Avi[vv * m + r] = acc;
      }
    }
    // Cholesky of Aii, then alpha rows solve Aii alpha^T = Avi^T
    std::vector<double> Lc(m * m, 0.0);
    for (int i = 0; i < m; i++)
      for (int j = 0; j <= i; j++) {
        double s = Aii[i * m + j];
        for (int t = 0; t < j; t++) s -= Lc[i * m + t] * Lc[j * m + t];
        if (i == j) {
          if (s <= 0) return false;
          Lc[i * m + i] = std::sqrt(s);
        } else {
          Lc[i * m + j] = s / Lc[j * m + j];
        }
      }
    for (int vv = 0; vv < 2; vv++) {
      std::vector<double> y(m), al(m);
      for (int i = 0; i < m; i++) {
        double s = Avi[vv * m + i];
        for (int t = 0; t < i; t++) s -= Lc[i * m + t] * y[t];
        y[i] = s / Lc[i * m + i];
      }
      for (int i = m - 1; i >= 0; i--) {
        double s = y[i];
        for (int t = i + 1; t < m; t++) s -= Lc[t * m + i] * al[t];
        al[i] = s / Lc[i * m + i];
      }
      int slot = vv == 0 ? 0 : P;
      for (int j = 0; j < n; j++) T[slot * n + j] = (j == vi[vv]) ? 1.0 : 0.0;
      for (int r = 0; r < m; r++)
        for (int j = 0; j < n; j++) T[slot * n + j] -= al[r] * Tint[r * n + j];
    }
    for (int r = 0; r < m; r++)
      for (int j = 0; j < n; j++) T[(r + 1) * n + j] = Tint[r * n + j];
  }
  // slot-order 1D mass and stiffness
  M1.assign(n * n, 0.0);
  K1.assign(n * n, 0.0);
  for (int s = 0; s < n; s++)
    for (int t = 0; t < n; t++) {
      double am = 0, ak = 0;
      for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
          am += T[s * n + a] * M[a * n + b] * T[t * n + b];
          ak += T[s * n + a] * K[a * n + b] * T[t * n + b];
        }
      M1[s * n + t] = am;
      K1[s * n + t] = ak;
    }
  return true;
}

void Basis::start_eval(double x, double *v, double *d) const {
  if (nodal) nodal_eval(P, z.data(), x, v, d);
  else modal_eval(P, x, v, d);
}

void Basis::eval(double x, double *v, double *d) const {
  int n = P + 1;
  std::vector<double> sv(n), sd(n);
  start_eval(x, sv.data(), sd.data());
  for (int s = 0; s < n; s++) {
    double a = 0, b = 0;
    for (int j = 0; j < n; j++) {
      a += T[s * n + j] * sv[j];
      b += T[s * n + j] * sd[j];
    }
    v[s] = a;
    if (d) d[s] = b;
  }
}

// Expansion of 1 and xi in the basis (both lie in the span): interpolation at
// P+1 distinct points, solved by Gaussian elimination with partial pivoting.
bool Basis::affine(double *g1, double *gx) const {
  int n = P + 1;
  std::vector<double> A(n * n), b1(n), bx(n), row(n);
  for (int i = 0; i < n; i++) {
    double xi = -std::cos(M_PI * (i + 0.5) / n);  // Chebyshev points
    eval(xi, row.data(), nullptr);
    for (int s = 0; s < n; s++) A[i * n + s] = row[s];
    b1[i] = 1.0;
    bx[i] = xi;
  }
  for (int c = 0; c < n; c++) {
    int piv = c;
    for (int r = c + 1; r < n; r++)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int s = 0; s < n; s++) std::swap(A[c * n + s], A[piv * n + s]);
      std::swap(b1[c], b1[piv]);
      std::swap(bx[c], bx[piv]);
    }
    for (int r = c + 1; r < n; r++) {
      double f = A[r * n + c] / A[c * n + c];
      for (int s = c; s < n; s++) A[r * n + s] -= f * A[c * n + s];
      b1[r] -= f * b1[c];
      bx[r] -= f * bx[c];
    }
  }
  for (int c = n - 1; c >= 0; c--) {
    double s1 = b1[c], sx = bx[c];
    for (int s = c + 1; s < n; s++) {
      s1 -= A[c * n + s] * g1[s];
      sx -= A[c * n + s] * gx[s];
    }
    g1[c] = s1 / A[c * n + c];
    gx[c] = sx / A[c * n + c];
  }
  return true;
}

}  // namespace sdme

extern "C" int sdme_basis_build(int P, int Q, int kind, double k, double lambda_h, double *x,
                                double *w, double *B, double *D, double *M1, double *K1,
                                double *lambda_s) {
  if (P < 1 || P > 10 || Q < P + 1 || Q > 16 || kind < 0 || kind > 4 || !(k >= 0 && k <= 1) ||
      !(lambda_h >= 0))
    return SDME_EINVAL;
  sdme::Basis b;
  if (!b.build(P, kind, k, lambda_h)) return SDME_EEIG;
  int n = P + 1;
  std::vector<double> xq(Q), wq(Q);
  if (!sdme::gauss_legendre(Q, xq.data(), wq.data())) return SDME_EEIG;
  if (x) std::memcpy(x, xq.data(), sizeof(double) * Q);
  if (w) std::memcpy(w, wq.data(), sizeof(double) * Q);
  std::vector<double> v(n), d(n);
  for (int q = 0; q < Q; q++) {
    b.eval(xq[q], v.data(), d.data());
    for (int s = 0; s < n; s++) {
      if (B) B[q * n + s] = v[s];
      if (D) D[q * n + s] = d[s];
    }
  }
  if (M1) std::memcpy(M1, b.M1.data(), sizeof(double) * n * n);
  if (K1) std::memcpy(K1, b.K1.data(), sizeof(double) * n * n);
  if (lambda_s)
    for (int i = 0; i < P - 1; i++) lambda_s[i] = b.lambda_s.empty() ? 0.0 : b.lambda_s[i];
  return SDME_OK;
}

extern "C" int sdme_basis_eval(int P, int kind, double k, double lambda_h, int npts,
                               const double *pts, double *V, double *dV) {
  if (P < 1 || P > 10 || kind < 0 || kind > 4 || npts < 0 || (npts > 0 && (!pts || !V)) ||
      !(k >= 0 && k <= 1) || !(lambda_h >= 0))
    return SDME_EINVAL;
  sdme::Basis b;
  if (!b.build(P, kind, k, lambda_h)) return SDME_EEIG;
  int n = P + 1;
  for (int i = 0; i < npts; i++) b.eval(pts[i], V + (size_t)i * n, dV ? dV + (size_t)i * n : nullptr);
  return SDME_OK;
}
