// Internal declarations of libsdme (not part of the C ABI).
#pragma once
#include <cstdint>
#include <vector>

#include "sdme.h"

namespace sdme {

bool gauss_legendre(int Q, double *x, double *w);
bool gll_rule(int Q, double *x, double *w);
// The volume rule of a mesh: Gauss-Legendre for Q = P + 2, Gauss-Lobatto-
// Legendre for Q = P + 1.
inline bool volume_rule(int P, int Q, double *x, double *w) {
  return Q == P + 1 ? gll_rule(Q, x, w) : gauss_legendre(Q, x, w);
}

// 1D basis held as a coefficient matrix T (slot x starting index) over its
// starting basis (Jacobi modal, or Lagrange on GLL points for the nodal kind).
struct Basis {
  int P = 0, kind = 0;
  double k = 0.5, lam = 100.0;
  bool nodal = false;
  std::vector<double> z;  // GLL points (nodal start)
  std::vector<double> T, M1, K1, lambda_s;
  bool build(int P, int kind, double k, double lam);
  void start_eval(double x, double *v, double *d) const;
  void eval(double x, double *v, double *d) const;
  bool affine(double *g1, double *gx) const;
};

}  // namespace sdme
