"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library's host basis construction (csrc/basis.cpp: Gauss rules, Jacobi
eigensolver, minimum-energy solves) and the oracle's C operators (oracle/fem.c)
are compiled with -fsanitize=address,undefined into small drivers that call
every entry point over the orders and kinds the tests use; any out-of-bounds
access, leak or undefined operation aborts the driver."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]

BASIS_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "sdme.h"
int main() {
  for (int P = 1; P <= 10; P++)
    for (int kind = 0; kind <= 4; kind++)
      for (int Q : {P + 1, P + 2}) {
        const int n = P + 1;
        std::vector<double> x(Q), w(Q), B(Q * n), D(Q * n), M(n * n), K(n * n), ls(n);
        for (double k : {0.0, 0.5, 1.0})
          if (sdme_basis_build(P, Q, kind, k, 100.0, x.data(), w.data(), B.data(), D.data(),
                               M.data(), K.data(), ls.data()) != 0) {
            std::printf("build failed P=%d kind=%d\n", P, kind);
            return 1;
          }
        std::vector<double> pts = {-1.0, -0.3, 0.0, 0.7, 1.0}, V(5 * n), dV(5 * n);
        if (sdme_basis_eval(P, kind, 0.5, 400.0, 5, pts.data(), V.data(), dV.data()) != 0) return 2;
      }
  // argument checks
  double d[4];
  if (sdme_basis_build(0, 2, 4, 0.5, 100.0, d, d, d, d, d, d, d) == 0) return 3;
  std::printf("ok\n");
  return 0;
}
"""

FEM_DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include <math.h>
/* the oracle's mesh arguments: nx, ny, nz, P, Q, h, B, D, w */
#define MA int, int, int, int, int, const double *, const double *, const double *, const double *
int64_t or_num_nodes(int, int, int, int);
void or_gather_map(int, int, int, int, int32_t *);
int or_internal_force(MA, const double *, const double *, const double *, double *);
int or_tangent_apply(MA, const double *, const double *, const double *, const double *, double,
                     double *);
void or_mass_apply(MA, double, const double *, double *);
int or_tangent_diag(MA, const double *, const double *, const double *, double, double *);
double or_strain_energy(MA, const double *, const double *, const double *);
int main(void) {
  for (int P = 1; P <= 3; P++) {
    int Q = P + 2, n = P + 1, nx = 2, ny = 1, nz = 2;
    double h[3] = {0.5, 1.0, 0.5};
    double *B = malloc(sizeof(double) * Q * n), *D = malloc(sizeof(double) * Q * n);
    double *w = malloc(sizeof(double) * Q);
    for (int q = 0; q < Q; q++) {
      double x = -1.0 + 2.0 * (q + 0.5) / Q;
      w[q] = 2.0 / Q;
      for (int a = 0; a < n; a++) {  /* any smooth table exercises the loops */
        B[q * n + a] = pow(0.5 * (1.0 + x), a) * pow(0.5 * (1.0 - x), P - a);
        D[q * n + a] = 0.1 * (a + 1) * x;
      }
    }
    int64_t Nn = or_num_nodes(nx, ny, nz, P);
    int E = nx * ny * nz;
    int32_t *g = malloc(sizeof(int32_t) * E * n * n * n);
    or_gather_map(nx, ny, nz, P, g);
    double *u = calloc(3 * Nn, sizeof(double)), *v = malloc(sizeof(double) * 3 * Nn);
    double *y = calloc(3 * Nn, sizeof(double)), *mu = malloc(sizeof(double) * E);
    double *lam = malloc(sizeof(double) * E);
    for (int i = 0; i < 3 * Nn; i++) v[i] = sin(0.37 * i);
    for (int e = 0; e < E; e++) { mu[e] = 384.6; lam[e] = 576.9; }
    if (or_internal_force(nx, ny, nz, P, Q, h, B, D, w, mu, lam, u, y)) return 1;
    if (or_tangent_apply(nx, ny, nz, P, Q, h, B, D, w, mu, lam, u, v, 3.0, y)) return 2;
    or_mass_apply(nx, ny, nz, P, Q, h, B, D, w, 1.5, v, y);
    if (or_tangent_diag(nx, ny, nz, P, Q, h, B, D, w, mu, lam, u, 3.0, y)) return 3;
    (void)or_strain_energy(nx, ny, nz, P, Q, h, B, D, w, mu, lam, u);
    free(B); free(D); free(w); free(g); free(u); free(v); free(y); free(mu); free(lam);
  }
  printf("ok\n");
  return 0;
}
"""


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                    reason="needs the host compilers")
def test_host_basis_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "driver.cpp")
        open(src, "w").write(BASIS_DRIVER)
        exe = os.path.join(d, "basis_san")
        _run(["g++", "-std=c++17"] + SAN +
             ["-I" + os.path.join(ROOT, "include"),
              "-I" + os.path.join(ROOT, "paper_2104_13466_amd", "csrc"),
              os.path.join(ROOT, "paper_2104_13466_amd", "csrc", "basis.cpp"), src, "-o", exe], d)
        assert "ok" in _run([exe], d)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs the host compiler")
def test_oracle_operators_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "driver.c")
        open(src, "w").write(FEM_DRIVER)
        exe = os.path.join(d, "fem_san")
        _run(["gcc", "-std=c11"] + SAN + [os.path.join(ROOT, "oracle", "fem.c"), src, "-o", exe,
                                          "-lm"], d)
        assert "ok" in _run([exe], d)
