/*
 * ORACLE -- test infrastructure only.  Plain, slow, direct FP64 element loops
 * for the operators of Section 3 (weak form) and Section 4 (non-linear
 * elastodynamics).  Only tests/, the smoke check and the benchmark's CPU
 * baseline leg load this file's shared object; the product library never does,
 * and this file shares no code with it.
 *
 * Every element quantity is evaluated from its definition: the displacement
 * gradient at a Gauss point is the sum over all (P+1)^3 tensor-product shape
 * functions N_l = phi_a(xi1) phi_b(xi2) phi_c(xi3) (Eq. ProdTensorialHexaedro)
 * times the element coefficients (Eq. interpolacao u); integrals are the plain
 * Gauss sums.  No sum factorisation, no fusion.
 *
 * Mesh: structured box of nx*ny*nz hexahedra with edge lengths hx, hy, hz
 * (affine map, constant Jacobian diag(h/2)).  Global slot grid with
 * Nd = nd*P+1 slots per direction, numbered x-fastest; vectors are SoA
 * [3][Nn].  Element e = (ez*ny+ey)*nx+ex, local mode l = (c*n+b)*n+a.
 *
 * Material: compressible neo-Hookean (Eq. hyperelastic strain energy,
 * Eq. second Piola-Kirchhoff relation) with per-element Lame parameters.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- 3x3 algebra */
static double det3(const double *A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
static void inv3(const double *A, double *Ai) {
  double d = det3(A);
  Ai[0] = (A[4] * A[8] - A[5] * A[7]) / d;
  Ai[1] = (A[2] * A[7] - A[1] * A[8]) / d;
  Ai[2] = (A[1] * A[5] - A[2] * A[4]) / d;
  Ai[3] = (A[5] * A[6] - A[3] * A[8]) / d;
  Ai[4] = (A[0] * A[8] - A[2] * A[6]) / d;
  Ai[5] = (A[2] * A[3] - A[0] * A[5]) / d;
  Ai[6] = (A[3] * A[7] - A[4] * A[6]) / d;
  Ai[7] = (A[1] * A[6] - A[0] * A[7]) / d;
  Ai[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}
static void mul3(const double *A, const double *B, double *C) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0;
      for (int k = 0; k < 3; k++) s += A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}
static void tr3(const double *A, double *At) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) At[j * 3 + i] = A[i * 3 + j];
}

/* ------------------------------------------------------- neo-Hookean material */
/* Right Cauchy-Green C = F^T F, J = det F, S = mu (I - C^-1) + lam lnJ C^-1,
 * first Piola-Kirchhoff P = F S.  Returns J. */
static double nh_first_pk(const double *F, double mu, double lam, double *Pk) {
  double Ft[9], C[9], Ci[9], S[9];
  tr3(F, Ft);
  mul3(Ft, F, C);
  inv3(C, Ci);
  double J = det3(F);
  double lnJ = log(J);
  for (int i = 0; i < 9; i++) S[i] = -mu * Ci[i] + lam * lnJ * Ci[i];
  S[0] += mu; S[4] += mu; S[8] += mu;
  mul3(F, S, Pk);
  return J;
}

/* Strain energy density Psi = mu/2 (tr C - 3) - mu lnJ + lam/2 (lnJ)^2. */
static double nh_energy(const double *F, double mu, double lam) {
  double trC = 0;
  for (int i = 0; i < 9; i++) trC += F[i] * F[i];
  double lnJ = log(det3(F));
  return 0.5 * mu * (trC - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
}

/* Directional derivative of P = F S in the direction dF (linearisation of the
 * internal virtual work, Section 3): dP = dF S + F dS with
 * dE = (dF^T F + F^T dF)/2,  dS = lam (C^-1 : dE) C^-1 + 2 (mu - lam lnJ) C^-1 dE C^-1. */
static void nh_dP(const double *F, const double *dF, double mu, double lam, double *dP) {
  double Ft[9], C[9], Ci[9], S[9], dFt[9], t1[9], t2[9], dE[9], tmp[9], CdEC[9], dS[9];
  tr3(F, Ft);
  mul3(Ft, F, C);
  inv3(C, Ci);
  double lnJ = log(det3(F));
  for (int i = 0; i < 9; i++) S[i] = -mu * Ci[i] + lam * lnJ * Ci[i];
  S[0] += mu; S[4] += mu; S[8] += mu;
  tr3(dF, dFt);
  mul3(dFt, F, t1);
  mul3(Ft, dF, t2);
  for (int i = 0; i < 9; i++) dE[i] = 0.5 * (t1[i] + t2[i]);
  double CidE = 0;
  for (int i = 0; i < 9; i++) CidE += Ci[i] * dE[i];
  mul3(Ci, dE, tmp);
  mul3(tmp, Ci, CdEC);
  for (int i = 0; i < 9; i++) dS[i] = lam * CidE * Ci[i] + 2.0 * (mu - lam * lnJ) * CdEC[i];
  mul3(dF, S, t1);
  mul3(F, dS, t2);
  for (int i = 0; i < 9; i++) dP[i] = t1[i] + t2[i];
}

/* ----------------------------------------------------------------- mesh data */
typedef struct {
  int nx, ny, nz, P, Q;
  double h[3];
  int n, n3, q3;
  int64_t Nx, Ny, Nz, Nn, E;
  double detJ;
  /* per (qp, mode): value N and reference-to-physical gradient dN/dX */
  double *N, *G;
  double *wq; /* tensor weight w1*w2*w3 per qp */
} mesh_t;

static void mesh_init(mesh_t *m, int nx, int ny, int nz, int P, int Q, const double *h,
                      const double *B, const double *D, const double *w) {
  m->nx = nx; m->ny = ny; m->nz = nz; m->P = P; m->Q = Q;
  m->h[0] = h[0]; m->h[1] = h[1]; m->h[2] = h[2];
  m->n = P + 1;
  m->n3 = m->n * m->n * m->n;
  m->q3 = Q * Q * Q;
  m->Nx = (int64_t)nx * P + 1; m->Ny = (int64_t)ny * P + 1; m->Nz = (int64_t)nz * P + 1;
  m->Nn = m->Nx * m->Ny * m->Nz;
  m->E = (int64_t)nx * ny * nz;
  m->detJ = h[0] * h[1] * h[2] / 8.0;
  int n = m->n;
  m->N = (double *)malloc(sizeof(double) * m->q3 * m->n3);
  m->G = (double *)malloc(sizeof(double) * m->q3 * m->n3 * 3);
  m->wq = (double *)malloc(sizeof(double) * m->q3);
  for (int q3 = 0; q3 < Q; q3++)
    for (int q2 = 0; q2 < Q; q2++)
      for (int q1 = 0; q1 < Q; q1++) {
        int q = (q3 * Q + q2) * Q + q1;
        m->wq[q] = w[q1] * w[q2] * w[q3];
        for (int c = 0; c < n; c++)
          for (int b = 0; b < n; b++)
            for (int a = 0; a < n; a++) {
              int l = (c * n + b) * n + a;
              double Ba = B[q1 * n + a], Bb = B[q2 * n + b], Bc = B[q3 * n + c];
              double Da = D[q1 * n + a], Db = D[q2 * n + b], Dc = D[q3 * n + c];
              m->N[(size_t)q * m->n3 + l] = Ba * Bb * Bc;
              double *g = m->G + ((size_t)q * m->n3 + l) * 3;
              g[0] = Da * Bb * Bc * 2.0 / h[0];
              g[1] = Ba * Db * Bc * 2.0 / h[1];
              g[2] = Ba * Bb * Dc * 2.0 / h[2];
            }
      }
}
static void mesh_free(mesh_t *m) { free(m->N); free(m->G); free(m->wq); }

/* Global slot of local mode (a,b,c) of element (ex,ey,ez). */
static int64_t slot_of(const mesh_t *m, int64_t e, int l) {
  int n = m->n, P = m->P;
  int64_t ex = e % m->nx, ey = (e / m->nx) % m->ny, ez = e / ((int64_t)m->nx * m->ny);
  int a = l % n, b = (l / n) % n, c = l / (n * n);
  return ((ez * P + c) * m->Ny + (ey * P + b)) * m->Nx + (ex * P + a);
}

int64_t or_num_nodes(int nx, int ny, int nz, int P) {
  return ((int64_t)nx * P + 1) * ((int64_t)ny * P + 1) * ((int64_t)nz * P + 1);
}

/* Element-to-global map, out[e*(P+1)^3 + l]. */
void or_gather_map(int nx, int ny, int nz, int P, int32_t *out) {
  mesh_t m;
  memset(&m, 0, sizeof(m));
  m.nx = nx; m.ny = ny; m.nz = nz; m.P = P; m.n = P + 1; m.n3 = m.n * m.n * m.n;
  m.Nx = (int64_t)nx * P + 1; m.Ny = (int64_t)ny * P + 1; m.Nz = (int64_t)nz * P + 1;
  m.E = (int64_t)nx * ny * nz;
  for (int64_t e = 0; e < m.E; e++)
    for (int l = 0; l < m.n3; l++) out[e * m.n3 + l] = (int32_t)slot_of(&m, e, l);
}

static void gather(const mesh_t *m, int64_t e, const double *v, double *ve) {
  for (int i = 0; i < 3; i++)
    for (int l = 0; l < m->n3; l++) ve[i * m->n3 + l] = v[i * m->Nn + slot_of(m, e, l)];
}

/* Serial assembly of element vectors (deterministic). */
static void assemble(const mesh_t *m, const double *ev, double *y) {
  memset(y, 0, sizeof(double) * 3 * m->Nn);
  for (int64_t e = 0; e < m->E; e++)
    for (int i = 0; i < 3; i++)
      for (int l = 0; l < m->n3; l++)
        y[i * m->Nn + slot_of(m, e, l)] += ev[(e * 3 + i) * m->n3 + l];
}

/* Deformation gradient F = I + sum_l u_l (x) dN_l/dX at qp. */
static void def_grad(const mesh_t *m, int q, const double *ue, double *F) {
  for (int i = 0; i < 9; i++) F[i] = 0;
  for (int l = 0; l < m->n3; l++) {
    const double *g = m->G + ((size_t)q * m->n3 + l) * 3;
    for (int i = 0; i < 3; i++) {
      double ul = ue[i * m->n3 + l];
      for (int J = 0; J < 3; J++) F[i * 3 + J] += ul * g[J];
    }
  }
  F[0] += 1; F[4] += 1; F[8] += 1;
}

#define MESH_ARGS int nx, int ny, int nz, int P, int Q, const double *h, const double *B, \
                  const double *D, const double *w

/* Internal force R_{l,i} = sum_q w_q detJ P_iJ dN_l/dX_J (second term of the
 * virtual work, Eq. material virtual work).  Returns the number of Gauss points
 * with det F <= 0 (R is then not meaningful). */
int or_internal_force(MESH_ARGS, const double *mu, const double *lam, const double *u,
                      double *R) {
  mesh_t m;
  mesh_init(&m, nx, ny, nz, P, Q, h, B, D, w);
  double *ev = (double *)calloc((size_t)m.E * 3 * m.n3, sizeof(double));
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t e = 0; e < m.E; e++) {
    double *ue = (double *)malloc(sizeof(double) * 3 * m.n3);
    double *re = ev + (size_t)e * 3 * m.n3;
    gather(&m, e, u, ue);
    for (int q = 0; q < m.q3; q++) {
      double F[9], Pk[9];
      def_grad(&m, q, ue, F);
      if (det3(F) <= 0) { bad++; continue; }
      nh_first_pk(F, mu[e], lam[e], Pk);
      double s = m.wq[q] * m.detJ;
      for (int l = 0; l < m.n3; l++) {
        const double *g = m.G + ((size_t)q * m.n3 + l) * 3;
        for (int i = 0; i < 3; i++)
          re[i * m.n3 + l] += s * (Pk[i * 3] * g[0] + Pk[i * 3 + 1] * g[1] + Pk[i * 3 + 2] * g[2]);
      }
    }
    free(ue);
  }
  assemble(&m, ev, R);
  free(ev);
  mesh_free(&m);
  return bad;
}

/* y = K_T(u_lin) v + cm * M v  with K_T the derivative of R (linearisation,
 * Eq. directional derivative / effective stiffness) and M the consistent mass
 * int N_l N_m (cm = mass_shift * rho, e.g. b1 rho for the Newmark matrix
 * b1 M + K_T). */
int or_tangent_apply(MESH_ARGS, const double *mu, const double *lam, const double *ulin,
                     const double *v, double cm, double *y) {
  mesh_t m;
  mesh_init(&m, nx, ny, nz, P, Q, h, B, D, w);
  double *ev = (double *)calloc((size_t)m.E * 3 * m.n3, sizeof(double));
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t e = 0; e < m.E; e++) {
    double *ue = (double *)malloc(sizeof(double) * 6 * m.n3);
    double *ve = ue + 3 * m.n3;
    double *ye = ev + (size_t)e * 3 * m.n3;
    gather(&m, e, ulin, ue);
    gather(&m, e, v, ve);
    for (int q = 0; q < m.q3; q++) {
      double F[9], dF[9], dP[9], vq[3] = {0, 0, 0};
      def_grad(&m, q, ue, F);
      if (det3(F) <= 0) { bad++; continue; }
      def_grad(&m, q, ve, dF);
      dF[0] -= 1; dF[4] -= 1; dF[8] -= 1;
      for (int l = 0; l < m.n3; l++) {
        double Nl = m.N[(size_t)q * m.n3 + l];
        for (int i = 0; i < 3; i++) vq[i] += Nl * ve[i * m.n3 + l];
      }
      nh_dP(F, dF, mu[e], lam[e], dP);
      double s = m.wq[q] * m.detJ;
      for (int l = 0; l < m.n3; l++) {
        const double *g = m.G + ((size_t)q * m.n3 + l) * 3;
        double Nl = m.N[(size_t)q * m.n3 + l];
        for (int i = 0; i < 3; i++)
          ye[i * m.n3 + l] += s * (dP[i * 3] * g[0] + dP[i * 3 + 1] * g[1] + dP[i * 3 + 2] * g[2] +
                                   cm * Nl * vq[i]);
      }
    }
    free(ue);
  }
  assemble(&m, ev, y);
  free(ev);
  mesh_free(&m);
  return bad;
}

/* y = rho M v, M the consistent mass int N_l N_m dOmega (inertia term). */
void or_mass_apply(MESH_ARGS, double rho, const double *v, double *y) {
  mesh_t m;
  mesh_init(&m, nx, ny, nz, P, Q, h, B, D, w);
  double *ev = (double *)calloc((size_t)m.E * 3 * m.n3, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m.E; e++) {
    double *ve = (double *)malloc(sizeof(double) * 3 * m.n3);
    double *ye = ev + (size_t)e * 3 * m.n3;
    gather(&m, e, v, ve);
    for (int q = 0; q < m.q3; q++) {
      double vq[3] = {0, 0, 0};
      for (int l = 0; l < m.n3; l++)
        for (int i = 0; i < 3; i++) vq[i] += m.N[(size_t)q * m.n3 + l] * ve[i * m.n3 + l];
      double s = rho * m.wq[q] * m.detJ;
      for (int l = 0; l < m.n3; l++)
        for (int i = 0; i < 3; i++) ye[i * m.n3 + l] += s * m.N[(size_t)q * m.n3 + l] * vq[i];
    }
    free(ve);
  }
  assemble(&m, ev, y);
  free(ev);
  mesh_free(&m);
}

/* Diagonal of K_T(u_lin) + cm M: for each global DOF (l,i) the sum over
 * elements of e_(l,i)^T K_e e_(l,i), with K_e applied to the unit vector by the
 * same directional derivative as or_tangent_apply. */
int or_tangent_diag(MESH_ARGS, const double *mu, const double *lam, const double *ulin,
                    double cm, double *d) {
  mesh_t m;
  mesh_init(&m, nx, ny, nz, P, Q, h, B, D, w);
  double *ev = (double *)calloc((size_t)m.E * 3 * m.n3, sizeof(double));
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t e = 0; e < m.E; e++) {
    double *ue = (double *)malloc(sizeof(double) * 3 * m.n3);
    double *de = ev + (size_t)e * 3 * m.n3;
    gather(&m, e, ulin, ue);
    for (int q = 0; q < m.q3; q++) {
      double F[9];
      def_grad(&m, q, ue, F);
      if (det3(F) <= 0) { bad++; continue; }
      double s = m.wq[q] * m.detJ;
      for (int l = 0; l < m.n3; l++) {
        const double *g = m.G + ((size_t)q * m.n3 + l) * 3;
        double Nl = m.N[(size_t)q * m.n3 + l];
        for (int i = 0; i < 3; i++) {
          double dF[9] = {0}, dP[9];
          for (int J = 0; J < 3; J++) dF[i * 3 + J] = g[J];
          nh_dP(F, dF, mu[e], lam[e], dP);
          de[i * m.n3 + l] += s * (dP[i * 3] * g[0] + dP[i * 3 + 1] * g[1] + dP[i * 3 + 2] * g[2] +
                                   cm * Nl * Nl);
        }
      }
    }
    free(ue);
  }
  assemble(&m, ev, d);
  free(ev);
  mesh_free(&m);
  return bad;
}

/* Stored strain energy sum_e sum_q w_q detJ Psi(F). */
double or_strain_energy(MESH_ARGS, const double *mu, const double *lam, const double *u) {
  mesh_t m;
  mesh_init(&m, nx, ny, nz, P, Q, h, B, D, w);
  double tot = 0;
#pragma omp parallel for schedule(static) reduction(+ : tot)
  for (int64_t e = 0; e < m.E; e++) {
    double *ue = (double *)malloc(sizeof(double) * 3 * m.n3);
    gather(&m, e, u, ue);
    for (int q = 0; q < m.q3; q++) {
      double F[9];
      def_grad(&m, q, ue, F);
      tot += m.wq[q] * m.detJ * nh_energy(F, mu[e], lam[e]);
    }
    free(ue);
  }
  mesh_free(&m);
  return tot;
}

/* Sensitivity of the internal force to the element Lame parameters, contracted
 * with a vector w:  g_mu[e] += scale * sum_q w_q detJ (dP/dmu)(F) : grad w,
 * g_lam[e] += scale * sum_q w_q detJ (dP/dlam)(F) : grad w, where
 * dP/dmu = F - F^-T and dP/dlam = lnJ F^-T (from P = F S, Eq. second
 * Piola-Kirchhoff relation). */
void or_material_grad(MESH_ARGS, const double *u, const double *wv, double scale,
                      double *g_mu, double *g_lam) {
  mesh_t m;
  mesh_init(&m, nx, ny, nz, P, Q, h, B, D, w);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m.E; e++) {
    double *ue = (double *)malloc(sizeof(double) * 6 * m.n3);
    double *we = ue + 3 * m.n3;
    gather(&m, e, u, ue);
    gather(&m, e, wv, we);
    double gm = 0, gl = 0;
    for (int q = 0; q < m.q3; q++) {
      double F[9], Gw[9], Fi[9], FiT[9];
      def_grad(&m, q, ue, F);
      def_grad(&m, q, we, Gw);
      Gw[0] -= 1; Gw[4] -= 1; Gw[8] -= 1;
      inv3(F, Fi);
      tr3(Fi, FiT);
      double lnJ = log(det3(F));
      double s = m.wq[q] * m.detJ, am = 0, al = 0;
      for (int k = 0; k < 9; k++) {
        am += (F[k] - FiT[k]) * Gw[k];
        al += lnJ * FiT[k] * Gw[k];
      }
      gm += s * am;
      gl += s * al;
    }
    g_mu[e] += scale * gm;
    g_lam[e] += scale * gl;
    free(ue);
  }
  mesh_free(&m);
}

/* Face index: 0 x=0, 1 x=max, 2 y=0, 3 y=max, 4 z=0, 5 z=max.  Surface
 * quadrature on the reference face with nq Gauss points per direction; Bf is the
 * 1D basis at those points [nq][P+1], wf the weights. */
static void face_setup(const mesh_t *m, int face, int *dir, int *t1, int *t2, int *side) {
  *dir = face / 2;
  *side = face % 2;
  *t1 = (*dir == 0) ? 1 : 0;
  *t2 = (*dir == 2) ? 1 : 2;
  (void)m;
}

/* Dead traction t (reference configuration, total Lagrangian) on a box face:
 * f_{l,i} += int_face N_l t_i dA (external work term of Eq. material virtual
 * work). */
void or_face_traction(MESH_ARGS, int face, const double *t, int nq, const double *Bf,
                      const double *wf, double *f) {
  mesh_t m;
  mesh_init(&m, nx, ny, nz, P, Q, h, B, D, w);
  int dir, t1, t2, side;
  face_setup(&m, face, &dir, &t1, &t2, &side);
  int n = m.n;
  int ne[3] = {nx, ny, nz};
  double dA = m.h[t1] * m.h[t2] / 4.0;
  for (int64_t e = 0; e < m.E; e++) {
    int64_t ei[3] = {e % nx, (e / nx) % ny, e / ((int64_t)nx * ny)};
    if (ei[dir] != (side ? ne[dir] - 1 : 0)) continue;
    for (int l = 0; l < m.n3; l++) {
      int li[3] = {l % n, (l / n) % n, l / (n * n)};
      if (li[dir] != (side ? P : 0)) continue; /* other modes vanish on the face */
      double s = 0;
      for (int i = 0; i < nq; i++)
        for (int j = 0; j < nq; j++)
          s += wf[i] * wf[j] * Bf[i * n + li[t1]] * Bf[j * n + li[t2]];
      int64_t g = slot_of(&m, e, l);
      for (int c = 0; c < 3; c++) f[c * m.Nn + g] += s * dA * t[c];
    }
  }
  mesh_free(&m);
}

/* Penalty contact with the rigid plane z = z0 (normal +z) on face z=0 of the
 * box: gap g = Z + u_z - z0 at the face Gauss points, contact pressure
 * eps * max(-g, 0) pushing in +z, f_{l,z} += int N_l eps max(-g,0) dA, and
 * energy += 1/2 eps int min(g,0)^2 dA.  Surface integration with nq Gauss
 * points per direction (P+1 in the paper's contact examples). */
double or_penalty_plane(MESH_ARGS, double eps, double z0, double origin_z, int nq,
                        const double *Bf, const double *wf, const double *u, double *f) {
  mesh_t m;
  mesh_init(&m, nx, ny, nz, P, Q, h, B, D, w);
  int n = m.n;
  double dA = m.h[0] * m.h[1] / 4.0, energy = 0;
  for (int64_t e = 0; e < (int64_t)nx * ny; e++) { /* ez = 0 layer */
    for (int i = 0; i < nq; i++)
      for (int j = 0; j < nq; j++) {
        double uz = 0;
        for (int b = 0; b < n; b++)
          for (int a = 0; a < n; a++) {
            int l = b * n + a; /* c = 0 */
            uz += Bf[i * n + a] * Bf[j * n + b] * u[2 * m.Nn + slot_of(&m, e, l)];
          }
        double gap = origin_z + uz - z0;
        if (gap >= 0) continue;
        double wgt = wf[i] * wf[j] * dA;
        energy += 0.5 * eps * gap * gap * wgt;
        for (int b = 0; b < n; b++)
          for (int a = 0; a < n; a++) {
            int l = b * n + a;
            f[2 * m.Nn + slot_of(&m, e, l)] += wgt * Bf[i * n + a] * Bf[j * n + b] * eps * (-gap);
          }
      }
  }
  mesh_free(&m);
  return energy;
}
