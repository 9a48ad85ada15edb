// Loads given at quadrature points, and the L2 error of a field, for the
// fabricated-solution problems of Section 5 (a body force and boundary
// tractions computed from a prescribed displacement field, Eq. of the
// material virtual work in Section 3):
//  - body load  f_a += sum_e sum_q w_q detJ N_a(X_q) b(X_q), b given at the
//    volume quadrature points of the mesh (Q per direction);
//  - face load  f_a += int_face N_a t dA, t given at the face Gauss points
//    (P+1 per direction, the rule of the contact face);
//  - squared L2 error per component, sum_e sum_q w_q detJ (u_h(X_q) - g(X_q))^2.
// Each element's three 1D contractions (transposed for the loads) run through
// LDS; one block per element (the loads) or a grid-stride over elements (the
// error, with per-block partial sums added in block order by a one-block
// kernel).  These run once per solve, not in the PCG loop.
#include <hip/hip_runtime.h>

#include "sdme_device.h"
#include "sdme_launch.h"

namespace sdme {

constexpr int NTL = 256;

// Slot of local (a, b, c) of element (ex, ey, ez) on the structured grid.
__device__ __forceinline__ size_t grid_slot(const MeshK<double> &m, int P, int ex, int ey, int ez,
                                            int a, int b, int c) {
  return ((size_t)(ez * P + c) * m.Ny + (ey * P + b)) * m.Nx + (ex * P + a);
}

template <int P, int Q>
__global__ __launch_bounds__(NTL) void k_body_load(MeshK<double> m, const double *__restrict__ bq,
                                                   double *__restrict__ f) {
  constexpr int n = P + 1, Q3 = Q * Q * Q;
  using Dm = Dims<P, Q, 8>;
  __shared__ double sB[Q * n], sW[Q];
  __shared__ double s0[3 * Q3];         // weighted b [c][q3][q2][q1], then [c][q3][b][a]
  __shared__ double s1[3 * Q * Q * n];  // [c][q3][q2][a]
  const int e = blockIdx.x;
  const int ex = e % m.nx, ey = (e / m.nx) % m.ny, ez = e / (m.nx * m.ny);
  for (int i = threadIdx.x; i < Q * n; i += NTL) sB[i] = m.tab[Dm::TB + i];
  for (int i = threadIdx.x; i < Q; i += NTL) sW[i] = m.tab[Dm::TW + i];
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * Q3; i += NTL) {
    const int c = i / Q3, q = i % Q3, q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
    s0[i] = bq[((size_t)c * m.E + e) * Q3 + q] * (sW[q1] * sW[q2] * sW[q3] * m.detJ);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * Q * Q * n; i += NTL) {
    const int a = i % n, r = i / n;  // r = (c Q + q3) Q + q2
    double acc = 0;
    for (int q1 = 0; q1 < Q; q1++) acc += sB[q1 * n + a] * s0[r * Q + q1];
    s1[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * Q * n * n; i += NTL) {
    const int a = i % n, b = (i / n) % n, r = i / (n * n);  // r = c Q + q3
    double acc = 0;
    for (int q2 = 0; q2 < Q; q2++) acc += sB[q2 * n + b] * s1[(r * Q + q2) * n + a];
    s0[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * n * n * n; i += NTL) {
    const int a = i % n, b = (i / n) % n, cc = (i / (n * n)) % n, c = i / (n * n * n);
    double acc = 0;
    for (int q3 = 0; q3 < Q; q3++) acc += sB[q3 * n + cc] * s0[((c * Q + q3) * n + b) * n + a];
    if (m.stage)  // ordered assembly: element vector, gathered afterwards
      m.stage[((size_t)e * 3 + c) * (n * n * n) + (cc * n + b) * n + a] = acc;
    else
      atomicAdd(&f[(size_t)c * m.Nn + grid_slot(m, P, ex, ey, ez, a, b, cc)], acc);
  }
}

// Face element fe of face `face` (index j ne[t1] + i as in the face kernels)
// and its local directions.
struct FaceGeo {
  int dir, side, t1, t2, ei[3];
  double dA;
};
__device__ __forceinline__ FaceGeo face_geo(const MeshK<double> &m, int face, int fe) {
  FaceGeo g;
  g.dir = face / 2;
  g.side = face % 2;
  g.t1 = g.dir == 0 ? 1 : 0;
  g.t2 = g.dir == 2 ? 1 : 2;
  const int ne[3] = {m.nx, m.ny, m.nz};
  g.ei[g.t1] = fe % ne[g.t1];
  g.ei[g.t2] = fe / ne[g.t1];
  g.ei[g.dir] = g.side ? ne[g.dir] - 1 : 0;
  const double hh[3] = {2.0 / m.ih[0], 2.0 / m.ih[1], 2.0 / m.ih[2]};
  g.dA = hh[g.t1] * hh[g.t2] / 4.0;
  return g;
}

template <int P>
__global__ __launch_bounds__(128) void k_face_load(MeshK<double> m, int face,
                                                   const double *__restrict__ t,
                                                   double *__restrict__ f) {
  constexpr int n = P + 1, nq = P + 1;
  __shared__ double s_t[3 * nq * nq];
  const double *Bf = m.tab + face_table_offset(n, m.Q), *Wf = Bf + n * n;
  const int fe = blockIdx.x, nfe = gridDim.x;
  const FaceGeo g = face_geo(m, face, fe);
  for (int i = threadIdx.x; i < 3 * nq * nq; i += blockDim.x) {
    const int c = i / (nq * nq), p = i % (nq * nq), pi = p % nq, pj = p / nq;
    s_t[i] = t[((size_t)c * nfe + fe) * nq * nq + p] * (Wf[pi] * Wf[pj] * g.dA);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int a = idx % n, b = idx / n;
    double acc[3] = {0, 0, 0};
    for (int pj = 0; pj < nq; pj++)
      for (int pi = 0; pi < nq; pi++) {
        const double N = Bf[pi * n + a] * Bf[pj * n + b];
#pragma unroll
        for (int c = 0; c < 3; c++) acc[c] += N * s_t[c * nq * nq + pj * nq + pi];
      }
    int li[3];
    li[g.t1] = a;
    li[g.t2] = b;
    li[g.dir] = g.side ? P : 0;
    const size_t s = grid_slot(m, P, g.ei[0], g.ei[1], g.ei[2], li[0], li[1], li[2]);
    if (m.stage) {  // ordered assembly: face-element vector, gathered afterwards
#pragma unroll
      for (int c = 0; c < 3; c++) m.stage[((size_t)fe * 3 + c) * n * n + idx] = acc[c];
    } else {
#pragma unroll
      for (int c = 0; c < 3; c++) atomicAdd(&f[(size_t)c * m.Nn + s], acc[c]);
    }
  }
}

template <int P, int Q>
__global__ __launch_bounds__(NTL) void k_l2_error(MeshK<double> m, const double *__restrict__ u,
                                                  const double *__restrict__ g,
                                                  double *__restrict__ partials) {
  constexpr int n = P + 1, Q3 = Q * Q * Q;
  using Dm = Dims<P, Q, 8>;
  __shared__ double sB[Q * n], sW[Q];
  __shared__ double s0[3 * n * Q * Q];  // coefficients [c][cc][b][a], then [c][cc][q2][q1]
  __shared__ double s1[3 * n * n * Q];  // [c][cc][b][q1]
  __shared__ double s_red[3][NTL / 64];
  for (int i = threadIdx.x; i < Q * n; i += NTL) sB[i] = m.tab[Dm::TB + i];
  for (int i = threadIdx.x; i < Q; i += NTL) sW[i] = m.tab[Dm::TW + i];
  double acc[3] = {0, 0, 0};
  for (int e = blockIdx.x; e < m.E; e += gridDim.x) {
    const int ex = e % m.nx, ey = (e / m.nx) % m.ny, ez = e / (m.nx * m.ny);
    __syncthreads();  // tables stored; the previous element's buffers consumed
    for (int i = threadIdx.x; i < 3 * n * n * n; i += NTL) {
      const int a = i % n, b = (i / n) % n, cc = (i / (n * n)) % n, c = i / (n * n * n);
      s0[i] = u[(size_t)c * m.Nn + grid_slot(m, P, ex, ey, ez, a, b, cc)];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * n * n * Q; i += NTL) {
      const int q1 = i % Q, r = i / Q;  // r = (c n + cc) n + b
      double v = 0;
      for (int a = 0; a < n; a++) v += sB[q1 * n + a] * s0[r * n + a];
      s1[i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * n * Q * Q; i += NTL) {
      const int q1 = i % Q, q2 = (i / Q) % Q, r = i / (Q * Q);  // r = c n + cc
      double v = 0;
      for (int b = 0; b < n; b++) v += sB[q2 * n + b] * s1[(r * n + b) * Q + q1];
      s0[i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * Q3; i += NTL) {
      const int c = i / Q3, q = i % Q3, q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
      double v = 0;
      for (int cc = 0; cc < n; cc++) v += sB[q3 * n + cc] * s0[((c * n + cc) * Q + q2) * Q + q1];
      const double d = v - g[((size_t)c * m.E + e) * Q3 + q];
      const double wq = sW[q1] * sW[q2] * sW[q3] * m.detJ;
      if (c == 0) acc[0] += wq * d * d;
      else if (c == 1) acc[1] += wq * d * d;
      else acc[2] += wq * d * d;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) s_red[c][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0;
    for (int w = 0; w < NTL / 64; w++) t += s_red[threadIdx.x][w];
    partials[3 * blockIdx.x + threadIdx.x] = t;
  }
}

// out[c] = sum over blocks b (in block order) of partials[3 b + c].
__global__ __launch_bounds__(64) void k_sum3(const double *__restrict__ partials, int nb,
                                             double *__restrict__ out) {
  if (threadIdx.x < 3) {
    double t = 0;
    for (int b = 0; b < nb; b++) t += partials[3 * b + threadIdx.x];
    out[threadIdx.x] = t;
  }
}

#define SDME_PSWITCH(X) \
  switch (P) {          \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) default : return -2; \
  }

int launch_body_load(int P, const MeshK<double> &m, const double *b, double *f, hipStream_t st) {
#define BL(p)                                                                                  \
  case p:                                                                                      \
    if (m.Q == p + 1)                                                                          \
      hipLaunchKernelGGL((k_body_load<p, p + 1>), dim3(m.E), dim3(NTL), 0, st, m, b, f);        \
    else                                                                                       \
      hipLaunchKernelGGL((k_body_load<p, p + 2>), dim3(m.E), dim3(NTL), 0, st, m, b, f);        \
    break;
  SDME_PSWITCH(BL)
#undef BL
  if (m.stage && launch_stage_gather_elem<double>(P, m, 0, f, st)) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_face_load(int P, const MeshK<double> &m, int face, const double *t, double *f,
                     hipStream_t st) {
  const int nfe = face_blocks(m, face);
#define FL(p)                                                                               \
  case p:                                                                                   \
    hipLaunchKernelGGL(k_face_load<p>, dim3(nfe), dim3(128), 0, st, m, face, t, f); \
    break;
  SDME_PSWITCH(FL)
#undef FL
  if (m.stage && launch_stage_gather_face(P, m, face, f, st)) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_l2_error(int P, const MeshK<double> &m, const double *u, const double *g,
                    double *partials, int max_blocks, double *out, hipStream_t st) {
  const int nb = m.E < max_blocks ? m.E : max_blocks;
#define LE(p)                                                                                  \
  case p:                                                                                      \
    if (m.Q == p + 1)                                                                          \
      hipLaunchKernelGGL((k_l2_error<p, p + 1>), dim3(nb), dim3(NTL), 0, st, m, u, g, partials); \
    else                                                                                       \
      hipLaunchKernelGGL((k_l2_error<p, p + 2>), dim3(nb), dim3(NTL), 0, st, m, u, g, partials); \
    break;
  SDME_PSWITCH(LE)
#undef LE
  hipLaunchKernelGGL(k_sum3, dim3(1), dim3(64), 0, st, partials, nb, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#undef SDME_PSWITCH

}  // namespace sdme
