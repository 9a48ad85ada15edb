// Static condensation of the element-interior modes (Section 4: the Schur
// complement of the element-interior block, Eqs. Eq:Matrix_form_schur1,
// Schur_split1/2 and Eq:Newmark_Matrix_form_schur1), FP64.
//
// Interior modes of an element are those whose three tensor indices are all
// internal (1..P-1 in slot order); in the structured numbering each lies on
// a slot (ex P + a, ey P + b, ez P + c) that belongs to that element alone.
// Interior index of an element: l = i m + alpha, i the component, alpha =
// ((c-1)(P-1) + (b-1))(P-1) + (a-1), m = (P-1)^3.
//
//  - k_interior_block: the interior block of K_T + s M of every element from
//    the stored linearisation (F^-1, mu - lam ln J) by its definition at the
//    Gauss points (dense, nI x nI, nI = 3 m);
//  - k_interior_invert: its inverse in place (Gauss-Jordan; the block is
//    symmetric positive definite, so no pivoting), a flag on a non-positive
//    pivot;
//  - k_interior_apply: y_I = scale * inv(K_II) t_I per element, gathered from
//    and scattered to the interior slots of global vectors;
//  - k_interior_set: a value on every interior slot of a vector.
#include <hip/hip_runtime.h>

#include "sdme_device.h"
#include "sdme_launch.h"

namespace sdme {

namespace {

constexpr int CT = 256;  // threads per block

__device__ __forceinline__ void elem_coords(const MeshK<double> &m, int e, int &ex, int &ey,
                                            int &ez) {
  ex = e % m.nx;
  ey = (e / m.nx) % m.ny;
  ez = e / (m.nx * m.ny);
}

// global slot of interior function alpha of element (ex, ey, ez)
__device__ __forceinline__ int64_t interior_slot(const MeshK<double> &m, int P, int ex, int ey,
                                                 int ez, int alpha) {
  const int pm = P - 1;
  const int a = alpha % pm + 1, b = (alpha / pm) % pm + 1, c = alpha / (pm * pm) + 1;
  return ((int64_t)(ez * P + c) * m.Ny + (ey * P + b)) * m.Nx + (ex * P + a);
}

// K_II[(i,al),(j,be)] = sum_q w_q detJ [mu d_ij g_al.g_be + c1 t_al,j t_be,i
//   + lam t_al,i t_be,j + s rho d_ij N_al N_be], t = G^T g (G = F^-1): the
// derivative of dP = mu dF + c1 (G dF G)^T + lam tr(G dF) G^T contracted
// with the shape-function gradients g.
__global__ __launch_bounds__(CT) void k_interior_block(MeshK<double> m, int P, const double *mu,
                                                       const double *lam, const double *state,
                                                       double msr, double *__restrict__ Kii) {
  const int e = blockIdx.x;
  const int n = P + 1, Q = m.Q, pm = P - 1, mI = pm * pm * pm, nI = 3 * mI, QQQ = Q * Q * Q;
  extern __shared__ double sh[];
  double *sg = sh;               // [mI][3] gradients at the current point
  double *st = sg + 3 * mI;      // [mI][3] G^T g
  double *sv = st + 3 * mI;      // [mI] values
  double *sG = sv + mI;          // [10] state at the point
  const double *B = m.tab, *D = m.tab + Q * n, *W = m.tab + 2 * Q * n;
  // without a state only the mass term remains (interior block of s rho M)
  const double mue = state ? mu[e] : 0.0, lae = state ? lam[e] : 0.0;
  // each thread accumulates the 3 x 3 component blocks of up to MAXPAIR pairs
  // (al, be) per sweep over the Gauss points (one sweep for P <= 4)
  constexpr int MAXPAIR = 3;
  const double *se = state ? state + (size_t)e * 10 * QQQ : nullptr;
  double *Ke = Kii + (size_t)e * nI * nI;
  for (int p0 = 0; p0 < mI * mI; p0 += CT * MAXPAIR) {
    double acc[MAXPAIR][9];
#pragma unroll
    for (int k = 0; k < MAXPAIR; k++)
#pragma unroll
      for (int t = 0; t < 9; t++) acc[k][t] = 0.0;
    for (int q = 0; q < QQQ; q++) {
      const int q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
      if (threadIdx.x < 10) sG[threadIdx.x] = state ? se[threadIdx.x * QQQ + q] : 0.0;
      __syncthreads();
      for (int al = threadIdx.x; al < mI; al += CT) {
        const int a = al % pm + 1, b = (al / pm) % pm + 1, c = al / (pm * pm) + 1;
        const double b1 = B[q1 * n + a], b2 = B[q2 * n + b], b3 = B[q3 * n + c];
        const double g0 = D[q1 * n + a] * b2 * b3 * m.ih[0],
                     g1 = b1 * D[q2 * n + b] * b3 * m.ih[1],
                     g2 = b1 * b2 * D[q3 * n + c] * m.ih[2];
        sg[3 * al] = g0;
        sg[3 * al + 1] = g1;
        sg[3 * al + 2] = g2;
        for (int k = 0; k < 3; k++)  // (G^T g)_k = sum_J G_Jk g_J
          st[3 * al + k] = sG[0 * 3 + k] * g0 + sG[1 * 3 + k] * g1 + sG[2 * 3 + k] * g2;
        sv[al] = b1 * b2 * b3;
      }
      __syncthreads();
      const double wq = W[q1] * W[q2] * W[q3] * m.detJ;
      const double wmu = wq * mue, wc1 = wq * sG[9], wla = wq * lae, wm = wq * msr;
#pragma unroll
      for (int k = 0; k < MAXPAIR; k++) {
        const int pr = p0 + threadIdx.x + k * CT;
        if (pr < mI * mI) {
          const int al = pr / mI, be = pr % mI;
          const double gg = sg[3 * al] * sg[3 * be] + sg[3 * al + 1] * sg[3 * be + 1] +
                            sg[3 * al + 2] * sg[3 * be + 2];
          const double diag = wmu * gg + wm * sv[al] * sv[be];
#pragma unroll
          for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
              acc[k][i * 3 + j] += (i == j ? diag : 0.0) + wc1 * st[3 * al + j] * st[3 * be + i] +
                                   wla * st[3 * al + i] * st[3 * be + j];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < MAXPAIR; k++) {
      const int pr = p0 + threadIdx.x + k * CT;
      if (pr < mI * mI) {
        const int al = pr / mI, be = pr % mI;
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++)
            Ke[(size_t)(i * mI + al) * nI + j * mI + be] = acc[k][i * 3 + j];
      }
    }
  }
}

// In-place Gauss-Jordan inverse of each element's nI x nI block (in LDS when
// it fits, else in place in global memory).
template <bool LDS>
__global__ __launch_bounds__(CT) void k_interior_invert(int nI, double *__restrict__ Kii,
                                                        int *flag) {
  extern __shared__ double sh[];
  double *Kg = Kii + (size_t)blockIdx.x * nI * nI;
  double *A = LDS ? sh : Kg;
  if (LDS) {
    for (int i = threadIdx.x; i < nI * nI; i += CT) A[i] = Kg[i];
    __syncthreads();
  }
  __shared__ double s_p;
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  for (int k = 0; k < nI; k++) {
    if (threadIdx.x == 0) {
      const double p = A[(size_t)k * nI + k];
      if (!(p > 0.0)) s_bad = 1;
      s_p = (p > 0.0) ? 1.0 / p : 0.0;
    }
    __syncthreads();
    const double ip = s_p;
    // row k scaled (its pivot entry becomes 1 / p)
    for (int j = threadIdx.x; j < nI; j += CT) {
      const size_t kj = (size_t)k * nI + j;
      A[kj] = (j == k) ? ip : A[kj] * ip;
    }
    __syncthreads();
    // eliminate column k from the other rows
    for (int idx = threadIdx.x; idx < nI * nI; idx += CT) {
      const int r = idx / nI, j = idx % nI;
      if (r == k) continue;
      const double f = A[(size_t)r * nI + k];
      if (j == k)
        continue;
      A[(size_t)r * nI + j] -= f * A[(size_t)k * nI + j];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nI; r += CT)
      if (r != k) A[(size_t)r * nI + k] = -A[(size_t)r * nI + k] * ip;
    __syncthreads();
  }
  if (LDS)
    for (int i = threadIdx.x; i < nI * nI; i += CT) Kg[i] = A[i];
  if (threadIdx.x == 0 && s_bad) atomicOr(flag, 1);
}

// y_I = scale inv(K_II) t_I on the interior slots of every element (each
// interior slot belongs to one element: plain stores).
__global__ __launch_bounds__(CT) void k_interior_apply(MeshK<double> m, int P,
                                                       const double *__restrict__ Kinv,
                                                       const double *__restrict__ t,
                                                       double *__restrict__ y, double scale,
                                                       const int *__restrict__ skip) {
  if (skip && *skip) return;
  const int e = blockIdx.x;
  const int pm = P - 1, mI = pm * pm * pm, nI = 3 * mI;
  extern __shared__ double sh[];
  int ex, ey, ez;
  elem_coords(m, e, ex, ey, ez);
  for (int l = threadIdx.x; l < nI; l += CT) {
    const int i = l / mI, al = l % mI;
    sh[l] = t[(int64_t)i * m.Nn + interior_slot(m, P, ex, ey, ez, al)];
  }
  __syncthreads();
  const double *A = Kinv + (size_t)e * nI * nI;
  for (int r = threadIdx.x; r < nI; r += CT) {
    double s = 0.0;
    for (int j = 0; j < nI; j++) s += A[(size_t)j * nI + r] * sh[j];  // symmetric
    const int i = r / mI, al = r % mI;
    y[(int64_t)i * m.Nn + interior_slot(m, P, ex, ey, ez, al)] = scale * s;
  }
}

__global__ __launch_bounds__(CT) void k_interior_set(MeshK<double> m, int P, double *x,
                                                     double val, const int *__restrict__ skip) {
  if (skip && *skip) return;
  const int64_t n = 3 * (int64_t)m.Nn;
  for (int64_t idx = blockIdx.x * (int64_t)CT + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * CT) {
    const int64_t g = idx % m.Nn;
    const int ix = (int)(g % m.Nx), iy = (int)((g / m.Nx) % m.Ny), iz = (int)(g / ((int64_t)m.Nx * m.Ny));
    if (ix % P != 0 && iy % P != 0 && iz % P != 0) x[idx] = val;
  }
}

}  // namespace

int interior_size(int P) { return P < 2 ? 0 : 3 * (P - 1) * (P - 1) * (P - 1); }

int launch_interior_block(int P, const MeshK<double> &m, const double *mu, const double *lam,
                          const double *state, double msr, double *Kii, hipStream_t st) {
  const int mI = interior_size(P) / 3;
  if (mI == 0) return 0;
  const size_t sh = sizeof(double) * (7 * mI + 10);
  hipLaunchKernelGGL(k_interior_block, dim3(m.E), dim3(CT), sh, st, m, P, mu, lam, state, msr,
                     Kii);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_interior_invert(int P, int E, double *Kii, int *flag, hipStream_t st) {
  const int nI = interior_size(P);
  if (nI == 0) return 0;
  const size_t sh = sizeof(double) * (size_t)nI * nI;
  if (sh <= 64 * 1024)
    hipLaunchKernelGGL(k_interior_invert<true>, dim3(E), dim3(CT), sh, st, nI, Kii, flag);
  else
    hipLaunchKernelGGL(k_interior_invert<false>, dim3(E), dim3(CT), 0, st, nI, Kii, flag);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_interior_apply(int P, const MeshK<double> &m, const double *Kinv, const double *t,
                          double *y, double scale, const int *skip, hipStream_t st) {
  const int nI = interior_size(P);
  if (nI == 0) return 0;
  hipLaunchKernelGGL(k_interior_apply, dim3(m.E), dim3(CT), sizeof(double) * nI, st, m, P, Kinv, t,
                     y, scale, skip);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_interior_set(int P, const MeshK<double> &m, double *x, double val, const int *skip,
                        hipStream_t st) {
  if (P < 2) return 0;
  int64_t n = 3 * (int64_t)m.Nn;
  int64_t b = (n + CT - 1) / CT;
  hipLaunchKernelGGL(k_interior_set, dim3((int)(b < 4096 ? b : 4096)), dim3(CT), 0, st, m, P, x,
                     val, skip);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sdme
