// Element kernels of libsdme: matrix-free, sum-factorised evaluation on
// tensor-product hexahedra (Eq. ProdTensorialHexaedro) of
//  - the neo-Hookean internal force R(u) (internal virtual work, Section 3),
//  - the tangent action (K_T + s M) v (linearisation of the virtual work),
//  - the consistent mass action rho M v,
//  - the diagonal of K_T + s M (Jacobi preconditioner),
//  - the strain energy and the material sensitivities of R.
// Gradients at Gauss points are three 1D contractions with the basis value and
// derivative tables B, D; the transposed contractions assemble element vectors
// which are scatter-added to the global SoA vector with hardware FP atomics.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sdme_device.h"
#include "sdme_launch.h"

namespace sdme {

template <int P, int Q, typename T>
struct EK {
  using Dm = Dims<P, Q, (int)sizeof(T)>;
  static constexpr int n = Dm::n, n3 = Dm::n3, QQ = Dm::QQ, NE = Dm::NE, NT = Dm::NT;
  static constexpr int SA = Dm::SA, SB = Dm::SB, SE = Dm::SE, TS = Dm::TSIZE;
};

// Thread/element coordinates inside a block.
struct Slab {
  int le, t2, i1, i2, e, ex, ey, ez;
  bool valid;
};

template <class K, typename T>
__device__ __forceinline__ Slab make_slab(const MeshK<T> &m) {
  Slab s;
  s.le = threadIdx.x / K::QQ;
  s.t2 = threadIdx.x % K::QQ;
  s.i1 = s.t2 % K::Dm::Q;
  s.i2 = s.t2 / K::Dm::Q;
  s.e = blockIdx.x * K::NE + s.le;
  s.valid = s.e < m.E;
  int e = s.valid ? s.e : 0;
  s.ex = e % m.nx;
  s.ey = (e / m.nx) % m.ny;
  s.ez = e / (m.nx * m.ny);
  return s;
}

template <class K, typename T>
__device__ __forceinline__ void load_tables(const MeshK<T> &m, T *s_tab) {
  for (int i = threadIdx.x; i < K::TS; i += K::NT) s_tab[i] = m.tab[i];
}

template <class K, typename T>
__device__ __forceinline__ size_t slot_index(const MeshK<T> &m, const Slab &s, int a, int b, int c) {
  constexpr int P = K::Dm::P;
  return ((size_t)(s.ez * P + c) * m.Ny + (s.ey * P + b)) * m.Nx + (s.ex * P + a);
}

// Gather one component of v into su[n^3] (zero for constrained DOFs if mask).
template <class K, typename T>
__device__ __forceinline__ void gather_comp(const MeshK<T> &m, const Slab &s, const T *__restrict__ v,
                                            int comp, bool mask, T *su) {
  constexpr int n = K::n, P = K::Dm::P;
  for (int idx = s.t2; idx < K::n3; idx += K::QQ) {
    int a = idx % n, b = (idx / n) % n, c = idx / (n * n);
    T val = T(0);
    if (s.valid) {
      int ix = s.ex * P + a, iy = s.ey * P + b, iz = s.ez * P + c;
      if (!(mask && is_constrained(m.bc, comp, ix, iy, iz, m.Nx, m.Ny, m.Nz)))
        val = v[(size_t)comp * m.Nn + ((size_t)iz * m.Ny + iy) * m.Nx + ix];
    }
    su[idx] = val;
  }
}

// xi1 contraction: st0[c][b][q1] = sum_a B[q1][a] u[c][b][a]; st1 with D.
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void stage1(const T *sB, const T *sD, const T *su, T *st, const Slab &s) {
  constexpr int n = K::n, Q = K::Dm::Q;
  if (s.i2 < n) {
    T rb[n], rd[n];
#pragma unroll
    for (int a = 0; a < n; a++) {
      rb[a] = sB[s.i1 * n + a];
      if (GRAD) rd[a] = sD[s.i1 * n + a];
    }
#pragma unroll
    for (int c = 0; c < n; c++) {
      T sb = T(0), sd = T(0);
#pragma unroll
      for (int a = 0; a < n; a++) {
        T x = su[(c * n + s.i2) * n + a];
        sb += rb[a] * x;
        if (GRAD) sd += rd[a] * x;
      }
      st[(c * n + s.i2) * Q + s.i1] = sb;
      if (GRAD) st[n * n * Q + (c * n + s.i2) * Q + s.i1] = sd;
    }
  }
}

// xi2 contraction into registers: XBB[c] (B in xi1, B in xi2), XBD (B, D),
// XDB (D, B) at column (q1, q2) = (i1, i2).
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void stage2(const T *sB, const T *sD, const T *st, const Slab &s,
                                       T (&XBB)[K::n], T (&XBD)[K::n], T (&XDB)[K::n]) {
  constexpr int n = K::n, Q = K::Dm::Q;
  T rb[n], rd[n];
#pragma unroll
  for (int b = 0; b < n; b++) {
    rb[b] = sB[s.i2 * n + b];
    if (GRAD) rd[b] = sD[s.i2 * n + b];
  }
#pragma unroll
  for (int c = 0; c < n; c++) {
    T bb = T(0), bd = T(0), db = T(0);
#pragma unroll
    for (int b = 0; b < n; b++) {
      T t0 = st[(c * n + b) * Q + s.i1];
      bb += rb[b] * t0;
      if (GRAD) {
        bd += rd[b] * t0;
        db += rb[b] * st[n * n * Q + (c * n + b) * Q + s.i1];
      }
    }
    XBB[c] = bb;
    if (GRAD) {
      XBD[c] = bd;
      XDB[c] = db;
    }
  }
}

// Forward pass of all three components of a vector field: registers
// X[comp][kind][c] with kind 0 = BB, 1 = BD, 2 = DB.  Uses su/st of this
// element; ends with a barrier.
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void forward3(const MeshK<T> &m, const Slab &s, const T *__restrict__ v,
                                         bool mask, const T *sB, const T *sD, T *su, T *st,
                                         T (&X)[3][3][K::n]) {
#pragma unroll
  for (int i = 0; i < 3; i++) {
    gather_comp<K>(m, s, v, i, mask, su);
    __syncthreads();
    stage1<K, T, GRAD>(sB, sD, su, st, s);
    __syncthreads();
    stage2<K, T, GRAD>(sB, sD, st, s, X[i][0], X[i][1], X[i][2]);
    __syncthreads();
  }
}

// Gradient (physical) of the field at Gauss point (i1, i2, q3) from X.
template <class K, typename T>
__device__ __forceinline__ void grad_at(const MeshK<T> &m, const T *tab, int q3,
                                        const T (&X)[3][3][K::n], T H[9]) {
  constexpr int n = K::n;
  using Dm = typename K::Dm;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    T g0 = T(0), g1 = T(0), g2 = T(0);
#pragma unroll
    for (int c = 0; c < n; c++) {
      T bq = tab[Dm::TB + q3 * n + c], dq = tab[Dm::TD + q3 * n + c];
      g0 += bq * X[i][2][c];
      g1 += bq * X[i][1][c];
      g2 += dq * X[i][0][c];
    }
    H[i * 3 + 0] = g0 * m.ih[0];
    H[i * 3 + 1] = g1 * m.ih[1];
    H[i * 3 + 2] = g2 * m.ih[2];
  }
}

template <class K, typename T>
__device__ __forceinline__ void value_at(const T *tab, int q3, const T (&X)[3][3][K::n], T val[3]) {
  constexpr int n = K::n;
  using Dm = typename K::Dm;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    T g = T(0);
#pragma unroll
    for (int c = 0; c < n; c++) g += tab[Dm::TB + q3 * n + c] * X[i][0][c];
    val[i] = g;
  }
}

// Transposed xi3 contraction: accumulate flux f (already scaled by the
// quadrature weight, detJ and 2/h) and a value-type flux mv into A.
template <class K, typename T, bool GRAD, bool VAL>
__device__ __forceinline__ void accum_at(const T *tab, int q3, const T f[9], const T mv[3],
                                         T (&A)[3][3][K::n]) {
  constexpr int n = K::n;
  using Dm = typename K::Dm;
#pragma unroll
  for (int c = 0; c < n; c++) {
    T bq = tab[Dm::TB + q3 * n + c], dq = tab[Dm::TD + q3 * n + c];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      if (GRAD) {
        A[i][2][c] += bq * f[i * 3 + 0];
        A[i][1][c] += bq * f[i * 3 + 1];
        A[i][0][c] += dq * f[i * 3 + 2];
      }
      if (VAL) A[i][0][c] += bq * mv[i];
    }
  }
}

// Transpose of the xi2 and xi1 contractions for one component and scatter-add
// into y.  Returns (in dot) sum over this thread's outputs of vdot * y_local
// when vdot != nullptr (element-local p^T A p).
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void transpose_scatter(const MeshK<T> &m, const Slab &s, int comp,
                                                  const T (&A)[3][K::n], const T *sB,
                                                  const T *sD, T *sg, T *st, T *__restrict__ y,
                                                  bool mask, const T *__restrict__ vdot,
                                                  double &dot) {
  constexpr int n = K::n, Q = K::Dm::Q, QQ = K::QQ;
  // A[0] = BB-kind (D or B in xi3 applied), A[1] = BD-kind, A[2] = DB-kind
#pragma unroll
  for (int c = 0; c < n; c++) {
    sg[(c * Q + s.i2) * Q + s.i1] = A[0][c];
    if (GRAD) {
      sg[n * QQ + (c * Q + s.i2) * Q + s.i1] = A[1][c];
      sg[2 * n * QQ + (c * Q + s.i2) * Q + s.i1] = A[2][c];
    }
  }
  __syncthreads();
  if (s.i2 < n) {  // thread (q1 = i1, b = i2)
    T cb[Q], cd[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
      cb[q] = sB[q * n + s.i2];
      if (GRAD) cd[q] = sD[q * n + s.i2];
    }
#pragma unroll
    for (int c = 0; c < n; c++) {
      T hb = T(0), hd = T(0);
#pragma unroll
      for (int q = 0; q < Q; q++) {
        T g0 = sg[(c * Q + q) * Q + s.i1];
        hb += cb[q] * g0;
        if (GRAD) {
          hb += cd[q] * sg[n * QQ + (c * Q + q) * Q + s.i1];
          hd += cb[q] * sg[2 * n * QQ + (c * Q + q) * Q + s.i1];
        }
      }
      st[(c * n + s.i2) * Q + s.i1] = hb;
      if (GRAD) st[n * n * Q + (c * n + s.i2) * Q + s.i1] = hd;
    }
  }
  __syncthreads();
  if (s.i1 < n && s.i2 < n) {  // thread (a = i1, b = i2)
    T cb[Q], cd[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
      cb[q] = sB[q * n + s.i1];
      if (GRAD) cd[q] = sD[q * n + s.i1];
    }
    constexpr int P = K::Dm::P;
#pragma unroll
    for (int c = 0; c < n; c++) {
      T val = T(0);
#pragma unroll
      for (int q = 0; q < Q; q++) {
        val += cb[q] * st[(c * n + s.i2) * Q + q];
        if (GRAD) val += cd[q] * st[n * n * Q + (c * n + s.i2) * Q + q];
      }
      if (s.valid) {
        int ix = s.ex * P + s.i1, iy = s.ey * P + s.i2, iz = s.ez * P + c;
        if (!(mask && is_constrained(m.bc, comp, ix, iy, iz, m.Nx, m.Ny, m.Nz))) {
          size_t gi = (size_t)comp * m.Nn + ((size_t)iz * m.Ny + iy) * m.Nx + ix;
          atomicAdd(&y[gi], val);
          if (vdot) dot += (double)vdot[gi] * (double)val;
        }
      }
    }
  }
  __syncthreads();
}

template <class K, typename T>
__device__ __forceinline__ void zero_acc(T (&A)[3][3][K::n]) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int c = 0; c < K::n; c++) A[i][k][c] = T(0);
}

// Compile-time loop helper.
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// ===================================================================== force
// R(u) (and optionally the linearisation state of u).
template <int P, int Q, typename T, bool STORE, bool OUT>
__global__ __launch_bounds__((EK<P, Q, T>::NT)) void k_force(MeshK<T> m, const double *__restrict__ mu,
                                                           const double *__restrict__ lam,
                                                           const T *__restrict__ u, T *__restrict__ R,
                                                           T *__restrict__ state, int mask) {
  using K = EK<P, Q, T>;
  __shared__ T smem[K::NE * K::SE + K::TS];
  T *s_tab = smem + K::NE * K::SE;
  load_tables<K>(m, s_tab);
  Slab s = make_slab<K>(m);
  T *su = smem + s.le * K::SE, *st = su + K::SA;
  const T *sB = s_tab + K::Dm::TB, *sD = s_tab + K::Dm::TD, *sW = s_tab + K::Dm::TW;
  __syncthreads();
  T X[3][3][K::n];
  forward3<K, T, true>(m, s, u, false, sB, sD, su, st, X);
  T mue = s.valid ? (T)mu[s.e] : T(0), lae = s.valid ? (T)lam[s.e] : T(0);
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ;
  T A[3][3][K::n];
  if (OUT) zero_acc<K>(A);
  bool bad = false;
#pragma unroll 1
  for (int q3 = 0; q3 < Q; q3++) {
    T H[9];
    grad_at<K, T>(m, s_tab, q3, X, H);
    Kin<T> kk;
    bool ok = kinematics(H, kk);
    if (!ok) {
      bad = true;
#pragma unroll
      for (int i = 0; i < 9; i++) kk.G[i] = T(0);
      kk.lnJ = T(0);
    }
    if (STORE && s.valid) {
      size_t base = (size_t)s.e * 10 * Q * Q * Q + (q3 * Q + s.i2) * Q + s.i1;
#pragma unroll
      for (int k = 0; k < 9; k++) state[base + (size_t)k * Q * Q * Q] = kk.G[k];
      state[base + (size_t)9 * Q * Q * Q] = mue - lae * kk.lnJ;
    }
    if (OUT) {
      T Pk[9], f[9], mv[3] = {T(0), T(0), T(0)};
      first_pk(H, kk, mue, lae, Pk);
      T wq = w12 * s_tab[K::Dm::TW + q3];
      if (!ok) wq = T(0);
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int J = 0; J < 3; J++) f[i * 3 + J] = Pk[i * 3 + J] * wq * m.ih[J];
      accum_at<K, T, true, false>(s_tab, q3, f, mv, A);
    }
  }
  if (bad && s.valid) atomicOr(m.flag, 1);
  if (OUT) {
    double dummy = 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
      transpose_scatter<K, T, true>(m, s, i, A[i], sB, sD, su, st, R, mask != 0, nullptr, dummy);
  }
}

// ============================================================ tangent action
// y = (K_T + s M) v with K_T from the stored state (REC = false) or from u_lin
// recomputed at every Gauss point (REC = true).  Optionally accumulates
// p^T A p (= sum_e v_e^T A_e v_e) into red.
template <int P, int Q, typename T, bool REC, bool MASS>
__global__ __launch_bounds__((EK<P, Q, T>::NT)) void k_tangent(
    MeshK<T> m, const double *__restrict__ mu, const double *__restrict__ lam,
    const T *__restrict__ ulin, const T *__restrict__ state, T mshift_rho, const T *__restrict__ v,
    T *__restrict__ y, int mask, Reduce red, int do_red, const int *__restrict__ skip) {
  using K = EK<P, Q, T>;
  if (skip && *skip) return;
  __shared__ T smem[K::NE * K::SE + K::TS];
  __shared__ double s_red[(K::NT + 63) / 64];
  T *s_tab = smem + K::NE * K::SE;
  load_tables<K>(m, s_tab);
  Slab s = make_slab<K>(m);
  T *su = smem + s.le * K::SE, *st = su + K::SA;
  const T *sB = s_tab + K::Dm::TB, *sD = s_tab + K::Dm::TD, *sW = s_tab + K::Dm::TW;
  __syncthreads();
  T XU[3][3][K::n];
  if (REC) forward3<K, T, true>(m, s, ulin, false, sB, sD, su, st, XU);
  T X[3][3][K::n];
  forward3<K, T, true>(m, s, v, mask != 0, sB, sD, su, st, X);
  T mue = s.valid ? (T)mu[s.e] : T(0), lae = s.valid ? (T)lam[s.e] : T(0);
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ;
  T A[3][3][K::n];
  zero_acc<K>(A);
  bool bad = false;
#pragma unroll 1
  for (int q3 = 0; q3 < Q; q3++) {
    T dF[9], G[9], c1;
    grad_at<K, T>(m, s_tab, q3, X, dF);
    if (REC) {
      T H[9];
      grad_at<K, T>(m, s_tab, q3, XU, H);
      Kin<T> kk;
      if (!kinematics(H, kk)) {
        bad = true;
        kk.lnJ = T(0);
#pragma unroll
        for (int i = 0; i < 9; i++) kk.G[i] = T(0);
      }
#pragma unroll
      for (int i = 0; i < 9; i++) G[i] = kk.G[i];
      c1 = mue - lae * kk.lnJ;
    } else {
      size_t base = (size_t)(s.valid ? s.e : 0) * 10 * Q * Q * Q + (q3 * Q + s.i2) * Q + s.i1;
#pragma unroll
      for (int k = 0; k < 9; k++) G[k] = state[base + (size_t)k * Q * Q * Q];
      c1 = state[base + (size_t)9 * Q * Q * Q];
    }
    T dP[9], f[9], mv[3];
    tangent_dp(G, c1, mue, lae, dF, dP);
    T wq = w12 * s_tab[K::Dm::TW + q3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int J = 0; J < 3; J++) f[i * 3 + J] = dP[i * 3 + J] * wq * m.ih[J];
    if (MASS) {
      T val[3];
      value_at<K, T>(s_tab, q3, X, val);
#pragma unroll
      for (int i = 0; i < 3; i++) mv[i] = mshift_rho * wq * val[i];
    }
    accum_at<K, T, true, MASS>(s_tab, q3, f, mv, A);
  }
  if (REC && bad && s.valid) atomicOr(m.flag, 1);
  double dot = 0;
#pragma unroll
  for (int i = 0; i < 3; i++)
    transpose_scatter<K, T, true>(m, s, i, A[i], sB, sD, su, st, y, mask != 0,
                                  do_red ? v : (const T *)nullptr, dot);
  if (do_red) {
    double t = block_sum<K::NT>(dot, s_red);
    grid_reduce_finish<K::NT>(t, red, s_red, gridDim.x);
  }
}

// ====================================================================== mass
template <int P, int Q, typename T>
__global__ __launch_bounds__((EK<P, Q, T>::NT)) void k_mass(MeshK<T> m, T rho, const T *__restrict__ v,
                                                          T *__restrict__ y, int mask, Reduce red,
                                                          int do_red, const int *__restrict__ skip) {
  using K = EK<P, Q, T>;
  if (skip && *skip) return;
  __shared__ T smem[K::NE * K::SE + K::TS];
  __shared__ double s_red[(K::NT + 63) / 64];
  T *s_tab = smem + K::NE * K::SE;
  load_tables<K>(m, s_tab);
  Slab s = make_slab<K>(m);
  T *su = smem + s.le * K::SE, *st = su + K::SA;
  const T *sB = s_tab + K::Dm::TB, *sD = s_tab + K::Dm::TD, *sW = s_tab + K::Dm::TW;
  __syncthreads();
  T X[3][3][K::n];
  forward3<K, T, false>(m, s, v, mask != 0, sB, sD, su, st, X);
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ * rho;
  T A[3][3][K::n];
  zero_acc<K>(A);
#pragma unroll 1
  for (int q3 = 0; q3 < Q; q3++) {
    T val[3], mv[3], f[9];
    value_at<K, T>(s_tab, q3, X, val);
    T wq = w12 * s_tab[K::Dm::TW + q3];
#pragma unroll
    for (int i = 0; i < 3; i++) mv[i] = wq * val[i];
    accum_at<K, T, false, true>(s_tab, q3, f, mv, A);
  }
  double dot = 0;
#pragma unroll
  for (int i = 0; i < 3; i++)
    transpose_scatter<K, T, false>(m, s, i, A[i], sB, sD, su, st, y, mask != 0,
                                   do_red ? v : (const T *)nullptr, dot);
  if (do_red) {
    double t = block_sum<K::NT>(dot, s_red);
    grid_reduce_finish<K::NT>(t, red, s_red, gridDim.x);
  }
}

// ================================================================= diagonal
// d_(l,i) += sum_q w detJ [sum_JL dN_l/dX_J A_iJiL dN_l/dX_L + s rho N_l^2]
// with A_iJiL = mu delta_JL + (c1 + lam) G_Ji G_Li; sum-factorised with the
// product tables B*B, D*D, B*D (tensor structure of N_l^2 and dN dN).
template <int P, int Q, typename T>
__global__ __launch_bounds__((EK<P, Q, T>::NT)) void k_diag(MeshK<T> m, const double *__restrict__ mu,
                                                          const double *__restrict__ lam,
                                                          const T *__restrict__ state, T mshift_rho,
                                                          T *__restrict__ d, int mask) {
  using K = EK<P, Q, T>;
  constexpr int n = K::n, QQ = K::QQ, QQQ = Q * Q * Q;
  using Dm = typename K::Dm;
  __shared__ T smem[K::NE * K::SE + K::TS];
  T *s_tab = smem + K::NE * K::SE;
  load_tables<K>(m, s_tab);
  Slab s = make_slab<K>(m);
  T *sg = smem + s.le * K::SE, *st = sg + K::SA;
  const T *sW = s_tab + Dm::TW, *sB2 = s_tab + Dm::TB2, *sD2 = s_tab + Dm::TD2,
          *sBD = s_tab + Dm::TBD;
  __syncthreads();
  // without a state only the mass term remains (diagonal of s M)
  const bool has_state = state != nullptr;
  T mue = (s.valid && has_state) ? (T)mu[s.e] : T(0), lae = (s.valid && has_state) ? (T)lam[s.e] : T(0);
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ;
  T ih[3] = {m.ih[0], m.ih[1], m.ih[2]};
#pragma unroll 1
  for (int i = 0; i < 3; i++) {
    // six xi3 accumulators, named by (xi1 table, xi2 table):
    // tA (D2,B2) tB (B2,D2) tC (B2,B2) tD (BD,BD) tE (BD,B2) tF (B2,BD)
    T tA[n], tB[n], tC[n], tD[n], tE[n], tF[n];
#pragma unroll
    for (int c = 0; c < n; c++) tA[c] = tB[c] = tC[c] = tD[c] = tE[c] = tF[c] = T(0);
#pragma unroll 1
    for (int q3 = 0; q3 < Q; q3++) {
      size_t base = (size_t)(s.valid ? s.e : 0) * 10 * QQQ + (q3 * Q + s.i2) * Q + s.i1;
      T G0 = T(0), G1 = T(0), G2 = T(0), c1 = T(0);
      if (has_state) {
        G0 = state[base + (size_t)(0 * 3 + i) * QQQ];
        G1 = state[base + (size_t)(1 * 3 + i) * QQQ];
        G2 = state[base + (size_t)(2 * 3 + i) * QQQ];
        c1 = state[base + (size_t)9 * QQQ];
      }
      T wq = w12 * s_tab[Dm::TW + q3];
      T cc = c1 + lae;
      T Gj[3] = {G0, G1, G2};
      T cJL[3][3];
#pragma unroll
      for (int J = 0; J < 3; J++)
#pragma unroll
        for (int L = 0; L < 3; L++)
          cJL[J][L] = wq * ih[J] * ih[L] * ((J == L ? mue : T(0)) + cc * Gj[J] * Gj[L]);
      T cm = mshift_rho * wq;
#pragma unroll
      for (int c = 0; c < n; c++) {
        T b2 = s_tab[Dm::TB2 + q3 * n + c], d2 = s_tab[Dm::TD2 + q3 * n + c],
          bd = s_tab[Dm::TBD + q3 * n + c];
        tA[c] += b2 * cJL[0][0];
        tB[c] += b2 * cJL[1][1];
        tC[c] += d2 * cJL[2][2] + b2 * cm;
        tD[c] += b2 * (cJL[0][1] + cJL[1][0]);
        tE[c] += bd * (cJL[0][2] + cJL[2][0]);
        tF[c] += bd * (cJL[1][2] + cJL[2][1]);
      }
    }
    // stage 2 transpose: h_D2 = sum_q2 B2 tA; h_B2 = sum_q2 (D2 tB + B2 tC + BD tF);
    // h_BD = sum_q2 (BD tD + B2 tE)
#pragma unroll
    for (int c = 0; c < n; c++) {
      sg[(0 * n + c) * QQ + s.t2] = tA[c];
      sg[(1 * n + c) * QQ + s.t2] = tB[c];
      sg[(2 * n + c) * QQ + s.t2] = tC[c];
    }
    // region A holds 3 n QQ words: store tD, tE, tF after a barrier in region B+A reuse
    __syncthreads();
    T hD2[n], hB2[n], hBD[n];
    if (s.i2 < n) {  // thread (q1 = i1, b = i2)
#pragma unroll
      for (int c = 0; c < n; c++) {
        T a0 = T(0), a1 = T(0);
#pragma unroll
        for (int q = 0; q < Q; q++) {
          a0 += sB2[q * n + s.i2] * sg[(0 * n + c) * QQ + q * Q + s.i1];
          a1 += sD2[q * n + s.i2] * sg[(1 * n + c) * QQ + q * Q + s.i1] +
                sB2[q * n + s.i2] * sg[(2 * n + c) * QQ + q * Q + s.i1];
        }
        hD2[c] = a0;
        hB2[c] = a1;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < n; c++) {
      sg[(0 * n + c) * QQ + s.t2] = tD[c];
      sg[(1 * n + c) * QQ + s.t2] = tE[c];
      sg[(2 * n + c) * QQ + s.t2] = tF[c];
    }
    __syncthreads();
    if (s.i2 < n) {
#pragma unroll
      for (int c = 0; c < n; c++) {
        T a1 = hB2[c], a2 = T(0);
#pragma unroll
        for (int q = 0; q < Q; q++) {
          a1 += sBD[q * n + s.i2] * sg[(2 * n + c) * QQ + q * Q + s.i1];
          a2 += sBD[q * n + s.i2] * sg[(0 * n + c) * QQ + q * Q + s.i1] +
                sB2[q * n + s.i2] * sg[(1 * n + c) * QQ + q * Q + s.i1];
        }
        hB2[c] = a1;
        hBD[c] = a2;
      }
    }
    __syncthreads();
    // region B (2 n^2 Q) is too small for three arrays: use region A for them
    if (s.i2 < n) {
#pragma unroll
      for (int c = 0; c < n; c++) {
        sg[(0 * n + c) * n * Q + s.i2 * Q + s.i1] = hD2[c];
        sg[(1 * n + c) * n * Q + s.i2 * Q + s.i1] = hB2[c];
        sg[(2 * n + c) * n * Q + s.i2 * Q + s.i1] = hBD[c];
      }
    }
    __syncthreads();
    if (s.i1 < n && s.i2 < n) {  // thread (a = i1, b = i2)
#pragma unroll
      for (int c = 0; c < n; c++) {
        T val = T(0);
#pragma unroll
        for (int q = 0; q < Q; q++)
          val += sD2[q * n + s.i1] * sg[(0 * n + c) * n * Q + s.i2 * Q + q] +
                 sB2[q * n + s.i1] * sg[(1 * n + c) * n * Q + s.i2 * Q + q] +
                 sBD[q * n + s.i1] * sg[(2 * n + c) * n * Q + s.i2 * Q + q];
        if (s.valid) {
          int ix = s.ex * P + s.i1, iy = s.ey * P + s.i2, iz = s.ez * P + c;
          if (!(mask && is_constrained(m.bc, i, ix, iy, iz, m.Nx, m.Ny, m.Nz)))
            atomicAdd(&d[(size_t)i * m.Nn + ((size_t)iz * m.Ny + iy) * m.Nx + ix], val);
        }
      }
    }
    __syncthreads();
  }
  (void)st;
}

// ============================================================ strain energy
template <int P, int Q>
__global__ __launch_bounds__((EK<P, Q, double>::NT)) void k_energy(MeshK<double> m,
                                                                 const double *__restrict__ mu,
                                                                 const double *__restrict__ lam,
                                                                 const double *__restrict__ u,
                                                                 Reduce red) {
  using T = double;
  using K = EK<P, Q, T>;
  __shared__ T smem[K::NE * K::SE + K::TS];
  __shared__ double s_red[(K::NT + 63) / 64];
  T *s_tab = smem + K::NE * K::SE;
  load_tables<K>(m, s_tab);
  Slab s = make_slab<K>(m);
  T *su = smem + s.le * K::SE, *st = su + K::SA;
  const T *sB = s_tab + K::Dm::TB, *sD = s_tab + K::Dm::TD, *sW = s_tab + K::Dm::TW;
  __syncthreads();
  T X[3][3][K::n];
  forward3<K, T, true>(m, s, u, false, sB, sD, su, st, X);
  T mue = s.valid ? mu[s.e] : 0.0, lae = s.valid ? lam[s.e] : 0.0;
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ;
  double acc = 0;
#pragma unroll 1
  for (int q3 = 0; q3 < Q; q3++) {
    T H[9];
    grad_at<K, T>(m, s_tab, q3, X, H);
    Kin<T> kk;
    if (kinematics(H, kk)) {
      // Psi = mu/2 (tr C - 3) - mu lnJ + lam/2 lnJ^2, tr C - 3 = 2 tr H + |H|^2
      T hh = 0;
#pragma unroll
      for (int k = 0; k < 9; k++) hh += H[k] * H[k];
      T trH = H[0] + H[4] + H[8];
      T psi = 0.5 * mue * (2.0 * trH + hh) - mue * kk.lnJ + 0.5 * lae * kk.lnJ * kk.lnJ;
      acc += w12 * s_tab[K::Dm::TW + q3] * psi;
    }
  }
  if (!s.valid) acc = 0;
  double t = block_sum<K::NT>(acc, s_red);
  grid_reduce_finish<K::NT>(t, red, s_red, gridDim.x);
}

// ===================================================== material sensitivity
// g_mu[e] += scale sum_q w detJ (F - F^-T) : grad w ; g_lam[e] += scale sum_q w
// detJ lnJ F^-T : grad w.  One element per Q x Q slab; element sums by wave
// shuffles and LDS (no global atomics needed: each element has one owner).
template <int P, int Q>
__global__ __launch_bounds__((EK<P, Q, double>::NT)) void k_matgrad(
    MeshK<double> m, const double *__restrict__ u, const double *__restrict__ wv, double scale,
    double *__restrict__ g_mu, double *__restrict__ g_lam) {
  using T = double;
  using K = EK<P, Q, T>;
  __shared__ T smem[K::NE * K::SE + K::TS];
  __shared__ double s_part[K::NE][2][K::QQ];
  T *s_tab = smem + K::NE * K::SE;
  load_tables<K>(m, s_tab);
  Slab s = make_slab<K>(m);
  T *su = smem + s.le * K::SE, *st = su + K::SA;
  const T *sB = s_tab + K::Dm::TB, *sD = s_tab + K::Dm::TD, *sW = s_tab + K::Dm::TW;
  __syncthreads();
  T XU[3][3][K::n], XW[3][3][K::n];
  forward3<K, T, true>(m, s, u, false, sB, sD, su, st, XU);
  forward3<K, T, true>(m, s, wv, false, sB, sD, su, st, XW);
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ;
  double am = 0, al = 0;
#pragma unroll 1
  for (int q3 = 0; q3 < Q; q3++) {
    T H[9], Gw[9];
    grad_at<K, T>(m, s_tab, q3, XU, H);
    grad_at<K, T>(m, s_tab, q3, XW, Gw);
    Kin<T> kk;
    if (kinematics(H, kk)) {
      T wq = w12 * s_tab[K::Dm::TW + q3];
      // F - F^-T = (H + H^T + H H^T) F^-T
      T Bm[9];
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
          Bm[i * 3 + j] = H[i * 3 + j] + H[j * 3 + i] + H[i * 3] * H[j * 3] +
                          H[i * 3 + 1] * H[j * 3 + 1] + H[i * 3 + 2] * H[j * 3 + 2];
      double sm = 0, sl = 0;
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int J = 0; J < 3; J++) {
          T GiT = kk.G[J * 3 + i];
          T dmu = Bm[i * 3 + 0] * kk.G[J * 3 + 0] + Bm[i * 3 + 1] * kk.G[J * 3 + 1] +
                  Bm[i * 3 + 2] * kk.G[J * 3 + 2];
          sm += dmu * Gw[i * 3 + J];
          sl += kk.lnJ * GiT * Gw[i * 3 + J];
        }
      am += wq * sm;
      al += wq * sl;
    }
  }
  s_part[s.le][0][s.t2] = am;
  s_part[s.le][1][s.t2] = al;
  __syncthreads();
  if (s.t2 == 0 && s.valid) {
    double tm = 0, tl = 0;
    for (int i = 0; i < K::QQ; i++) {
      tm += s_part[s.le][0][i];
      tl += s_part[s.le][1][i];
    }
    g_mu[s.e] += scale * tm;
    g_lam[s.e] += scale * tl;
  }
}

// ============================================================ launch wrappers
template <int P, typename T>
int launch_force_t(const MeshK<T> &m, const double *mu, const double *lam, const T *u, T *R,
                          T *state, int mask, hipStream_t st) {
  constexpr int Q = P + 2;
  using K = EK<P, Q, T>;
  dim3 grid((m.E + K::NE - 1) / K::NE), block(K::NT);
  if (R && state)
    hipLaunchKernelGGL((k_force<P, Q, T, true, true>), grid, block, 0, st, m, mu, lam, u, R, state, mask);
  else if (R)
    hipLaunchKernelGGL((k_force<P, Q, T, false, true>), grid, block, 0, st, m, mu, lam, u, R, state, mask);
  else
    hipLaunchKernelGGL((k_force<P, Q, T, true, false>), grid, block, 0, st, m, mu, lam, u, R, state, mask);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int P, typename T>
int launch_tangent_t(const MeshK<T> &m, const double *mu, const double *lam, const T *ulin,
                            const T *state, T msr, const T *v, T *y, int mask, Reduce red,
                            int do_red, const int *skip, hipStream_t st) {
  constexpr int Q = P + 2;
  using K = EK<P, Q, T>;
  dim3 grid((m.E + K::NE - 1) / K::NE), block(K::NT);
  bool mass = msr != T(0);
  if (ulin) {
    if (mass)
      hipLaunchKernelGGL((k_tangent<P, Q, T, true, true>), grid, block, 0, st, m, mu, lam, ulin, state, msr, v, y, mask, red, do_red, skip);
    else
      hipLaunchKernelGGL((k_tangent<P, Q, T, true, false>), grid, block, 0, st, m, mu, lam, ulin, state, msr, v, y, mask, red, do_red, skip);
  } else {
    if (mass)
      hipLaunchKernelGGL((k_tangent<P, Q, T, false, true>), grid, block, 0, st, m, mu, lam, ulin, state, msr, v, y, mask, red, do_red, skip);
    else
      hipLaunchKernelGGL((k_tangent<P, Q, T, false, false>), grid, block, 0, st, m, mu, lam, ulin, state, msr, v, y, mask, red, do_red, skip);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int P, typename T>
int launch_mass_t(const MeshK<T> &m, T rho, const T *v, T *y, int mask, Reduce red,
                         int do_red, const int *skip, hipStream_t st) {
  constexpr int Q = P + 2;
  using K = EK<P, Q, T>;
  dim3 grid((m.E + K::NE - 1) / K::NE), block(K::NT);
  hipLaunchKernelGGL((k_mass<P, Q, T>), grid, block, 0, st, m, rho, v, y, mask, red, do_red, skip);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int P, typename T>
int launch_diag_t(const MeshK<T> &m, const double *mu, const double *lam, const T *state,
                         T msr, T *d, int mask, hipStream_t st) {
  constexpr int Q = P + 2;
  using K = EK<P, Q, T>;
  static_assert(3 * K::n * K::n * Q <= K::SE, "diag LDS layout");
  dim3 grid((m.E + K::NE - 1) / K::NE), block(K::NT);
  hipLaunchKernelGGL((k_diag<P, Q, T>), grid, block, 0, st, m, mu, lam, state, msr, d, mask);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int P>
int launch_energy_t(const MeshK<double> &m, const double *mu, const double *lam,
                           const double *u, Reduce red, hipStream_t st) {
  constexpr int Q = P + 2;
  using K = EK<P, Q, double>;
  dim3 grid((m.E + K::NE - 1) / K::NE), block(K::NT);
  hipLaunchKernelGGL((k_energy<P, Q>), grid, block, 0, st, m, mu, lam, u, red);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int P>
int launch_matgrad_t(const MeshK<double> &m, const double *u, const double *w, double scale,
                            double *gm, double *gl, hipStream_t st) {
  constexpr int Q = P + 2;
  using K = EK<P, Q, double>;
  dim3 grid((m.E + K::NE - 1) / K::NE), block(K::NT);
  hipLaunchKernelGGL((k_matgrad<P, Q>), grid, block, 0, st, m, u, w, scale, gm, gl);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#ifdef SDME_P
// explicit instantiation of the wrappers for one polynomial order per
// translation unit (the build compiles this file once per order)
template int launch_force_t<SDME_P, double>(const MeshK<double> &, const double *, const double *,
                                            const double *, double *, double *, int, hipStream_t);
template int launch_force_t<SDME_P, float>(const MeshK<float> &, const double *, const double *,
                                           const float *, float *, float *, int, hipStream_t);
template int launch_tangent_t<SDME_P, double>(const MeshK<double> &, const double *, const double *,
                                              const double *, const double *, double, const double *,
                                              double *, int, Reduce, int, const int *, hipStream_t);
template int launch_tangent_t<SDME_P, float>(const MeshK<float> &, const double *, const double *,
                                             const float *, const float *, float, const float *,
                                             float *, int, Reduce, int, const int *, hipStream_t);
template int launch_mass_t<SDME_P, double>(const MeshK<double> &, double, const double *, double *,
                                           int, Reduce, int, const int *, hipStream_t);
template int launch_mass_t<SDME_P, float>(const MeshK<float> &, float, const float *, float *, int,
                                          Reduce, int, const int *, hipStream_t);
template int launch_diag_t<SDME_P, double>(const MeshK<double> &, const double *, const double *,
                                           const double *, double, double *, int, hipStream_t);
template int launch_diag_t<SDME_P, float>(const MeshK<float> &, const double *, const double *,
                                          const float *, float, float *, int, hipStream_t);
template int launch_energy_t<SDME_P>(const MeshK<double> &, const double *, const double *,
                                     const double *, Reduce, hipStream_t);
template int launch_matgrad_t<SDME_P>(const MeshK<double> &, const double *, const double *, double,
                                      double *, double *, hipStream_t);
#endif

}  // namespace sdme
