// Vector, reduction and face kernels of libsdme: fused PCG updates with
// deterministic FP64 reductions (wave shuffles, one partial per block, a
// one-block kernel sums the partials in a fixed order), conversions, Dirichlet
// masking, and the surface terms (dead traction, rigid-plane penalty).
#include <hip/hip_runtime.h>

#include <cmath>

#include "sdme_device.h"
#include "sdme_launch.h"

namespace sdme {

constexpr int NTV = VEC_THREADS;

// Two-value deterministic reductions in two passes: every block of the
// streaming kernel writes its two block sums to partials[2 b], partials[2 b + 1]
// (plain stores, no fence or atomic), and a one-block kernel launched after it
// on the same stream sums the partials in block order.  A device-scope fence
// per block (a writeback of the XCD's L2) and a counter atomic shared by all
// blocks cost more than the extra launch.
__device__ __forceinline__ void block_partials2(double a, double b, Reduce red, double *s_red) {
  double ta = block_sum<NTV>(a, s_red);
  double tb = block_sum<NTV>(b, s_red);
  if (threadIdx.x == 0) {
    red.partials[2 * blockIdx.x] = ta;
    red.partials[2 * blockIdx.x + 1] = tb;
  }
}

// Sums of the partials of nb blocks in a fixed order (one block of NT
// threads: thread t adds partials t, t + NT, ... in turn, then the block sum
// adds the threads' sums in thread order); valid in thread 0.  The finishing
// kernels run alone on the device and wait on memory: with many partials
// (~4e3 from the streaming kernels, ~1.5e4 from the FP64 fused operator at
// 2e7 DOF) a wide block with UF independent loads per thread in flight keeps
// them short; with few (small meshes) the narrow block's shorter block sum
// is faster.
constexpr int NTF = 1024, UF = 4, FIN_WIDE_MIN = 1024;
template <int NT>
__device__ __forceinline__ void sum_partials2(const double *partials, int nb, double &a, double &b,
                                              double *s_red) {
  double pa = 0, pb = 0;
  for (int i0 = threadIdx.x; i0 < nb; i0 += UF * NT) {
    double xa[UF], xb[UF];
#pragma unroll
    for (int u = 0; u < UF; u++) {
      const int i = i0 + u * NT;
      xa[u] = i < nb ? partials[2 * i] : 0.0;
      xb[u] = i < nb ? partials[2 * i + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UF; u++) {
      pa += xa[u];
      pb += xb[u];
    }
  }
  a = block_sum<NT>(pa, s_red);
  b = block_sum<NT>(pb, s_red);
}
// One-block finishing kernel K<NT> over nb partials, NT = NTF or NTV by nb.
#define SDME_FIN(K, nb, st, ...)                                                   \
  do {                                                                            \
    if ((nb) > FIN_WIDE_MIN)                                                      \
      hipLaunchKernelGGL(K<NTF>, dim3(1), dim3(NTF), 0, st, __VA_ARGS__);         \
    else                                                                          \
      hipLaunchKernelGGL(K<NTV>, dim3(1), dim3(NTV), 0, st, __VA_ARGS__);         \
  } while (0)

static int grid_for(int64_t n) {
  int64_t b = (n + NTV - 1) / NTV;
  return (int)(b < VEC_BLOCKS ? (b > 0 ? b : 1) : VEC_BLOCKS);
}

template <typename T>
__global__ __launch_bounds__(NTV) void k_fill(T *x, T val, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV) x[i] = val;
}
template <typename T>
int launch_fill(T *x, T val, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(NTV), 0, st, x, val, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename Td, typename Ts>
__global__ __launch_bounds__(NTV) void k_convert(Td *dst, const Ts *src, double scale, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV)
    dst[i] = (Td)((double)src[i] * scale);
}
template <typename Td, typename Ts>
int launch_convert(Td *dst, const Ts *src, double scale, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<Td, Ts>), dim3(grid_for(n)), dim3(NTV), 0, st, dst, src, scale, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ __launch_bounds__(NTV) void k_axpbypcz(double *y, double alpha, const double *x,
                                                  double beta, double gamma, const double *z,
                                                  int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV) {
    double v = alpha * x[i];
    if (beta != 0.0) v += beta * y[i];
    if (z) v += gamma * z[i];
    y[i] = v;
  }
}
int launch_axpby(double *y, double alpha, const double *x, double beta, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpbypcz, dim3(grid_for(n)), dim3(NTV), 0, st, y, alpha, x, beta, 0.0,
                     (const double *)nullptr, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_axpbypcz(double *y, double alpha, const double *x, double beta, double gamma,
                    const double *z, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpbypcz, dim3(grid_for(n)), dim3(NTV), 0, st, y, alpha, x, beta, gamma, z, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ __launch_bounds__(NTV) void k_recip(double *x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV)
    x[i] = 1.0 / x[i];
}
int launch_recip(double *x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_recip, dim3(grid_for(n)), dim3(NTV), 0, st, x, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ __launch_bounds__(NTV) void k_add_scaled_f(double *x, const float *e, double scale,
                                                      int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV)
    x[i] += scale * (double)e[i];
}
int launch_add_scaled_f(double *x, const float *e, double scale, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_add_scaled_f, dim3(grid_for(n)), dim3(NTV), 0, st, x, e, scale, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
__global__ __launch_bounds__(NTV) void k_bc(T *x, int mode, MeshK<T> m) {
  int64_t n = 3 * (int64_t)m.Nn;
  for (int64_t i = blockIdx.x * (int64_t)NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV) {
    int comp = (int)(i / m.Nn);
    int64_t g = i - (int64_t)comp * m.Nn;
    int ix = (int)(g % m.Nx), iy = (int)((g / m.Nx) % m.Ny), iz = (int)(g / ((int64_t)m.Nx * m.Ny));
    if (is_constrained(m.bc, comp, ix, iy, iz, m.Nx, m.Ny, m.Nz)) x[i] = mode ? T(1) : T(0);
  }
}
template <typename T>
int launch_bc(T *x, int mode, const MeshK<T> &m, hipStream_t st) {
  hipLaunchKernelGGL(k_bc<T>, dim3(grid_for(3 * (int64_t)m.Nn)), dim3(NTV), 0, st, x, mode, m);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Streaming loops process U elements per thread and sweep, at i, i + NTV,
// ..., i + (U - 1) NTV inside a chunk of U NTV elements (coalesced, U loads
// per array in flight); the chunks are strided over the grid.
constexpr int U = 4;
#define SDME_VLOOP(BODY)                                                                    \
  for (int64_t c0 = (int64_t)blockIdx.x * (NTV * U) + threadIdx.x; c0 < n;                  \
       c0 += (int64_t)gridDim.x * (NTV * U)) {                                              \
    if (c0 + (U - 1) * NTV < n) {                                                           \
      _Pragma("unroll") for (int u = 0; u < U; u++) {                                      \
        const int64_t i = c0 + u * NTV;                                                     \
        BODY                                                                                \
      }                                                                                     \
    } else {                                                                                \
      for (int u = 0; u < U; u++) {                                                         \
        const int64_t i = c0 + u * NTV;                                                     \
        if (i < n) { BODY }                                                                 \
      }                                                                                     \
    }                                                                                       \
  }

static int grid_for_u(int64_t n) {
  int64_t b = (n + NTV * U - 1) / (NTV * U);
  return (int)(b < VEC_BLOCKS ? (b > 0 ? b : 1) : VEC_BLOCKS);
}

template <typename T>
__global__ __launch_bounds__(NTV) void k_dot2(const T *__restrict__ x, const T *__restrict__ y,
                                              int64_t n, Reduce red) {
  __shared__ double s_red[NTV / 64];
  double a = 0, b = 0;
  SDME_VLOOP(double xv = (double)x[i]; double yv = (double)y[i]; a += xv * yv; b += yv * yv;)
  block_partials2(a, b, red, s_red);
}
template <int NT>
__global__ __launch_bounds__(NT) void k_fin2(Reduce red, int nb) {
  __shared__ double s_red[NT / 64];
  double a, b;
  sum_partials2<NT>(red.partials, nb, a, b, s_red);
  if (threadIdx.x == 0) {
    red.result[0] = a;
    red.result[1] = b;
  }
}
template <typename T>
int launch_dot2(const T *x, const T *y, int64_t n, Reduce red2, hipStream_t st) {
  const int nb = grid_for_u(n);
  hipLaunchKernelGGL(k_dot2<T>, dim3(nb), dim3(NTV), 0, st, x, y, n, red2);
  SDME_FIN(k_fin2, nb, st, red2, nb);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------- PCG
// The PCG kernels take d = the inverse Jacobi diagonal (z = d r).
// init: p = d r; rz = r.z; rr = r.r; tol2 = rtol^2 rr (r = b at x = 0).
template <typename T>
__global__ __launch_bounds__(NTV) void k_pcg_init(const T *__restrict__ r, const T *__restrict__ d,
                                                  T *__restrict__ p, int64_t n, Reduce red) {
  __shared__ double s_red[NTV / 64];
  double a = 0, b = 0;
  SDME_VLOOP(T ri = r[i]; T z = ri * d[i]; p[i] = z; a += (double)ri * (double)z;
             b += (double)ri * (double)ri;)
  block_partials2(a, b, red, s_red);
}
template <int NT>
__global__ __launch_bounds__(NT) void k_pcg_init_fin(PcgDev *s, double rtol, int maxit,
                                                     double delta, Reduce red, int nb) {
  __shared__ double s_red[NT / 64];
  double rz, rr;
  sum_partials2<NT>(red.partials, nb, rz, rr, s_red);
  if (threadIdx.x == 0) {
    s->rz = rz;
    s->rr = rr;
    s->bb = rr;
    s->tol2 = rtol * rtol * rr;
    s->rz_old = rz;
    s->upd2 = delta * delta * rr;
    s->iters = 0;
    s->maxit = maxit;
    s->pAp = 0;
    s->beta = 0;
    s->alpha_pend = 0;
    s->xpend = 0;
    s->done = (rr <= s->tol2) ? 1 : (std::isfinite(rr) ? 0 : 3);
  }
}
template <typename T>
int launch_pcg_init(const T *r, const T *d, T *p, PcgDev *s, double rtol, int maxit, double delta,
                    int64_t n, Reduce red2, hipStream_t st) {
  const int nb = grid_for_u(n);
  hipLaunchKernelGGL(k_pcg_init<T>, dim3(nb), dim3(NTV), 0, st, r, d, p, n, red2);
  SDME_FIN(k_pcg_init_fin, nb, st, s, rtol, maxit, delta, red2, nb);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
__global__ __launch_bounds__(NTV) void k_pcg_pap(const T *__restrict__ p, const T *__restrict__ Ap,
                                                 PcgDev *s, int64_t n, Reduce red) {
  __shared__ double s_red[NTV / 64];
  if (s->done) return;
  double a = 0;
  SDME_VLOOP(a += (double)p[i] * (double)Ap[i];)
  block_partials2(a, 0.0, red, s_red);
}
template <int NT>
__global__ __launch_bounds__(NT) void k_pcg_pap_fin(PcgDev *s, Reduce red, int nb) {
  __shared__ double s_red[NT / 64];
  if (s->done) return;
  double a, b;
  sum_partials2<NT>(red.partials, nb, a, b, s_red);
  if (threadIdx.x == 0) s->pAp = a;
}
// Finishing passes for reductions whose block partials were written by an
// element kernel of nb blocks.
int launch_fin2(Reduce red2, int nb, hipStream_t st) {
  SDME_FIN(k_fin2, nb, st, red2, nb);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_pcg_pap_fin(PcgDev *s, Reduce red2, int nb, hipStream_t st) {
  SDME_FIN(k_pcg_pap_fin, nb, st, s, red2, nb);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_pcg_pap(const T *p, const T *Ap, PcgDev *s, int64_t n, Reduce red2, hipStream_t st) {
  const int nb = grid_for_u(n);
  hipLaunchKernelGGL(k_pcg_pap<T>, dim3(nb), dim3(NTV), 0, st, p, Ap, s, n, red2);
  SDME_FIN(k_pcg_pap_fin, nb, st, s, red2, nb);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Residual replacement of the mixed-precision CG: the recursively updated
// FP32 residual is replaced by the true FP64 residual b - A x (computed by the
// caller); the search direction is kept (reliable updates).
__global__ __launch_bounds__(NTV) void k_pcg_replace(float *__restrict__ r32,
                                                     const double *__restrict__ r64,
                                                     const float *__restrict__ d, int64_t n,
                                                     Reduce red) {
  __shared__ double s_red[NTV / 64];
  double a = 0, b = 0;
  SDME_VLOOP(double rv = r64[i]; float rf = (float)rv; r32[i] = rf;
             a += (double)rf * (double)(rf * d[i]); b += rv * rv;)
  block_partials2(a, b, red, s_red);
}
template <int NT>
__global__ __launch_bounds__(NT) void k_pcg_replace_fin(PcgDev *s, double delta, Reduce red,
                                                        int nb) {
  __shared__ double s_red[NT / 64];
  double rz, rr;
  sum_partials2<NT>(red.partials, nb, rz, rr, s_red);
  if (threadIdx.x == 0) {
    s->beta = rz / s->rz_old;
    s->rz = rz;
    s->rr = rr;
    s->upd2 = delta * delta * rr;
    s->done = (rr <= s->tol2) ? 1 : (std::isfinite(rr) ? 0 : 3);
  }
}
__global__ __launch_bounds__(NTV) void k_pcg_pupdate_force(float *p, const float *r,
                                                           const float *d, const PcgDev *s,
                                                           int64_t n) {
  if (s->done == 1 || s->done == 3) return;
  float beta = (float)s->beta;
  for (int64_t i = blockIdx.x * (int64_t)NTV + threadIdx.x; i < n; i += (int64_t)gridDim.x * NTV)
    p[i] = r[i] * d[i] + beta * p[i];
}
int launch_pcg_replace(float *r32, const double *r64, const float *d, float *p, PcgDev *s,
                       double delta, int64_t n, Reduce red2, bool update_p, hipStream_t st) {
  const int nb = grid_for_u(n);
  hipLaunchKernelGGL(k_pcg_replace, dim3(nb), dim3(NTV), 0, st, r32, r64, d, n, red2);
  SDME_FIN(k_pcg_replace_fin, nb, st, s, delta, red2, nb);
  if (update_p)
    hipLaunchKernelGGL(k_pcg_pupdate_force, dim3(grid_for(n)), dim3(NTV), 0, st, p, r32, d, s, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// update: alpha = rz / pAp; x += alpha p; r -= alpha Ap; Ap = 0;
// rznew = r.(d r); rr = r.r; then beta = rznew / rz, convergence test.
// With the previous direction p_prev (the fused operator keeps p_k and p_k-1
// in two buffers) the x update is done every other iteration: a step with
// xpend = 0 leaves x alone (alpha is kept as alpha_pend), the next one adds
// alpha_pend p_prev + alpha p, so two iterations read x once instead of twice
// (16 instead of 24 bytes per FP32 DOF); launch_pcg_xflush completes x.
template <typename T>
__global__ __launch_bounds__(NTV) void k_pcg_update(T *__restrict__ x, T *__restrict__ r,
                                                    const T *__restrict__ p, T *__restrict__ Ap,
                                                    const T *__restrict__ d, PcgDev *s, int64_t n,
                                                    Reduce red, const T *__restrict__ p_prev) {
  __shared__ double s_red[NTV / 64];
  if (s->done) return;
  double pAp = s->pAp;
  double alpha_d = (pAp > 0.0) ? s->rz / pAp : 0.0;
  T alpha = (T)alpha_d;
  double a = 0, b = 0;
  if (!p_prev) {
    SDME_VLOOP(T pi = p[i]; T api = Ap[i]; T xi = x[i]; T ri = r[i]; T di = d[i];
               x[i] = xi + alpha * pi; ri = ri - alpha * api; r[i] = ri; Ap[i] = T(0);
               T z = ri * di; a += (double)ri * (double)z; b += (double)ri * (double)ri;)
  } else if (!s->xpend) {
    SDME_VLOOP(T api = Ap[i]; T ri = r[i]; T di = d[i];
               ri = ri - alpha * api; r[i] = ri; Ap[i] = T(0);
               T z = ri * di; a += (double)ri * (double)z; b += (double)ri * (double)ri;)
  } else {
    const T alpha0 = (T)s->alpha_pend;
    SDME_VLOOP(T p0 = p_prev[i]; T pi = p[i]; T api = Ap[i]; T xi = x[i]; T ri = r[i];
               T di = d[i]; x[i] = xi + (alpha0 * p0 + alpha * pi); ri = ri - alpha * api;
               r[i] = ri; Ap[i] = T(0); T z = ri * di; a += (double)ri * (double)z;
               b += (double)ri * (double)ri;)
  }
  block_partials2(a, b, red, s_red);
}
template <int NT>
__global__ __launch_bounds__(NT) void k_pcg_update_fin(PcgDev *s, Reduce red, int nb, int defer) {
  __shared__ double s_red[NT / 64];
  if (s->done) return;
  double rznew, rr;
  sum_partials2<NT>(red.partials, nb, rznew, rr, s_red);
  if (threadIdx.x == 0) {
    double pAp = s->pAp;
    s->alpha = (pAp > 0.0) ? s->rz / pAp : 0.0;
    if (defer) {
      if (s->xpend) {
        s->xpend = 0;
      } else {
        s->xpend = 1;
        s->alpha_pend = s->alpha;
      }
    }
    s->beta = rznew / s->rz;
    s->rz_old = s->rz;
    s->rz = rznew;
    s->rr = rr;
    s->iters += 1;
    if (!(pAp > 0.0)) s->done = std::isfinite(pAp) ? 2 : 3;
    else if (!std::isfinite(rr)) s->done = 3;
    else if (rr <= s->tol2) s->done = 1;
    else if (s->iters >= s->maxit) s->done = 4;
    else if (rr <= s->upd2) s->done = 5;
  }
}
template <typename T>
int launch_pcg_update(T *x, T *r, const T *p, T *Ap, const T *d, PcgDev *s, int64_t n,
                      Reduce red2, hipStream_t st, const T *p_prev) {
  const int nb = grid_for_u(n);
  hipLaunchKernelGGL(k_pcg_update<T>, dim3(nb), dim3(NTV), 0, st, x, r, p, Ap, d, s, n, red2,
                     p_prev);
  SDME_FIN(k_pcg_update_fin, nb, st, s, red2, nb, p_prev ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The pending half of a deferred x update (launched by the host when it has
// read xpend = 1; no other block reads xpend, so block 0 clears it).
template <typename T>
__global__ __launch_bounds__(NTV) void k_pcg_xflush(T *__restrict__ x, const T *__restrict__ p,
                                                    PcgDev *s, int64_t n) {
  const T a = (T)s->alpha_pend;
  SDME_VLOOP(x[i] += a * p[i];)
  if (blockIdx.x == 0 && threadIdx.x == 0) s->xpend = 0;
}
template <typename T>
int launch_pcg_xflush(T *x, const T *p, PcgDev *s, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_xflush<T>, dim3(grid_for_u(n)), dim3(NTV), 0, st, x, p, s, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
__global__ __launch_bounds__(NTV) void k_pcg_pupdate(T *__restrict__ p, const T *__restrict__ r,
                                                     const T *__restrict__ d, const PcgDev *s,
                                                     int64_t n) {
  if (s->done) return;
  T beta = (T)s->beta;
  SDME_VLOOP(p[i] = r[i] * d[i] + beta * p[i];)
}
template <typename T>
int launch_pcg_pupdate(T *p, const T *r, const T *d, const PcgDev *s, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_pupdate<T>, dim3(grid_for_u(n)), dim3(NTV), 0, st, p, r, d, s, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// -------------------------------------------------------------- face terms
// One block per boundary-face element; nq = P+1 Gauss points per direction
// (table Bf[nq][n], weights Wf[nq] in the mesh tables).
template <int P>
__global__ __launch_bounds__(128) void k_face(MeshK<double> m, int mode, int face, double t0,
                                              double t1, double t2, double scale, double eps,
                                              double z0, double origin_z, const double *u,
                                              double *f, Reduce red, int do_red) {
  constexpr int n = P + 1, nq = P + 1;
  __shared__ double s_val[nq * nq];
  __shared__ double s_red[2];
  const double *Bf = m.tab + face_table_offset(n, m.Q), *Wf = Bf + n * n;
  int dir = face / 2, side = face % 2;
  int t1d = dir == 0 ? 1 : 0, t2d = dir == 2 ? 1 : 2;
  int ne[3] = {m.nx, m.ny, m.nz};
  int fe = blockIdx.x;  // index over face elements: (j * ne[t1d] + i)
  int ei[3];
  ei[t1d] = fe % ne[t1d];
  ei[t2d] = fe / ne[t1d];
  ei[dir] = side ? ne[dir] - 1 : 0;
  int Nd[3] = {m.Nx, m.Ny, m.Nz};
  double hh[3] = {2.0 / m.ih[0], 2.0 / m.ih[1], 2.0 / m.ih[2]};
  double dA = hh[t1d] * hh[t2d] / 4.0;
  int local_d = side ? P : 0;
  double energy = 0;
  // point values (mode 1: gap pressure; mode 2: x_z at the point)
  for (int pidx = threadIdx.x; pidx < nq * nq; pidx += blockDim.x) {
    int i = pidx % nq, j = pidx / nq;
    double val = 0;
    if (mode != 0) {
      for (int b = 0; b < n; b++)
        for (int a = 0; a < n; a++) {
          int li[3];
          li[t1d] = a; li[t2d] = b; li[dir] = local_d;
          int gi[3] = {ei[0] * P + li[0], ei[1] * P + li[1], ei[2] * P + li[2]};
          size_t g = ((size_t)gi[2] * Nd[1] + gi[1]) * Nd[0] + gi[0];
          val += Bf[i * n + a] * Bf[j * n + b] * u[2 * (size_t)m.Nn + g];
        }
      if (mode == 1) {
        double gap = origin_z + val - z0;
        double w = Wf[i] * Wf[j] * dA;
        if (gap < 0) energy += 0.5 * eps * gap * gap * w;
        val = gap < 0 ? eps * (-gap) : 0.0;
      } else {
        val = eps * val;
      }
    }
    s_val[pidx] = val;
  }
  __syncthreads();
  for (int midx = threadIdx.x; midx < n * n; midx += blockDim.x) {
    int a = midx % n, b = midx / n;
    double acc[3] = {0, 0, 0};
    for (int j = 0; j < nq; j++)
      for (int i = 0; i < nq; i++) {
        double wN = Wf[i] * Wf[j] * dA * Bf[i * n + a] * Bf[j * n + b];
        if (mode == 0) {
          acc[0] += wN * t0; acc[1] += wN * t1; acc[2] += wN * t2;
        } else {
          acc[2] += wN * s_val[j * nq + i];
        }
      }
    int li[3];
    li[t1d] = a; li[t2d] = b; li[dir] = local_d;
    int gi[3] = {ei[0] * P + li[0], ei[1] * P + li[1], ei[2] * P + li[2]};
    size_t g = ((size_t)gi[2] * Nd[1] + gi[1]) * Nd[0] + gi[0];
    if (m.stage) {  // ordered assembly: face-element vector, gathered afterwards
      for (int c = 0; c < 3; c++)
        m.stage[((size_t)fe * 3 + c) * n * n + midx] = c >= (mode == 0 ? 0 : 2) ? scale * acc[c] : 0.0;
    } else {
      for (int c = (mode == 0 ? 0 : 2); c < 3; c++)
        if (acc[c] != 0.0) atomicAdd(&f[c * (size_t)m.Nn + g], scale * acc[c]);
    }
  }
  if (do_red) {
    // block energy -> partial; last block sums (deterministic)
    double e = energy;
    for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = e;
    __syncthreads();
    __shared__ bool s_last;
    if (threadIdx.x == 0) {
      red.partials[blockIdx.x] = s_red[0] + s_red[1];
      __threadfence();
      s_last = atomicAdd(red.counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
      __threadfence();
      double t = 0;
      for (int i = 0; i < (int)gridDim.x; i++) t += __builtin_nontemporal_load(&red.partials[i]);
      *red.result = t;
      *red.counter = 0u;
    }
  }
}

int face_blocks(const MeshK<double> &m, int face) {
  int dir = face / 2;
  int ne[3] = {m.nx, m.ny, m.nz};
  int t1d = dir == 0 ? 1 : 0, t2d = dir == 2 ? 1 : 2;
  return ne[t1d] * ne[t2d];
}

int launch_face(int P, const MeshK<double> &m, int mode, int face, const double *t3, double scale,
                double eps, double z0, double origin_z, const double *u, double *f, Reduce red,
                int do_red, hipStream_t st) {
  dim3 grid(face_blocks(m, face)), block(128);
  double t0 = t3 ? t3[0] : 0, t1 = t3 ? t3[1] : 0, t2 = t3 ? t3[2] : 0;
#define FC(p)                                                                                     \
  case p:                                                                                         \
    hipLaunchKernelGGL(k_face<p>, grid, block, 0, st, m, mode, face, t0, t1, t2, scale, eps, z0, \
                       origin_z, u, f, red, do_red);                                              \
    break;
  switch (P) {
    FC(1) FC(2) FC(3) FC(4) FC(5) FC(6) FC(7) FC(8)
    default: return -2;
  }
#undef FC
  if (f && m.stage && launch_stage_gather_face(P, m, face, f, st)) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------ instantiations
template int launch_fill<double>(double *, double, int64_t, hipStream_t);
template int launch_fill<float>(float *, float, int64_t, hipStream_t);
template int launch_fill<int>(int *, int, int64_t, hipStream_t);
template int launch_convert<float, double>(float *, const double *, double, int64_t, hipStream_t);
template int launch_convert<double, float>(double *, const float *, double, int64_t, hipStream_t);
template int launch_convert<double, double>(double *, const double *, double, int64_t, hipStream_t);
template int launch_convert<float, float>(float *, const float *, double, int64_t, hipStream_t);
template int launch_bc<double>(double *, int, const MeshK<double> &, hipStream_t);
template int launch_bc<float>(float *, int, const MeshK<float> &, hipStream_t);
template int launch_dot2<double>(const double *, const double *, int64_t, Reduce, hipStream_t);
template int launch_dot2<float>(const float *, const float *, int64_t, Reduce, hipStream_t);
template int launch_pcg_init<double>(const double *, const double *, double *, PcgDev *, double,
                                     int, double, int64_t, Reduce, hipStream_t);
template int launch_pcg_init<float>(const float *, const float *, float *, PcgDev *, double, int,
                                    double, int64_t, Reduce, hipStream_t);
template int launch_pcg_update<double>(double *, double *, const double *, double *,
                                       const double *, PcgDev *, int64_t, Reduce, hipStream_t,
                                       const double *);
template int launch_pcg_update<float>(float *, float *, const float *, float *, const float *,
                                      PcgDev *, int64_t, Reduce, hipStream_t, const float *);
template int launch_pcg_xflush<double>(double *, const double *, PcgDev *, int64_t, hipStream_t);
template int launch_pcg_xflush<float>(float *, const float *, PcgDev *, int64_t, hipStream_t);
template int launch_pcg_pupdate<double>(double *, const double *, const double *, const PcgDev *,
                                        int64_t, hipStream_t);
template int launch_pcg_pap<double>(const double *, const double *, PcgDev *, int64_t, Reduce,
                                    hipStream_t);
template int launch_pcg_pap<float>(const float *, const float *, PcgDev *, int64_t, Reduce,
                                   hipStream_t);
template int launch_pcg_pupdate<float>(float *, const float *, const float *, const PcgDev *,
                                       int64_t, hipStream_t);

}  // namespace sdme
