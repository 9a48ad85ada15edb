// Host-side launch wrappers shared between the kernel and API translation
// units of libsdme (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "sdme_device.h"

namespace sdme {

// ------------------------------------------------------------ element kernels
template <typename T>
int launch_force(int P, const MeshK<T> &m, const double *mu, const double *lam, const T *u, T *R,
                 T *state, int mask, hipStream_t st);
// Search-direction update fused into the PCG operator: while gathering its
// input the operator forms p = r * dinv + beta * v (v = the previous p) and
// stores p to pnew (from every block whose tile holds the slot: identical
// values).
template <typename T>
struct PUpd {
  const T *r;
  const T *dinv;
  T *pnew;
  const double *beta;
  // block partials [2 b] of p^T A p (the element-energy form, see the
  // tangent kernel), summed by launch_pcg_pap_fin; nullptr: not formed
  double *pap;
};
template <typename T>
int launch_tangent(int P, const MeshK<T> &m, const double *mu, const double *lam, const T *ulin,
                   const T *state, T msr, const T *v, T *y, int mask, const PUpd<T> *pu,
                   const int *skip, hipStream_t st);
// y = rho M v, every slot of y written (constrained slots as zero with
// mask); do_red: block partials of v^T y in red.partials[2 b], over the
// mass_blocks(P, m) blocks of the launch.
template <typename T>
int launch_mass(int P, const MeshK<T> &m, T rho, const T *v, T *y, int mask, Reduce red,
                int do_red, const int *skip, hipStream_t st);
template <typename T>
int mass_blocks(int P, const MeshK<T> &m);
template <typename T>
int launch_diag(int P, const MeshK<T> &m, const double *mu, const double *lam, const T *state,
                T msr, T *d, int mask, hipStream_t st);
int launch_energy(int P, const MeshK<double> &m, const double *mu, const double *lam,
                  const double *u, Reduce red, hipStream_t st);
int launch_matgrad(int P, const MeshK<double> &m, const double *u, const double *w, double scale,
                   double *gm, double *gl, hipStream_t st);
// Blocks of an element kernel launch with Q points per direction (grad =
// false: the value-only mass kernel).
int elem_blocks(int P, int Q, int word, int nx, int ny, int nz, bool grad = true);
// Words of one block's output tile (the staging stride of the ordered
// assembly; 0 for the mass kernel, which writes every slot once).
int elem_tile_words(int P, int Q, int word, bool grad = true);
// Deterministic assembly: y[slot] = sum of the staged tiles holding the slot
// (runs of ne elements, tiles of tx slots along x, stride tile words), in
// ascending block order; constrained slots get 0 with mask.
template <typename T>
int launch_stage_gather(int P, const MeshK<T> &m, int ne, int tx, int tile, int mask, T *y,
                        const int *skip, hipStream_t st);
// The same over element vectors [E][3][(P+1)^3] (the Jacobi diagonal).
template <typename T>
int launch_stage_gather_elem(int P, const MeshK<T> &m, int mask, T *y, hipStream_t st);
// The same over face-element vectors [fe][3][(P+1)^2] of one boundary face.
int launch_stage_gather_face(int P, const MeshK<double> &m, int face, double *f, hipStream_t st);

// ------------------------------------------------------------- face kernels
// mode 0: traction f += scale * int N t dA on face `face`
// mode 1: penalty force from u (plane z0) on face z=0, energy into red
// mode 2: penalty stiffness apply y_z += eps int N N x_z dA (all points active)
int launch_face(int P, const MeshK<double> &m, int mode, int face, const double *t3, double scale,
                double eps, double z0, double origin_z, const double *u, double *f, Reduce red,
                int do_red, hipStream_t st);
int face_blocks(const MeshK<double> &m, int face);

// ------------------------------------------------- loads at quadrature points
// f += int N b dV with b at the volume Gauss points [3][E][Q^3]
int launch_body_load(int P, const MeshK<double> &m, const double *b, double *f, hipStream_t st);
// f += int_face N t dA with t at the face Gauss points [3][nfe][(P+1)^2]
int launch_face_load(int P, const MeshK<double> &m, int face, const double *t, double *f,
                     hipStream_t st);
// out[c] = sum_e sum_q w detJ (u_h - g)^2 at the volume Gauss points; partials
// of 3 doubles per block, at most max_blocks blocks
int launch_l2_error(int P, const MeshK<double> &m, const double *u, const double *g,
                    double *partials, int max_blocks, double *out, hipStream_t st);

// ------------------------------------------------- static condensation (FP64)
// interior modes per element, 3 (P - 1)^3
int interior_size(int P);
// Kii [E][nI][nI] = interior block of K_T + (msr / rho) rho M from the stored state
int launch_interior_block(int P, const MeshK<double> &m, const double *mu, const double *lam,
                          const double *state, double msr, double *Kii, hipStream_t st);
// Kii -> inv(Kii) in place; *flag |= 1 on a non-positive pivot
int launch_interior_invert(int P, int E, double *Kii, int *flag, hipStream_t st);
// y_I = scale inv(K_II) t_I on every element's interior slots
int launch_interior_apply(int P, const MeshK<double> &m, const double *Kinv, const double *t,
                          double *y, double scale, const int *skip, hipStream_t st);
// x = val on every interior slot
int launch_interior_set(int P, const MeshK<double> &m, double *x, double val, const int *skip,
                        hipStream_t st);

// ------------------------------------------------------------ vector kernels
// PCG scalars living in device memory (all double).
struct PcgDev {
  double rz, pAp, rznew, rr, tol2, bb, alpha, beta;
  double upd2;   // residual-replacement threshold (mixed precision); 0 = off
  double rz_old; // r.z before the last update (for beta after a replacement)
  double alpha_pend;  // step length of the direction whose x update is pending
  int done;  // 0 running, 1 converged, 2 breakdown, 3 non-finite, 4 iteration limit,
             // 5 residual replacement requested
  int iters;
  int maxit;
  int xpend;  // 1: x lacks alpha_pend times the previous direction (deferred update)
};

constexpr int VEC_BLOCKS = 4096;
constexpr int VEC_THREADS = 256;

template <typename T>
int launch_fill(T *x, T val, int64_t n, hipStream_t st);
template <typename Td, typename Ts>
int launch_convert(Td *dst, const Ts *src, double scale, int64_t n, hipStream_t st);
int launch_axpby(double *y, double alpha, const double *x, double beta, int64_t n, hipStream_t st);
// y = alpha * x + beta * y + gamma * z
int launch_axpbypcz(double *y, double alpha, const double *x, double beta, double gamma,
                    const double *z, int64_t n, hipStream_t st);
// zero constrained entries (mode 0) or set them to one (mode 1)
template <typename T>
int launch_bc(T *x, int mode, const MeshK<T> &m, hipStream_t st);
// res[0] = sum x*y, res[1] = sum y*y (double accumulation)
template <typename T>
int launch_dot2(const T *x, const T *y, int64_t n, Reduce red2, hipStream_t st);
// x = 1 / x (inverse Jacobi diagonal for the PCG kernels)
int launch_recip(double *x, int64_t n, hipStream_t st);
// x += scale * double(e)
int launch_add_scaled_f(double *x, const float *e, double scale, int64_t n, hipStream_t st);

template <typename T>
int launch_pcg_init(const T *r, const T *d, T *p, PcgDev *s, double rtol, int maxit, double delta,
                    int64_t n, Reduce red2, hipStream_t st);
template <typename T>
int launch_pcg_update(T *x, T *r, const T *p, T *Ap, const T *d, PcgDev *s, int64_t n,
                      Reduce red2, hipStream_t st, const T *p_prev = nullptr);
// x += alpha_pend p (the update deferred by launch_pcg_update), xpend = 0
template <typename T>
int launch_pcg_xflush(T *x, const T *p, PcgDev *s, int64_t n, hipStream_t st);
template <typename T>
int launch_pcg_pupdate(T *p, const T *r, const T *d, const PcgDev *s, int64_t n, hipStream_t st);
// pAp = p . Ap (skipped when done)
template <typename T>
int launch_pcg_pap(const T *p, const T *Ap, PcgDev *s, int64_t n, Reduce red2, hipStream_t st);
// One-block finishing passes over nb block partials (written by a streaming or
// element kernel with a reduction): result[0..1], or the solver's p^T A p.
int launch_fin2(Reduce red2, int nb, hipStream_t st);
int launch_pcg_pap_fin(PcgDev *s, Reduce red2, int nb, hipStream_t st);
// residual replacement: r32 = float(r64); rz = r32.(r32/d); beta = rz/rz_old;
// done = (r64.r64 <= tol2); upd2 = delta^2 r64.r64; then p = r32/d + beta p
int launch_pcg_replace(float *r32, const double *r64, const float *d, float *p, PcgDev *s,
                       double delta, int64_t n, Reduce red2, bool update_p, hipStream_t st);

}  // namespace sdme
