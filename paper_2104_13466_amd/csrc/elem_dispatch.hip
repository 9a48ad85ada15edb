// Runtime dispatch on the polynomial order to the per-order element-kernel
// wrappers (each order is compiled in its own translation unit).
#include <hip/hip_runtime.h>

#include "sdme_device.h"
#include "sdme_launch.h"

namespace sdme {

template <int P, typename T>
int launch_force_t(const MeshK<T> &, const double *, const double *, const T *, T *, T *, int,
                   hipStream_t);
template <int P, typename T>
int launch_tangent_t(const MeshK<T> &, const double *, const double *, const T *, const T *, T,
                     const T *, T *, int, const PUpd<T> *, const int *, hipStream_t);
template <int P, typename T>
int launch_mass_t(const MeshK<T> &, T, const T *, T *, int, Reduce, int, const int *, hipStream_t);
template <int P, typename T>
int mass_blocks_t(const MeshK<T> &);
template <int P, typename T>
int launch_diag_t(const MeshK<T> &, const double *, const double *, const T *, T, T *, int,
                  hipStream_t);
template <int P>
int launch_energy_t(const MeshK<double> &, const double *, const double *, const double *, Reduce,
                    hipStream_t);
template <int P>
int launch_matgrad_t(const MeshK<double> &, const double *, const double *, double, double *,
                     double *, hipStream_t);

#define SDME_DISPATCH(P_, CALL) \
  switch (P_) {                 \
    case 1: return CALL(1);     \
    case 2: return CALL(2);     \
    case 3: return CALL(3);     \
    case 4: return CALL(4);     \
    case 5: return CALL(5);     \
    case 6: return CALL(6);     \
    case 7: return CALL(7);     \
    case 8: return CALL(8);     \
    default: return -2;         \
  }

template <typename T>
int launch_force(int P, const MeshK<T> &m, const double *mu, const double *lam, const T *u, T *R,
                 T *state, int mask, hipStream_t st) {
#define C(p) launch_force_t<p, T>(m, mu, lam, u, R, state, mask, st)
  SDME_DISPATCH(P, C)
#undef C
}
template <typename T>
int launch_tangent(int P, const MeshK<T> &m, const double *mu, const double *lam, const T *ulin,
                   const T *state, T msr, const T *v, T *y, int mask, const PUpd<T> *pu,
                   const int *skip, hipStream_t st) {
#define C(p) launch_tangent_t<p, T>(m, mu, lam, ulin, state, msr, v, y, mask, pu, skip, st)
  SDME_DISPATCH(P, C)
#undef C
}
template <typename T>
int launch_mass(int P, const MeshK<T> &m, T rho, const T *v, T *y, int mask, Reduce red,
                int do_red, const int *skip, hipStream_t st) {
#define C(p) launch_mass_t<p, T>(m, rho, v, y, mask, red, do_red, skip, st)
  SDME_DISPATCH(P, C)
#undef C
}
template <typename T>
int launch_diag(int P, const MeshK<T> &m, const double *mu, const double *lam, const T *state,
                T msr, T *d, int mask, hipStream_t st) {
#define C(p) launch_diag_t<p, T>(m, mu, lam, state, msr, d, mask, st)
  SDME_DISPATCH(P, C)
#undef C
}
template <typename T>
int mass_blocks(int P, const MeshK<T> &m) {
#define C(p) mass_blocks_t<p, T>(m)
  SDME_DISPATCH(P, C)
#undef C
}
template int mass_blocks<double>(int, const MeshK<double> &);
template int mass_blocks<float>(int, const MeshK<float> &);

int launch_energy(int P, const MeshK<double> &m, const double *mu, const double *lam,
                  const double *u, Reduce red, hipStream_t st) {
#define C(p) launch_energy_t<p>(m, mu, lam, u, red, st)
  SDME_DISPATCH(P, C)
#undef C
}
int launch_matgrad(int P, const MeshK<double> &m, const double *u, const double *w, double scale,
                   double *gm, double *gl, hipStream_t st) {
#define C(p) launch_matgrad_t<p>(m, u, w, scale, gm, gl, st)
  SDME_DISPATCH(P, C)
#undef C
}

namespace {
struct TileShape {
  int ne, tx, tile;
};
template <class D>
TileShape shape_of() {
  return {D::NE, D::TX, D::TILE};
}
// Elements per block, tile slots along x and tile words of an element kernel
// launch with a gradient (the mass kernel has no tile).
TileShape tile_shape(int P, int Q, int word) {
  const int g = Q == P + 1 ? 1 : 0;
  switch (P * 100 + g * 10 + (word == 8 ? 1 : 0)) {
#define NEC(p)                                                 \
  case p * 100 + 1: return shape_of<Dims<p, p + 2, 8>>();  \
  case p * 100 + 0: return shape_of<Dims<p, p + 2, 4>>();  \
  case p * 100 + 11: return shape_of<Dims<p, p + 1, 8>>(); \
  case p * 100 + 10: return shape_of<Dims<p, p + 1, 4>>();
    NEC(1) NEC(2) NEC(3) NEC(4) NEC(5) NEC(6) NEC(7) NEC(8)
#undef NEC
    default: return {1, P + 1, 3 * (P + 1) * (P + 1) * (P + 1)};
  }
}
// Upper bound of the mass kernel's blocks (one z chunk per element).
int mass_blocks_max(int P, int word, int nx, int ny, int nz) {
  switch (P * 10 + (word == 8 ? 1 : 0)) {
#define NEM(p)                                                                         \
  case p * 10 + 1: return kron_grid<KronDims<p, 8>>(nx, ny, nz, 1 << 30).blocks(); \
  case p * 10 + 0: return kron_grid<KronDims<p, 4>>(nx, ny, nz, 1 << 30).blocks();
    NEM(1) NEM(2) NEM(3) NEM(4) NEM(5) NEM(6) NEM(7) NEM(8)
#undef NEM
    default: return 1;
  }
}
}  // namespace

int elem_blocks(int P, int Q, int word, int nx, int ny, int nz, bool grad) {
  if (!grad) return mass_blocks_max(P, word, nx, ny, nz);
  const int ne = tile_shape(P, Q, word).ne;
  return ((nx + ne - 1) / ne) * ny * nz;
}
int elem_tile_words(int P, int Q, int word, bool grad) {
  return grad ? tile_shape(P, Q, word).tile : 0;
}

template int launch_force<double>(int, const MeshK<double> &, const double *, const double *,
                                  const double *, double *, double *, int, hipStream_t);
template int launch_force<float>(int, const MeshK<float> &, const double *, const double *,
                                 const float *, float *, float *, int, hipStream_t);
template int launch_tangent<double>(int, const MeshK<double> &, const double *, const double *,
                                    const double *, const double *, double, const double *,
                                    double *, int, const PUpd<double> *, const int *, hipStream_t);
template int launch_tangent<float>(int, const MeshK<float> &, const double *, const double *,
                                   const float *, const float *, float, const float *, float *,
                                   int, const PUpd<float> *, const int *, hipStream_t);
template int launch_mass<double>(int, const MeshK<double> &, double, const double *, double *,
                                 int, Reduce, int, const int *, hipStream_t);
template int launch_mass<float>(int, const MeshK<float> &, float, const float *, float *, int,
                                Reduce, int, const int *, hipStream_t);
template int launch_diag<double>(int, const MeshK<double> &, const double *, const double *,
                                 const double *, double, double *, int, hipStream_t);
template int launch_diag<float>(int, const MeshK<float> &, const double *, const double *,
                                const float *, float, float *, int, hipStream_t);

}  // namespace sdme
