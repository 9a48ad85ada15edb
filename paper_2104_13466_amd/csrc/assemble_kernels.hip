// Ordered assembly: the alternative to hardware atomics in the scatter of
// element contributions to global slots (the assembly over elements of
// Section 2's topological association).  The element kernels store their
// output (a block's tile of slots, an element vector or a face-element
// vector) in a staging array; one thread per global slot then adds every
// staged copy of the slot in ascending block / element order and adds the
// sum to the output.  Inside a tile a slot receives at most two element
// contributions (neighbours along x), each added once to zero, which is exact
// in either order; so the assembled vector has the same bits on every run,
// and Krylov iterations built on it repeat exactly.
#include <hip/hip_runtime.h>

#include "sdme_device.h"
#include "sdme_launch.h"

namespace sdme {
namespace {

constexpr int NTG = 256;

// The (at most two) runs of `span` grid intervals that contain grid index g
// along one direction, with g's local index in each, ascending; runs past
// `runs` do not exist.
__device__ __forceinline__ int runs_of(int g, int span, int runs, int (&k)[2], int (&l)[2]) {
  const int k1 = g / span, l1 = g - k1 * span;
  int c = 0;
  if (l1 == 0 && k1 > 0) {
    k[c] = k1 - 1;
    l[c] = span;
    c++;
  }
  if (k1 < runs) {
    k[c] = k1;
    l[c] = l1;
    c++;
  }
  return c;
}

inline int grid_for(int64_t n) {
  const int64_t b = (n + NTG - 1) / NTG;
  return (int)(b < (1 << 20) ? (b > 0 ? b : 1) : (1 << 20));
}

// Tiles of the element kernels: block (ez ny + ey) bpr + k holds the slots
// x0 .. x0 + tx - 1 (x0 = k ne P) of rows ey P + b, ez P + c as
// tile[((comp n + c) n + b) tx + x].
template <typename T>
__global__ __launch_bounds__(NTG) void k_gather_tiles(MeshK<T> m, int P, int ne, int tx, int tile,
                                                      int mask, const T *__restrict__ stage,
                                                      T *__restrict__ y,
                                                      const int *__restrict__ skip) {
  if (skip && *skip) return;
  const int n = P + 1, bpr = (m.nx + ne - 1) / ne, N = 3 * m.Nn;
  for (int gi = blockIdx.x * NTG + threadIdx.x; gi < N; gi += gridDim.x * NTG) {
    const int comp = gi / m.Nn, s = gi - comp * m.Nn;
    const int ix = s % m.Nx, iy = (s / m.Nx) % m.Ny, iz = s / (m.Nx * m.Ny);
    if (mask && is_constrained(m.bc, comp, ix, iy, iz, m.Nx, m.Ny, m.Nz)) continue;
    int kx[2], lx[2], ky[2], ly[2], kz[2], lz[2];
    const int cx = runs_of(ix, ne * P, bpr, kx, lx), cy = runs_of(iy, P, m.ny, ky, ly),
              cz = runs_of(iz, P, m.nz, kz, lz);
    T acc = T(0);
    for (int a = 0; a < cz; a++)
      for (int b = 0; b < cy; b++)
        for (int c = 0; c < cx; c++) {
          const size_t blk = ((size_t)kz[a] * m.ny + ky[b]) * bpr + kx[c];
          acc += stage[blk * tile + ((comp * n + lz[a]) * n + ly[b]) * tx + lx[c]];
        }
    y[gi] += acc;
  }
}

// Element vectors: stage[(e 3 + comp) n^3 + (c n + b) n + a] for element
// e = (ez ny + ey) nx + ex and local slot (a, b, c).
template <typename T>
__global__ __launch_bounds__(NTG) void k_gather_elems(MeshK<T> m, int P, int mask,
                                                      const T *__restrict__ stage,
                                                      T *__restrict__ y) {
  const int n = P + 1, n3 = n * n * n, N = 3 * m.Nn;
  for (int gi = blockIdx.x * NTG + threadIdx.x; gi < N; gi += gridDim.x * NTG) {
    const int comp = gi / m.Nn, s = gi - comp * m.Nn;
    const int ix = s % m.Nx, iy = (s / m.Nx) % m.Ny, iz = s / (m.Nx * m.Ny);
    if (mask && is_constrained(m.bc, comp, ix, iy, iz, m.Nx, m.Ny, m.Nz)) continue;
    int kx[2], lx[2], ky[2], ly[2], kz[2], lz[2];
    const int cx = runs_of(ix, P, m.nx, kx, lx), cy = runs_of(iy, P, m.ny, ky, ly),
              cz = runs_of(iz, P, m.nz, kz, lz);
    T acc = T(0);
    for (int a = 0; a < cz; a++)
      for (int b = 0; b < cy; b++)
        for (int c = 0; c < cx; c++) {
          const size_t e = ((size_t)kz[a] * m.ny + ky[b]) * m.nx + kx[c];
          acc += stage[(e * 3 + comp) * n3 + (lz[a] * n + ly[b]) * n + lx[c]];
        }
    y[gi] += acc;
  }
}

// Face-element vectors of face `face` (direction dir = face / 2, side face %
// 2; tangential directions t1 < t2): stage[(fe 3 + comp) n^2 + b n + a] for
// face element fe = j ne[t1] + i and local slot (a along t1, b along t2).
__global__ __launch_bounds__(NTG) void k_gather_faces(MeshK<double> m, int P, int face,
                                                      const double *__restrict__ stage,
                                                      double *__restrict__ f) {
  const int n = P + 1, dir = face / 2, side = face % 2;
  const int t1 = dir == 0 ? 1 : 0, t2 = dir == 2 ? 1 : 2;
  const int ne[3] = {m.nx, m.ny, m.nz}, Nd[3] = {m.Nx, m.Ny, m.Nz};
  const int F = Nd[t1] * Nd[t2];
  for (int gi = blockIdx.x * NTG + threadIdx.x; gi < 3 * F; gi += gridDim.x * NTG) {
    const int comp = gi / F, s = gi - comp * F, i = s % Nd[t1], j = s / Nd[t1];
    int ki[2], li[2], kj[2], lj[2];
    const int ci = runs_of(i, P, ne[t1], ki, li), cj = runs_of(j, P, ne[t2], kj, lj);
    double acc = 0.0;
    for (int b = 0; b < cj; b++)
      for (int a = 0; a < ci; a++) {
        const size_t fe = (size_t)kj[b] * ne[t1] + ki[a];
        acc += stage[(fe * 3 + comp) * n * n + lj[b] * n + li[a]];
      }
    int g[3];
    g[t1] = i;
    g[t2] = j;
    g[dir] = side ? Nd[dir] - 1 : 0;
    f[(size_t)comp * m.Nn + ((size_t)g[2] * m.Ny + g[1]) * m.Nx + g[0]] += acc;
  }
}

}  // namespace

template <typename T>
int launch_stage_gather(int P, const MeshK<T> &m, int ne, int tx, int tile, int mask, T *y,
                        const int *skip, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_tiles<T>, dim3(grid_for(3 * (int64_t)m.Nn)), dim3(NTG), 0, st, m,
                     P, ne, tx, tile, mask, (const T *)m.stage, y, skip);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_stage_gather_elem(int P, const MeshK<T> &m, int mask, T *y, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_elems<T>, dim3(grid_for(3 * (int64_t)m.Nn)), dim3(NTG), 0, st, m,
                     P, mask, (const T *)m.stage, y);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_stage_gather_face(int P, const MeshK<double> &m, int face, double *f,
                             hipStream_t st) {
  const int dir = face / 2, t1 = dir == 0 ? 1 : 0, t2 = dir == 2 ? 1 : 2;
  const int Nd[3] = {m.Nx, m.Ny, m.Nz};
  hipLaunchKernelGGL(k_gather_faces, dim3(grid_for(3 * (int64_t)Nd[t1] * Nd[t2])), dim3(NTG), 0,
                     st, m, P, face, (const double *)m.stage, f);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_stage_gather<double>(int, const MeshK<double> &, int, int, int, int, double *,
                                         const int *, hipStream_t);
template int launch_stage_gather<float>(int, const MeshK<float> &, int, int, int, int, float *,
                                        const int *, hipStream_t);
template int launch_stage_gather_elem<double>(int, const MeshK<double> &, int, double *,
                                              hipStream_t);
template int launch_stage_gather_elem<float>(int, const MeshK<float> &, int, float *,
                                             hipStream_t);

}  // namespace sdme
