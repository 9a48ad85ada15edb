// Device-side building blocks of libsdme (gfx950, wave64).
//
// Element kernels use a Q x Q thread slab per hexahedron: thread (i1, i2)
// owns the Gauss-point column (q1 = i1, q2 = i2, q3 = 0..Q-1).  Contractions
// along xi1 and xi2 go through LDS; the contraction along xi3, the pointwise
// constitutive update and the transposed xi3 contraction stay in registers.
// Several elements share a block of at most 256 threads (NE = 256 / Q^2).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sdme {

// Offset of the face tables (Bf [P+1][n], then Wf [P+1]) in the mesh tables
// of Dims<P, Q>: they follow B, D, W, B*B, D*D, B*D.
__host__ __device__ constexpr int face_table_offset(int n, int Q) { return 5 * Q * n + Q; }

// GRAD = false sizes the LDS regions for value-only contractions (the mass
// action: B tables only, one kind per stage).
template <int P_, int Q_, int WORD, bool GRAD = true>
struct Dims {
  static constexpr int P = P_, Q = Q_, n = P_ + 1;
  static constexpr int n3 = n * n * n;
  static constexpr int QQ = Q * Q;
  // tables: B, D (Q n), W (Q), B2, D2, BD (Q n), Bf (n n), Wf (n)
  static constexpr int TB = 0, TD = Q * n, TW = 2 * Q * n, TB2 = 2 * Q * n + Q,
                       TD2 = TB2 + Q * n, TBD = TD2 + Q * n, TBF = TBD + Q * n,
                       TWF = TBF + n * n, TSIZE = TWF + n;
  static_assert(TBF == face_table_offset(n, Q), "face table offset");
  // A block owns NE consecutive elements of one x-row of the mesh.  LDS:
  //  - per element, region A: the xi3-contracted fluxes g1..g3 of one
  //    component, [kind][c][q1][QP] with q2 fastest; region B: DBUF buffers
  //    of xi1 partial sums, [kind][c][q1][NP] with b fastest (forward) or
  //    [kind][c][b][QP] with q1 fastest (transposed).  Every row a thread
  //    reads is contiguous and 16-byte aligned (row lengths padded to
  //    multiples of VW words) so that it is read with wide LDS loads.  Three
  //    buffers let the xi1 stages of the three components run before a
  //    single barrier, two let consecutive components overlap;
  //  - per block, the tile: the block's slots [3][n][n][TX] with
  //    TX = NE P + 1 (input gathered once, then the output accumulated),
  //    and the 64-bit global offsets of its 3 n^2 rows (RW words).
  static constexpr int VW = 16 / WORD;
  static constexpr int rup(int x) { return (x + VW - 1) / VW * VW; }
  static constexpr int NP = rup(n), QP = rup(Q);
  static constexpr int KA = GRAD ? 3 : 1, KB = GRAD ? 2 : 1;
  static constexpr int SA = KA * n * Q * QP;
  static constexpr int SB1 = (KB * n * Q * NP > KB * n * n * QP) ? KB * n * Q * NP : KB * n * n * QP;
  static constexpr int NE_T = (256 / QQ) > 0 ? (256 / QQ) : 1;
  static constexpr int ROWS = 3 * n * n;
  static constexpr int RW = rup(ROWS * 8 / WORD);
  // at most 96 KiB of LDS per block (gfx950 has 160 KiB per CU)
  static constexpr int LDS_CAP = 98304;
  static constexpr int lds_words(int ne, int dbuf) {
    return ne * (SA + dbuf * SB1) + 3 * n * n * (ne * P + 1) + TSIZE + RW;
  }
  static constexpr int ne_fit(int dbuf) {
    int ne = NE_T;
    while (ne > 1 && lds_words(ne, dbuf) * WORD > LDS_CAP) ne--;
    return ne;
  }
  // three buffers (the xi1 stages of all components before one barrier) when
  // they fit in 80 KiB, else two, else one
#ifndef SDME_TRIPLE
#define SDME_TRIPLE 1
#endif
  static constexpr int DBUF = (SDME_TRIPLE && lds_words(NE_T, 3) * WORD <= 81920) ? 3
                              : (lds_words(1, 2) * WORD <= LDS_CAP)             ? 2
                                                                                : 1;
  static constexpr int NE = ne_fit(DBUF);
  static constexpr int SB = DBUF * SB1;
  static constexpr int SE = SA + SB;
  static constexpr int NT = NE * QQ;
  static constexpr int TX = NE * P + 1;
  static constexpr int TILE = 3 * n * n * TX;
};

// Mass action on affine hexahedra with one density: the element mass is
// rho detJ (Mq x Mq x Mq), Mq[a][b] = sum_q w_q B[q][a] B[q][b] the 1D mass
// of the rule, so the assembled mass is rho detJ times the Kronecker product
// of the three assembled 1D masses (banded: a slot couples with the slots of
// the elements it belongs to).  A block owns a box of output slots: EX
// elements along x (one lane per slot), EY along y (each wave RY rows of one
// element) and a chunk of elements along z, which it marches through plane by
// plane: the x and y passes of each input plane run through LDS, the z pass
// accumulates in registers per element, and every output slot is written
// once (no atomics).  Element indices run to n_d inclusive along each
// direction: the last "element" n_d only owns the final vertex slot.
template <int P_, int WORD>
struct KronDims {
  static constexpr int P = P_, n = P_ + 1;
  // Waves per block: 12 where the kernel's registers fit 3 waves per SIMD
  // per block (FP32 P <= 5, FP64 P <= 4), else 8 (FP32) or 4 (FP64)
  // (measured at ~2e7 DOF for P = 2, 4, 6).  MQR: the 1D mass held in
  // registers (where they are free at that occupancy), else read from LDS.
#ifdef SDME_KRON_WAVES
  static constexpr int WAVES = SDME_KRON_WAVES;
#else
  static constexpr int WAVES = WORD == 4 ? (P_ <= 5 ? 12 : 8) : (P_ <= 4 ? 12 : 4);
#endif
#ifdef SDME_KRON_MQR
  static constexpr bool MQR = SDME_KRON_MQR;
#else
  static constexpr bool MQR = WORD == 4 ? P_ <= 7 : P_ <= 3;
#endif
  static constexpr int NT = 64 * WAVES;
  static constexpr int EX = 64 / P_, TX = EX * P_;
  // rows per wave: one element's P rows, or half of them at P = 8 (register
  // budget of the z accumulators)
  static constexpr int RY = P_ == 8 ? 4 : P_;
  static constexpr int GPE = P_ / RY, EY = WAVES / GPE, TY = EY * P_;
  // input plane (x0 - P .. x0 + TX, y0 - P .. y0 + TY) and x-filtered plane;
  // row pitches in 16-byte units (an element's slots are read and written
  // with wide LDS accesses where they are 16-byte aligned)
  static constexpr int IX = TX + P_ + 1, IY = TY + P_ + 1;
  static constexpr int VW = 16 / WORD;
  static constexpr int IXP = (IX + VW - 1) / VW * VW, TXP = (TX + VW - 1) / VW * VW;
  static constexpr int NLD = (IX * IY + NT - 1) / NT;
  // an element's P slots start 16-byte aligned in a row when P is a
  // multiple of the vector width
  static constexpr bool VEC = P_ % VW == 0;
};
// Launch shape of the mass kernel: x, y tiles and z chunks of cz elements,
// as many chunks as keep the grid within `target` blocks (the blocks the
// device holds at once, so that every block starts at once).
struct KronGrid {
  int nxt, nyt, nzc, cz;
  __host__ __device__ int blocks() const { return nxt * nyt * nzc * 3; }
};
template <class D>
__host__ __device__ inline KronGrid kron_grid(int nx, int ny, int nz, int target) {
  KronGrid g;
  g.nxt = (nx + D::EX) / D::EX;  // elements 0 .. nx
  g.nyt = (ny + D::EY) / D::EY;
  const int base = g.nxt * g.nyt * 3;
  int nzc = target / base;
  nzc = nzc < 1 ? 1 : (nzc > nz ? nz : nzc);
  g.cz = (nz + nzc - 1) / nzc;
  g.nzc = (nz + g.cz - 1) / g.cz;
  return g;
}

// Mesh parameters passed by value to every kernel.
template <typename T>
struct MeshK {
  int nx, ny, nz, E;
  int Nx, Ny, Nz, Nn;
  int Q;         // volume points per direction: P + 2 (Gauss-Legendre) or P + 1 (GLL)
  uint32_t bc;   // Dirichlet bits (face*3 + comp)
  T ih[3];       // 2 / h_J  (reference-to-physical derivative scale)
  T detJ;        // h_x h_y h_z / 8
  const T *tab;  // device basis tables (layout of Dims)
  int *flag;     // device status words: [0] set to 1 when det F <= 0 at a Gauss
                 // point, [1] the smallest index of an element where it was
  // deterministic assembly: element kernels store their blocks' output tiles
  // (or element vectors) here and a gather kernel sums every slot's
  // contributions in a fixed order; nullptr: hardware atomics
  T *stage;
};

// Deterministic block reduction target: each block writes a partial, the last
// block to finish sums all partials in block order into *result.
struct Reduce {
  double *partials;
  unsigned *counter;
  double *result;
};

__device__ __forceinline__ bool is_constrained(uint32_t bc, int comp, int ix, int iy, int iz,
                                               int Nx, int Ny, int Nz) {
  uint32_t m = bc >> comp;
  return ((m & 1u) && ix == 0) || (((m >> 3) & 1u) && ix == Nx - 1) ||
         (((m >> 6) & 1u) && iy == 0) || (((m >> 9) & 1u) && iy == Ny - 1) ||
         (((m >> 12) & 1u) && iz == 0) || (((m >> 15) & 1u) && iz == Nz - 1);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block-wide sum of v (all threads call); returns the block total in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *s_red) {
  constexpr int NW = (NT + 63) / 64;
  v = wave_sum(v);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s_red[wid] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NW; i++) t += s_red[i];
  return t;
}

// Finish a deterministic grid reduction: thread 0 of each block passes its
// block total; the last block sums all partials in order.
template <int NT>
__device__ __forceinline__ void grid_reduce_finish(double block_total, Reduce r, double *s_red,
                                                   int nblocks) {
  __shared__ bool s_last;
  if (threadIdx.x == 0) {
    r.partials[blockIdx.x] = block_total;
    __threadfence();
    unsigned prev = atomicAdd(r.counter, 1u);
    s_last = (prev == (unsigned)nblocks - 1);
  }
  __syncthreads();
  if (s_last) {
    __threadfence();
    double t = 0;
    for (int i = threadIdx.x; i < nblocks; i += NT) t += __builtin_nontemporal_load(&r.partials[i]);
    t = block_sum<NT>(t, s_red);
    if (threadIdx.x == 0) {
      *r.result = t;
      *r.counter = 0u;
    }
  }
}

// ----------------------------------------------------------- 3x3 kinematics
// Compressible neo-Hookean quantities from H = grad u (F = I + H), written
// without cancellation at small strain:
//   J - 1 = I1(H) + I2(H) + I3(H),  ln J = log1p(J - 1),
//   F - F^-T = (H + H^T + H H^T) F^-T.
template <typename T>
struct Kin {
  T G[9];   // F^-1
  T lnJ;
  T Jm1;
};

template <typename T>
__device__ __forceinline__ T t_log1p(T x);
template <>
__device__ __forceinline__ double t_log1p<double>(double x) { return log1p(x); }
template <>
__device__ __forceinline__ float t_log1p<float>(float x) { return log1pf(x); }

template <typename T>
__device__ __forceinline__ bool kinematics(const T H[9], Kin<T> &k) {
  T I1 = H[0] + H[4] + H[8];
  T I2 = H[0] * H[4] - H[1] * H[3] + H[0] * H[8] - H[2] * H[6] + H[4] * H[8] - H[5] * H[7];
  T I3 = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
         H[2] * (H[3] * H[7] - H[4] * H[6]);
  T Jm1 = I1 + I2 + I3;
  T J = T(1) + Jm1;
  k.Jm1 = Jm1;
  if (!(J > T(0))) return false;
  k.lnJ = t_log1p<T>(Jm1);
  T F0 = T(1) + H[0], F4 = T(1) + H[4], F8 = T(1) + H[8];
  T iJ = T(1) / J;
  k.G[0] = (F4 * F8 - H[5] * H[7]) * iJ;
  k.G[1] = (H[2] * H[7] - H[1] * F8) * iJ;
  k.G[2] = (H[1] * H[5] - H[2] * F4) * iJ;
  k.G[3] = (H[5] * H[6] - H[3] * F8) * iJ;
  k.G[4] = (F0 * F8 - H[2] * H[6]) * iJ;
  k.G[5] = (H[2] * H[3] - F0 * H[5]) * iJ;
  k.G[6] = (H[3] * H[7] - F4 * H[6]) * iJ;
  k.G[7] = (H[1] * H[6] - F0 * H[7]) * iJ;
  k.G[8] = (F0 * F4 - H[1] * H[3]) * iJ;
  return true;
}

// First Piola-Kirchhoff stress P = mu (F - F^-T) + lam lnJ F^-T
//   = [mu (H + H^T + H H^T) + lam lnJ I] F^-T.
template <typename T>
__device__ __forceinline__ void first_pk(const T H[9], const Kin<T> &k, T mu, T lam, T Pk[9]) {
  T Bm[9];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      T hh = H[i * 3 + 0] * H[j * 3 + 0] + H[i * 3 + 1] * H[j * 3 + 1] + H[i * 3 + 2] * H[j * 3 + 2];
      Bm[i * 3 + j] = mu * (H[i * 3 + j] + H[j * 3 + i] + hh);
    }
  T ll = lam * k.lnJ;
  Bm[0] += ll; Bm[4] += ll; Bm[8] += ll;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int J = 0; J < 3; J++)
      Pk[i * 3 + J] = Bm[i * 3 + 0] * k.G[J * 3 + 0] + Bm[i * 3 + 1] * k.G[J * 3 + 1] +
                      Bm[i * 3 + 2] * k.G[J * 3 + 2];
}

// Linearised stress dP = mu dF + c1 (G dF G)^T + lam tr(G dF) G^T with
// G = F^-1 and c1 = mu - lam lnJ (derivative of P along dF).
template <typename T>
__device__ __forceinline__ void tangent_dp(const T G[9], T c1, T mu, T lam, const T dF[9],
                                           T dP[9]) {
  T A[9];
#pragma unroll
  for (int I = 0; I < 3; I++)
#pragma unroll
    for (int L = 0; L < 3; L++)
      A[I * 3 + L] = G[I * 3 + 0] * dF[0 * 3 + L] + G[I * 3 + 1] * dF[1 * 3 + L] +
                     G[I * 3 + 2] * dF[2 * 3 + L];
  T trA = lam * (A[0] + A[4] + A[8]);
#pragma unroll
  for (int J = 0; J < 3; J++)
#pragma unroll
    for (int i = 0; i < 3; i++) {
      // (A G)_{J i}
      T AG = A[J * 3 + 0] * G[0 * 3 + i] + A[J * 3 + 1] * G[1 * 3 + i] + A[J * 3 + 2] * G[2 * 3 + i];
      dP[i * 3 + J] = mu * dF[i * 3 + J] + c1 * AG + trA * G[J * 3 + i];
    }
}

}  // namespace sdme
