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

// p^T A p of the PCG formed inside the operator with the fused direction
// update (1) or by a separate streaming dot (0)
#ifndef SDME_FUSED_PAP
#define SDME_FUSED_PAP 1
#endif


namespace sdme {

template <int P, int Q, typename T, bool GRAD = true>
struct EK {
  using Dm = Dims<P, Q, (int)sizeof(T), GRAD>;
  static constexpr int n = Dm::n, n3 = Dm::n3, QQ = Dm::QQ, NE = Dm::NE, NT = Dm::NT;
  static constexpr int SA = Dm::SA, SB = Dm::SB, SE = Dm::SE, TS = Dm::TSIZE;
  static constexpr int TX = Dm::TX, TILE = Dm::TILE, ROWS = Dm::ROWS, RW = Dm::RW;
  static constexpr int NP = Dm::NP, QP = Dm::QP, TILEP = Dm::rup(TILE);
  // basis tables as the contraction stages read them from LDS (rows padded
  // and aligned for wide loads): B as [Q][NP]; D scaled by 2/h of direction
  // d = 0, 1, 2 as [Q][NP] at LD + d DS (contractions with them give physical
  // derivatives); the transpose Bt and the scaled Dt of directions 0, 1 as
  // [n][QP] (at LDT + d DTS); the weights W[Q]
  static constexpr int DS = Dm::Q * NP, DTS = n * QP;
  static constexpr int LB = 0, LD = DS, LBT = 4 * DS, LDT = LBT + DTS, LW = LDT + 2 * DTS,
                       TSX = LW + Dm::Q;
  // shared memory words of a block: row offsets, per-element regions, the
  // tile, tables
  // x-face contributions of the transposed xi1 stage, [3 n n][NE] (see
  // stage1t_tile)
  static constexpr int FACEW = 3 * n * n * NE, FACEP = Dm::rup(FACEW);
  static constexpr int SMEM = RW + NE * SE + TILEP + FACEP + TSX;
  // Stored-state tangent action: PIPE selects DEPTH named buffers of
  // Gauss-point slabs requested ahead (the first DEPTH before the forward
  // contractions); otherwise one slab is prefetched per step.  Chosen by
  // measurement at ~2e7 DOF per order and precision (FP32, P >= 4); three
  // buffers where they keep the kernel within 256 VGPRs (P <= 6), two above.
#ifndef SDME_PIPE3
#define SDME_PIPE3 1
#endif
  static constexpr bool PIPE = sizeof(T) == 4 && P >= 4;
  static constexpr int DEPTH = (SDME_PIPE3 && P <= 6) ? 3 : 2;
  // every element's Q^2 threads lie in one wave (Q^2 divides the wave size):
  // the element-private LDS exchanges of the contraction stages then need
  // only a wave-level synchronisation
  static constexpr bool WAVE_ELEM = 64 % QQ == 0;
  // The xi1 contraction of the gradient kernels on the matrix cores: when one
  // element fills one wave (Q^2 = 64) and the stacked [B; D] table has
  // exactly 16 rows (2Q = 16, i.e. P = 6), in FP32 (v_mfma_f32_16x16x4f32).
#ifndef SDME_MFMA_XI1
#define SDME_MFMA_XI1 1
#endif
  static constexpr bool MFMA_XI1 =
      SDME_MFMA_XI1 && std::is_same<T, float>::value && QQ == 64 && 2 * Dm::Q == 16 && n <= 8;
};

// Thread/element coordinates inside a block.  Block b owns the run of NE
// consecutive elements ex = k NE .. k NE + NE - 1 of the x-row (ey, ez), with
// k = b mod ceil(nx / NE); elements past the end of the row are idle.
struct Slab {
  int le, t2, i1, i2, e, ex, ey, ez;
  int x0;     // first slot (x) of the block's tile
  bool valid;
  bool bnd;   // the block's tile touches a face carrying Dirichlet constraints
};

template <class K, typename T>
__device__ __forceinline__ Slab make_slab(const MeshK<T> &m) {
  Slab s;
  s.le = threadIdx.x / K::QQ;
  s.t2 = threadIdx.x % K::QQ;
  s.i1 = s.t2 % K::Dm::Q;
  s.i2 = s.t2 / K::Dm::Q;
  const int bpr = (m.nx + K::NE - 1) / K::NE;
  const int k = blockIdx.x % bpr, row = blockIdx.x / bpr;
  s.ey = row % m.ny;
  s.ez = row / m.ny;
  const int ex0 = k * K::NE;
  s.ex = ex0 + s.le;
  s.valid = s.ex < m.nx;
  s.e = (s.ez * m.ny + s.ey) * m.nx + (s.valid ? s.ex : 0);
  if (!s.valid) s.ex = m.nx - 1;
  s.x0 = ex0 * K::Dm::P;
  const uint32_t b = m.bc;
  const int exl = min(ex0 + K::NE, m.nx) - 1;
  s.bnd = (ex0 == 0 && (b & 07u)) || (exl == m.nx - 1 && (b & 070u)) ||
          (s.ey == 0 && (b & 0700u)) || (s.ey == m.ny - 1 && (b & 07000u)) ||
          (s.ez == 0 && (b & 070000u)) || (s.ez == m.nz - 1 && (b & 0700000u));
  return s;
}

template <class K>
__host__ __device__ constexpr int blocks_for(int nx, int ny, int nz) {
  return ((nx + K::NE - 1) / K::NE) * ny * nz;
}

template <class K, typename T>
__device__ __forceinline__ void load_tables(const MeshK<T> &m, T *s_tab) {
  for (int i = threadIdx.x; i < K::TS; i += K::NT) s_tab[i] = m.tab[i];
}

// The stage tables of EK (LB .. TSX) from the mesh tables (B, D as [Q][n]):
// entry i of the LDS tables, requested from global memory with one
// unconditional load (a valid index; padding entries are zeroed after).
template <class K, typename T>
__device__ __forceinline__ T stage_table_entry(const MeshK<T> &m, int i) {
  constexpr int n = K::n, Q = K::Dm::Q, NP = K::NP, QP = K::QP;
  using Dm = typename K::Dm;
  int src = Dm::TB, t = 0;
  bool pad = true;
  if (i < K::LBT) {  // B, D rows (t = 0: B; 1..3: D scaled by 2/h of direction t - 1)
    const int r = i % K::DS, q = r / NP, c = r % NP;
    t = i / K::DS;
    src = (t ? Dm::TD : Dm::TB) + q * n + c;
    pad = c >= n;
  } else if (i < K::LW) {  // Bt, Dt rows (t = 0: Bt; 1, 2: Dt of direction t - 1)
    const int j = i - K::LBT, r = j % K::DTS, a = r / QP, q = r % QP;
    t = j / K::DTS;
    src = (t ? Dm::TD : Dm::TB) + q * n + a;
    pad = q >= Q;
  } else if (i < K::TSX) {
    src = Dm::TW + (i - K::LW);
    pad = false;
  }
  const T v = m.tab[pad ? Dm::TB : src];
  const T sc = t == 1 ? m.ih[0] : t == 2 ? m.ih[1] : t == 3 ? m.ih[2] : T(1);
  return pad ? T(0) : v * sc;
}
template <class K>
constexpr int stage_table_nit() {
  return (K::TSX + K::NT - 1) / K::NT;
}
// Request a thread's table entries (registers), then store them to LDS.
template <class K, typename T>
__device__ __forceinline__ void request_stage_tables(const MeshK<T> &m,
                                                     T (&tv)[stage_table_nit<K>()]) {
#pragma unroll
  for (int k = 0; k < stage_table_nit<K>(); k++)
    tv[k] = stage_table_entry<K>(m, (int)threadIdx.x + k * K::NT);
}
template <class K, typename T>
__device__ __forceinline__ void store_stage_tables(const T (&tv)[stage_table_nit<K>()], T *s_tab) {
#pragma unroll
  for (int k = 0; k < stage_table_nit<K>(); k++) {
    const int i = (int)threadIdx.x + k * K::NT;
    if (i < K::TSX) s_tab[i] = tv[k];
  }
}

// Global offset of row r of the block's tile: row r = (comp n + c) n + b
// holds the slots (x0 .. x0 + TX - 1, ey P + b, ez P + c) of component comp.
template <class K, typename T>
__device__ __forceinline__ int64_t tile_row_offset(const MeshK<T> &m, const Slab &s, int r) {
  constexpr int n = K::n, P = K::Dm::P;
  const int b = r % n, c = (r / n) % n, comp = r / (n * n);
  return (int64_t)comp * m.Nn + ((int64_t)(s.ez * P + c) * m.Ny + (s.ey * P + b)) * m.Nx + s.x0;
}
// The row offsets of the tile, in LDS.
template <class K, typename T>
__device__ __forceinline__ void tile_rows(const MeshK<T> &m, const Slab &s, int64_t *s_row) {
  for (int r = threadIdx.x; r < K::ROWS; r += K::NT) s_row[r] = tile_row_offset<K>(m, s, r);
}

// Visit the tile slots idx = r TX + x, idx = threadIdx.x + k NT, with the
// (row, x) pair advanced incrementally (no divisions in the loop).
template <class K, typename F>
__device__ __forceinline__ void tile_for(F &&f) {
  constexpr int TX = K::TX, NT = K::NT, DX = NT % TX, DR = NT / TX;
  int x = threadIdx.x % TX, r = threadIdx.x / TX;
  for (int idx = threadIdx.x; idx < K::TILE; idx += NT) {
    f(idx, r, x);
    x += DX;
    r += DR;
    if (x >= TX) {
      x -= TX;
      r += 1;
    }
  }
}

// The same visit unrolled over the NIT = ceil(TILE / NT) slots of a thread:
// f(k, idx, r, x) for k = 0 .. NIT - 1 (idx >= TILE, with r >= ROWS, in the
// last step of some threads).  Two such visits let a thread issue all its
// loads before it waits for the first.
template <class K>
constexpr int tile_nit() {
  return (K::TILE + K::NT - 1) / K::NT;
}
template <class K, typename F>
__device__ __forceinline__ void tile_for_all(F &&f) {
  constexpr int TX = K::TX, NT = K::NT, DX = NT % TX, DR = NT / TX;
  int x = threadIdx.x % TX, r = threadIdx.x / TX;
#pragma unroll
  for (int k = 0; k < tile_nit<K>(); k++) {
    f(k, (int)threadIdx.x + k * NT, r, x);
    x += DX;
    r += DR;
    if (x >= TX) {
      x -= TX;
      r += 1;
    }
  }
}

// Global index of tile slot (r, x), clamped into the mesh and the tile rows:
// an address that is always safe to load (the value is discarded where the
// slot lies outside).  Computed from the mesh, so that requests can be issued
// before the row offsets are in LDS.
template <class K, typename T>
__device__ __forceinline__ int64_t tile_gidx(const MeshK<T> &m, const Slab &s, int r, int x,
                                             int xe) {
  return tile_row_offset<K>(m, s, min(r, K::ROWS - 1)) + min(x, xe - 1);
}

// Is slot x of tile row r a constrained DOF (only blocks with s.bnd)?
template <class K, typename T>
__device__ __forceinline__ bool tile_constrained(const MeshK<T> &m, const Slab &s, int r, int x) {
  constexpr int n = K::n, P = K::Dm::P;
  int b = r % n, c = (r / n) % n, comp = r / (n * n);
  return is_constrained(m.bc, comp, s.x0 + x, s.ey * P + b, s.ez * P + c, m.Nx, m.Ny, m.Nz);
}

// Cooperative, coalesced load of the block's tile: tile[comp][c][b][x] =
// v(comp, x0 + x, ey P + b, ez P + c) for x < TX inside the mesh (zero outside
// and, with mask, on constrained DOFs).
// In two phases: all of a thread's loads are requested (unconditionally, at
// clamped addresses) into registers, then stored to the tile.
template <class K, typename T>
__device__ __forceinline__ void tile_request(const MeshK<T> &m, const Slab &s,
                                             const T *__restrict__ v, T (&val)[tile_nit<K>()]) {
  const int xe = m.Nx - s.x0;  // tile slots x < xe lie inside the mesh
  tile_for_all<K>([&](int k, int idx, int r, int x) { val[k] = v[tile_gidx<K>(m, s, r, x, xe)]; });
}
template <class K, typename T>
__device__ __forceinline__ void tile_store(const MeshK<T> &m, const Slab &s,
                                           const T (&val)[tile_nit<K>()], bool mask, T *tile) {
  const int xe = m.Nx - s.x0;
  const bool chk = mask && s.bnd;
  tile_for_all<K>([&](int k, int idx, int r, int x) {
    if (idx < K::TILE)
      tile[idx] = (x < xe && !(chk && tile_constrained<K>(m, s, r, x))) ? val[k] : T(0);
  });
}
// Both phases once the row offsets are in LDS (addresses from s_row).
template <class K, typename T>
__device__ __forceinline__ void gather_tile(const MeshK<T> &m, const Slab &s, const int64_t *s_row,
                                            const T *__restrict__ v, bool mask, T *tile) {
  const int xe = m.Nx - s.x0;
  T val[tile_nit<K>()];
  tile_for_all<K>([&](int k, int idx, int r, int x) {
    val[k] = v[s_row[min(r, K::ROWS - 1)] + min(x, xe - 1)];
  });
  tile_store<K>(m, s, val, mask, tile);
}

// Contiguous, 16-byte aligned LDS row of N values (wide LDS loads).
template <int N, typename T>
__device__ __forceinline__ void lds_row(const T *p, T (&r)[N]) {
  const T *a = (const T *)__builtin_assume_aligned(p, 16);
#pragma unroll
  for (int k = 0; k < N; k++) r[k] = a[k];
}

// Gather of the PCG operator's input with the fused search-direction update:
// tile = p = r dinv + beta pold, and p stored to pu.pnew by every block whose
// tile holds the slot.  Blocks that share a slot compute bit-identical values
// from the same inputs with the same instructions, so the repeated stores are
// benign; no block reads pnew during the launch (it is the other direction
// buffer).  Storing only from the owning block cost more in predicate
// arithmetic than the repeated stores cost in bandwidth.
// Requests (registers; clamped addresses) and updates in separate phases,
// like tile_request and tile_store.
template <class K, typename T>
struct PuReq {
  T r[tile_nit<K>()], d[tile_nit<K>()], p[tile_nit<K>()];
};
template <class K, typename T>
__device__ __forceinline__ void tile_request_pu(const MeshK<T> &m, const Slab &s,
                                                const PUpd<T> &pu, const T *__restrict__ pold,
                                                PuReq<K, T> &q) {
  const int xe = m.Nx - s.x0;
  const T *__restrict__ r = pu.r;
  const T *__restrict__ d = pu.dinv;
  tile_for_all<K>([&](int k, int idx, int rr, int x) {
    const int64_t g = tile_gidx<K>(m, s, rr, x, xe);
    q.r[k] = r[g];
    q.d[k] = d[g];
    q.p[k] = pold[g];
  });
}
template <class K, typename T>
__device__ __forceinline__ void tile_store_pu(const MeshK<T> &m, const Slab &s,
                                              const int64_t *s_row, const PUpd<T> &pu,
                                              const PuReq<K, T> &q, T beta, bool mask, T *tile) {
  const int xe = m.Nx - s.x0;
  const bool chk = mask && s.bnd;
  T *__restrict__ pn = pu.pnew;
  tile_for_all<K>([&](int k, int idx, int rr, int x) {
    if (idx >= K::TILE) return;
    T val = T(0);
    if (x < xe) {
      val = q.r[k] * q.d[k] + beta * q.p[k];
      pn[s_row[rr] + x] = val;
      if (chk && tile_constrained<K>(m, s, rr, x)) val = T(0);
    }
    tile[idx] = val;
  });
}

// xi1 contraction of one component: st[0][c][q1][b] = sum_a B[q1][a]
// u[c][b][a], st[1][c][q1][b] with D (rows of NP); su points at the element's
// first slot in the tile (rows of stride TX).
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void stage1(const T *sB, const T *sD, const T *su, T *st, const Slab &s) {
  constexpr int n = K::n, Q = K::Dm::Q, TX = K::TX, NP = K::Dm::NP;
  if (s.i2 < n) {
    T rb[n], rd[n];
    lds_row<n>(sB + s.i1 * NP, rb);
    if (GRAD) lds_row<n>(sD + s.i1 * NP, rd);
#pragma unroll
    for (int c = 0; c < n; c++) {
      T sb = T(0), sd = T(0);
#pragma unroll
      for (int a = 0; a < n; a++) {
        T x = su[(c * n + s.i2) * TX + a];
        sb += rb[a] * x;
        if (GRAD) sd += rd[a] * x;
      }
      st[(c * Q + s.i1) * NP + s.i2] = sb;
      if (GRAD) st[((n + c) * Q + s.i1) * NP + s.i2] = sd;
    }
  }
}

// xi1 contraction of one component on the matrix cores (EK::MFMA_XI1): the
// 16 x 64 block out[(kind, q1)][(c, b)] = sum_a T_kind[q1][a] u[c][b][a]
// (T_0 = B, T_1 = D; a padded from n to 8, the n^2 columns (c, b) padded to
// 64) as four 16 x 16 tiles, each two 16x16x4 FP32 MFMA steps.  Operand
// layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[4 (l / 16) + r][l % 16], r = 0..3.  The
// lane's two table entries (A rows = (kind, q1), columns a = l/16 and
// l/16 + 4) are loaded once per kernel.
struct MfmaTab {
  float a0, a1;
};
template <class K>
__device__ __forceinline__ MfmaTab mfma_xi1_table(const float *sB, const float *sD) {
  constexpr int NP = K::Dm::NP;
  static_assert(NP >= 8, "padded table rows hold 8 entries");
  const int l = threadIdx.x & 63, m = l & 15, k = l >> 4;
  const float *row = m < 8 ? sB + m * NP : sD + (m - 8) * NP;
  return MfmaTab{row[k], row[k + 4]};  // entries past n are the rows' zero padding
}
template <class K>
__device__ __forceinline__ void stage1_mfma(const MfmaTab &t, const float *su, float *st) {
  constexpr int n = K::n, Q = K::Dm::Q, TX = K::TX, NP = K::Dm::NP;
  static_assert(2 * Q == 16 && n <= 8 && n * n <= 64, "MFMA xi1 shape");
  using f4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
  const int l = threadIdx.x & 63, col = l & 15, kr = l >> 4;
#pragma unroll
  for (int tt = 0; tt < 4; tt++) {
    const int nn = col + 16 * tt;
    const bool valid = nn < n * n;
    const int c = valid ? nn / n : 0, b = valid ? nn % n : 0;
    const float *urow = su + (c * n + b) * TX;
    const float x0 = valid ? urow[kr] : 0.f;
    const float x1 = (valid && kr + 4 < n) ? urow[kr + 4] : 0.f;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(t.a0, x0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(t.a1, x1, acc, 0, 0, 0);
    if (valid) {
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int m = 4 * kr + r, kind = m >> 3, q1 = m & 7;
        st[((kind * n + c) * Q + q1) * NP + b] = acc[r];
      }
    }
  }
}

// xi2 contraction into registers at column (q1, q2) = (i1, i2): X[0][c]
// (B in xi1, B in xi2), X[1][c] (B, D), X[2][c] (D, B).
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void stage2(const T *sB, const T *sD, const T *st, const Slab &s,
                                       T (&X)[3][K::n]) {
  constexpr int n = K::n, Q = K::Dm::Q, NP = K::Dm::NP;
  T rb[n], rd[n];
  lds_row<n>(sB + s.i2 * NP, rb);
  if (GRAD) lds_row<n>(sD + s.i2 * NP, rd);
#pragma unroll
  for (int c = 0; c < n; c++) {
    T t0[n], t1[n];
    lds_row<n>(st + (c * Q + s.i1) * NP, t0);
    if (GRAD) lds_row<n>(st + ((n + c) * Q + s.i1) * NP, t1);
    T bb = T(0), bd = T(0), db = T(0);
#pragma unroll
    for (int b = 0; b < n; b++) {
      bb += rb[b] * t0[b];
      if (GRAD) {
        bd += rd[b] * t0[b];
        db += rb[b] * t1[b];
      }
    }
    X[0][c] = bb;
    if (GRAD) {
      X[1][c] = bd;
      X[2][c] = db;
    }
  }
}

// Synchronisation of the threads of one element between contraction stages
// (exchanges through the element's private LDS regions): a wave barrier with
// LDS ordering when the element lies in one wave, else a block barrier.
template <class K>
__device__ __forceinline__ void elem_sync() {
  if constexpr (K::WAVE_ELEM) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Forward contractions of the three gathered components (tile, synchronised)
// into X[comp][kind][c]; sD: the scaled D tables, direction 0 first.  With three LDS buffers the xi1 stages of all
// components run before one barrier; with two, the xi1 stage of one component
// overlaps the xi2 stage of the previous one; with one, extra barriers.  Ends
// after a barrier that follows the last read of the tile.
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void forward_lds(const T *sB, const T *sD, const T *tile, T *st,
                                            const Slab &s, T (&X)[3][3][K::n]) {
  constexpr int n = K::n, SB1 = K::Dm::SB1, CS = n * n * K::TX, NB = K::Dm::DBUF;
  const T *su = tile + s.le * K::Dm::P;
  const T *sD2 = sD + K::DS;
  if constexpr (NB == 3 && GRAD && K::MFMA_XI1) {
    const MfmaTab mt = mfma_xi1_table<K>(sB, sD);
    stage1_mfma<K>(mt, su, st);
    stage1_mfma<K>(mt, su + CS, st + SB1);
    stage1_mfma<K>(mt, su + 2 * CS, st + 2 * SB1);
    __syncthreads();
    stage2<K, T, GRAD>(sB, sD2, st, s, X[0]);
    stage2<K, T, GRAD>(sB, sD2, st + SB1, s, X[1]);
    stage2<K, T, GRAD>(sB, sD2, st + 2 * SB1, s, X[2]);
  } else if constexpr (NB == 3) {
    stage1<K, T, GRAD>(sB, sD, su, st, s);
    stage1<K, T, GRAD>(sB, sD, su + CS, st + SB1, s);
    stage1<K, T, GRAD>(sB, sD, su + 2 * CS, st + 2 * SB1, s);
    __syncthreads();
    stage2<K, T, GRAD>(sB, sD2, st, s, X[0]);
    stage2<K, T, GRAD>(sB, sD2, st + SB1, s, X[1]);
    stage2<K, T, GRAD>(sB, sD2, st + 2 * SB1, s, X[2]);
  } else if constexpr (K::WAVE_ELEM) {
    // element-local exchanges; one block barrier once the tile has been read
    constexpr bool single = NB == 1;
    T *st1 = single ? st : st + SB1;
    stage1<K, T, GRAD>(sB, sD, su, st, s);
    elem_sync<K>();
    stage2<K, T, GRAD>(sB, sD2, st, s, X[0]);
    if (single) elem_sync<K>();
    stage1<K, T, GRAD>(sB, sD, su + CS, st1, s);
    elem_sync<K>();
    stage2<K, T, GRAD>(sB, sD2, st1, s, X[1]);
    if (single) elem_sync<K>();
    stage1<K, T, GRAD>(sB, sD, su + 2 * CS, st, s);
    __syncthreads();
    stage2<K, T, GRAD>(sB, sD2, st, s, X[2]);
  } else {
    constexpr bool single = NB == 1;
    T *st1 = single ? st : st + SB1;
    stage1<K, T, GRAD>(sB, sD, su, st, s);
    __syncthreads();
    stage2<K, T, GRAD>(sB, sD2, st, s, X[0]);
    if (single) __syncthreads();
    stage1<K, T, GRAD>(sB, sD, su + CS, st1, s);
    __syncthreads();
    stage2<K, T, GRAD>(sB, sD2, st1, s, X[1]);
    if (single) __syncthreads();
    stage1<K, T, GRAD>(sB, sD, su + 2 * CS, st, s);
    __syncthreads();
    stage2<K, T, GRAD>(sB, sD2, st, s, X[2]);
  }
}

// Physical gradient of the field at Gauss point (i1, i2, q3) from X (tab:
// the stage tables of EK).
template <class K, typename T>
__device__ __forceinline__ void grad_at(const MeshK<T> &m, const T *tab, int q3,
                                        const T (&X)[3][3][K::n], T H[9]) {
  constexpr int n = K::n;
  T bq[n], dq[n];
  lds_row<n>(tab + K::LB + q3 * K::NP, bq);
  lds_row<n>(tab + K::LD + 2 * K::DS + q3 * K::NP, dq);
#pragma unroll
  for (int i = 0; i < 3; i++) {
    T g0 = T(0), g1 = T(0), g2 = T(0);
#pragma unroll
    for (int c = 0; c < n; c++) {
      g0 += bq[c] * X[i][2][c];
      g1 += bq[c] * X[i][1][c];
      g2 += dq[c] * X[i][0][c];
    }
    H[i * 3 + 0] = g0;
    H[i * 3 + 1] = g1;
    H[i * 3 + 2] = g2;
  }
}

template <class K, typename T>
__device__ __forceinline__ void value_at(const T *tab, int q3, const T (&X)[3][3][K::n], T val[3]) {
  constexpr int n = K::n;
  T bq[n];
  lds_row<n>(tab + K::LB + q3 * K::NP, bq);
#pragma unroll
  for (int i = 0; i < 3; i++) {
    T g = T(0);
#pragma unroll
    for (int c = 0; c < n; c++) g += bq[c] * X[i][0][c];
    val[i] = g;
  }
}

// Transposed xi3 contraction: accumulate flux f (already scaled by the
// quadrature weight and detJ; the 2/h factors are in the D tables) and a
// value-type flux mv into A.
template <class K, typename T, bool GRAD, bool VAL>
__device__ __forceinline__ void accum_at(const T *tab, int q3, const T f[9], const T mv[3],
                                         T (&A)[3][3][K::n]) {
  constexpr int n = K::n;
  T bq[n], dq[n];
  lds_row<n>(tab + K::LB + q3 * K::NP, bq);
  if (GRAD) lds_row<n>(tab + K::LD + 2 * K::DS + q3 * K::NP, dq);
#pragma unroll
  for (int c = 0; c < n; c++) {
#pragma unroll
    for (int i = 0; i < 3; i++) {
      if (GRAD) {
        A[i][2][c] += bq[c] * f[i * 3 + 0];
        A[i][1][c] += bq[c] * f[i * 3 + 1];
        A[i][0][c] += dq[c] * f[i * 3 + 2];
      }
      if (VAL) A[i][0][c] += bq[c] * mv[i];
    }
  }
}

// Store the xi3-contracted fluxes of one component (kinds 0 BB-type, 1 BD,
// 2 DB) into sg[kind][c][q1][q2] (rows of QP).
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void write_g(const T (&A)[3][K::n], T *sg, const Slab &s) {
  constexpr int n = K::n, Q = K::Dm::Q, QP = K::Dm::QP;
#pragma unroll
  for (int c = 0; c < n; c++) {
    sg[(c * Q + s.i1) * QP + s.i2] = A[0][c];
    if (GRAD) {
      sg[((n + c) * Q + s.i1) * QP + s.i2] = A[1][c];
      sg[((2 * n + c) * Q + s.i1) * QP + s.i2] = A[2][c];
    }
  }
}

// Transposed xi2 contraction: thread (q1 = i1, b = i2) -> st[0][c][b][q1]
// (B in xi1) and st[1][c][b][q1] (D in xi1), rows of QP.
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void stage2t(const T *sB, const T *sD, const T *sg, T *st,
                                        const Slab &s) {
  constexpr int n = K::n, Q = K::Dm::Q, QP = K::Dm::QP;
  if (s.i2 < n) {
    T cb[Q], cd[Q];
    lds_row<Q>(sB + s.i2 * QP, cb);
    if (GRAD) lds_row<Q>(sD + s.i2 * QP, cd);
#pragma unroll
    for (int c = 0; c < n; c++) {
      T g0[Q], g1[Q], g2[Q];
      lds_row<Q>(sg + (c * Q + s.i1) * QP, g0);
      if (GRAD) {
        lds_row<Q>(sg + ((n + c) * Q + s.i1) * QP, g1);
        lds_row<Q>(sg + ((2 * n + c) * Q + s.i1) * QP, g2);
      }
      T hb = T(0), hd = T(0);
#pragma unroll
      for (int q = 0; q < Q; q++) {
        hb += cb[q] * g0[q];
        if (GRAD) {
          hb += cd[q] * g1[q];
          hd += cb[q] * g2[q];
        }
      }
      st[(c * n + s.i2) * QP + s.i1] = hb;
      if (GRAD) st[((n + c) * n + s.i2) * QP + s.i1] = hd;
    }
  }
}

// Transposed xi1 contraction of component comp, thread (a = i1, b = i2),
// into the block's output tile.  Slots a < P of the element are its own in
// the tile (plain stores, no zeroing needed); slot a = P is slot 0 of the
// next element of the run, kept in face[row][le] for add_faces.  (Adding
// every slot with LDS atomics into a zeroed tile was 15-39 % slower.)
template <class K, typename T, bool GRAD>
__device__ __forceinline__ void stage1t_tile(const Slab &s, int comp, const T *sB, const T *sD,
                                             const T *st, T *tile, T *face) {
  constexpr int n = K::n, Q = K::Dm::Q, P = K::Dm::P, TX = K::TX, QP = K::Dm::QP;
  if (s.valid && s.i1 < n && s.i2 < n) {
    T cb[Q], cd[Q];
    lds_row<Q>(sB + s.i1 * QP, cb);
    if (GRAD) lds_row<Q>(sD + s.i1 * QP, cd);
    T *row = tile + ((comp * n) * n + s.i2) * TX + s.le * P + s.i1;
#pragma unroll
    for (int c = 0; c < n; c++) {
      T h0[Q], h1[Q];
      lds_row<Q>(st + (c * n + s.i2) * QP, h0);
      if (GRAD) lds_row<Q>(st + ((n + c) * n + s.i2) * QP, h1);
      T val = T(0);
#pragma unroll
      for (int q = 0; q < Q; q++) {
        val += cb[q] * h0[q];
        if (GRAD) val += cd[q] * h1[q];
      }
      if (s.i1 < P)
        row[c * n * TX] = val;
      else
        face[((comp * n + c) * n + s.i2) * K::NE + s.le] = val;
    }
  }
}

// The x-face slots of the tile: slot (le + 1) P of row r is the next
// element's slot 0 (stored by it) plus element le's slot P; past the run's
// last element (or before an idle one) element le's value alone.  Elements
// past the mesh contribute nothing.
template <class K, typename T>
__device__ __forceinline__ void add_faces(const MeshK<T> &m, const Slab &s, T *tile,
                                          const T *face) {
  constexpr int n = K::n, P = K::Dm::P, NE = K::NE, TX = K::TX;
  const int ex0 = s.x0 / P;
  for (int k = threadIdx.x; k < 3 * n * n * NE; k += K::NT) {
    const int le = k % NE, r = k / NE;  // r = (comp n + c) n + b, the tile row
    if (ex0 + le >= m.nx) continue;
    T *dst = tile + r * TX + (le + 1) * P;
    const T f = face[k];
    if (le + 1 < NE && ex0 + le + 1 < m.nx)
      *dst += f;
    else
      *dst = f;
  }
}

// Add the block's output tile to y with hardware FP atomics (slots on the
// tile's faces are shared with neighbouring blocks; interior slots are not,
// but one uniform atomic loop is faster than separate store and atomic
// loops).  Constrained DOFs are skipped when mask is set.  RED adds
// vdot . tile.
template <class K, typename T, bool RED>
__device__ __forceinline__ void tile_writeback(const MeshK<T> &m, const Slab &s,
                                               const int64_t *s_row, const T *tile,
                                               T *__restrict__ y, bool mask,
                                               const T *__restrict__ vdot, double &dot) {
  const int xe = m.Nx - s.x0;
  const bool chk = mask && s.bnd;
  if (m.stage) {
    // deterministic assembly: the tile is staged, a gather kernel adds it
    T *__restrict__ out = m.stage + (size_t)blockIdx.x * K::TILE;
    tile_for<K>([&](int idx, int r, int x) {
      out[idx] = tile[idx];
      if (RED && !(x >= xe || (chk && tile_constrained<K>(m, s, r, x))))
        dot += (double)vdot[s_row[r] + x] * (double)tile[idx];
    });
    return;
  }
  tile_for<K>([&](int idx, int r, int x) {
    if (x >= xe || (chk && tile_constrained<K>(m, s, r, x))) return;
    const int64_t gi = s_row[r] + x;
    const T val = tile[idx];
    atomicAdd(&y[gi], val);
    if (RED) dot += (double)vdot[gi] * (double)val;
  });
}

// Transposes of the xi2 and xi1 contractions for the three components into
// the block's tile (each element's own slots stored, the shared x-face slots
// completed by add_faces), then written back to y.  The flux write of component i+1 overlaps
// the xi1 stage of component i (sg and the st buffers alternate).  sD: the
// scaled transposed D tables, direction 0 then 1.
template <class K, typename T, bool GRAD, bool RED>
__device__ __forceinline__ void transpose_all(const MeshK<T> &m, const Slab &s,
                                              const T (&A)[3][3][K::n], const T *sB, const T *sD,
                                              T *sg, T *st, T *tile, T *face,
                                              const int64_t *s_row, T *__restrict__ y, bool mask,
                                              const T *__restrict__ vdot, double &dot) {
  constexpr int HB = (K::Dm::DBUF >= 2) ? K::Dm::SB1 : 0;
  write_g<K, T, GRAD>(A[0], sg, s);
  __syncthreads();  // also: the forward pass is done with the tile
#pragma unroll
  for (int i = 0; i < 3; i++) {
    T *sti = st + (i & 1) * HB;
    stage2t<K, T, GRAD>(sB, sD + K::DTS, sg, sti, s);
    elem_sync<K>();
    if (i < 2) write_g<K, T, GRAD>(A[i + 1], sg, s);
    stage1t_tile<K, T, GRAD>(s, i, sB, sD, sti, tile, face);
    if (i < 2) elem_sync<K>();
  }
  __syncthreads();  // every element's slots and faces are in LDS
  add_faces<K>(m, s, tile, face);
  __syncthreads();
  tile_writeback<K, T, RED>(m, s, s_row, tile, y, mask, vdot, dot);
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

// Block sum of v (all threads call) stored by thread 0 as the block's
// partial (partials[2 b], partials[2 b + 1] = 0), summed in block order by a
// one-block kernel launched after the element kernel.
template <int NT>
__device__ __forceinline__ void block_partial_t(double v, Reduce red, double *s_red) {
  double t = block_sum<NT>(v, s_red);
  if (threadIdx.x == 0) {
    red.partials[2 * blockIdx.x] = t;
    red.partials[2 * blockIdx.x + 1] = 0.0;
  }
}

// Common kernel prologue.  SDME_SETUP_A: slab coordinates and LDS pointers;
// the thread's basis-table entries are requested.  The kernel then requests
// its other inputs (SDME_REQUEST: the first field of the tile), so that all
// are in flight together.  SDME_SETUP_B: tile row offsets and tables stored
// to LDS (waits only for the table requests, the first issued), barrier.
// SDME_STORE: the requested field stored to the tile, barrier.
#define SDME_SETUP_A                                                            \
  __shared__ __align__(16) T smem[K::SMEM];                                     \
  int64_t *s_row = (int64_t *)smem;                                             \
  T *tile = smem + K::RW + K::NE * K::SE, *s_face = tile + K::TILEP;            \
  T *s_tab = s_face + K::FACEP;                                                 \
  Slab s = make_slab<K>(m);                                                     \
  T s_tv[stage_table_nit<K>()];                                                 \
  request_stage_tables<K>(m, s_tv);                                             \
  T *su = smem + K::RW + s.le * K::SE, *st = su + K::SA;                        \
  const T *sB = s_tab + K::LB, *sD = s_tab + K::LD, *sW = s_tab + K::LW;       \
  const T *sBt = s_tab + K::LBT, *sDt = s_tab + K::LDT;
#define SDME_SETUP_B                                                            \
  tile_rows<K>(m, s, s_row);                                                    \
  store_stage_tables<K>(s_tv, s_tab);                                           \
  __syncthreads();
#define SDME_REQUEST(FIELD)                                                     \
  T s_gv[tile_nit<K>()];                                                        \
  tile_request<K>(m, s, FIELD, s_gv);
#define SDME_STORE(MASK)                                                        \
  tile_store<K>(m, s, s_gv, MASK, tile);                                        \
  __syncthreads();
#define SDME_PROLOGUE(FIELD, MASK) \
  SDME_SETUP_A SDME_REQUEST(FIELD) SDME_SETUP_B SDME_STORE(MASK)

// ===================================================================== force
// R(u) (and optionally the linearisation state of u).
template <int P, int Q, typename T, bool STORE, bool OUT>
__global__ __launch_bounds__((EK<P, Q, T>::NT)) void k_force(MeshK<T> m, const double *__restrict__ mu,
                                                           const double *__restrict__ lam,
                                                           const T *__restrict__ u, T *__restrict__ R,
                                                           T *__restrict__ state, int mask) {
  using K = EK<P, Q, T>;
  SDME_SETUP_A
  // material of the element (s.e is a valid index also for idle slabs),
  // requested with the gather and converted after the forward pass
  const double mud = mu[s.e], lad = lam[s.e];
  SDME_SETUP_B
  gather_tile<K>(m, s, s_row, u, false, tile);
  __syncthreads();
  T X[3][3][K::n];
  forward_lds<K, T, true>(sB, sD, tile, st, s, X);
  T mue = s.valid ? (T)mud : T(0), lae = s.valid ? (T)lad : T(0);
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ;
  T A[3][3][K::n];
  if (OUT) zero_acc<K>(A);
  bool bad = false;
  constexpr int QQQ = Q * Q * Q;
  T *__restrict__ sp = state + (size_t)(s.valid ? s.e : 0) * 10 * QQQ + s.t2;
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
#pragma unroll
      for (int k = 0; k < 9; k++) sp[k * QQQ + q3 * K::QQ] = kk.G[k];
      sp[9 * QQQ + q3 * K::QQ] = mue - lae * kk.lnJ;
    }
    if (OUT) {
      // P is linear in (mu, lam): the quadrature weight enters through them
      T f[9], mv[3] = {T(0), T(0), T(0)};
      const T wq = ok ? w12 * sW[q3] : T(0);
      first_pk(H, kk, wq * mue, wq * lae, f);
      accum_at<K, T, true, false>(s_tab, q3, f, mv, A);
    }
  }
  if (bad && s.valid) {
    atomicOr(m.flag, 1);
    atomicMin(m.flag + 1, s.e);
  }
  if (OUT) {
    double dummy = 0;
    transpose_all<K, T, true, false>(m, s, A, sBt, sDt, su, st, tile, s_face, s_row, R, mask != 0, (const T *)nullptr,
                                     dummy);
  }
}

// ============================================================ tangent action
// y = (K_T + s M) v with K_T from the stored state (REC = false; the state
// of the next Gauss-point slabs is in flight while the current one is
// processed) or from u_lin recomputed at every Gauss point (REC = true).
template <int P, int Q, typename T, bool REC, bool MASS, bool PU>
__global__ __launch_bounds__((EK<P, Q, T>::NT)) void k_tangent(
    MeshK<T> m, const double *__restrict__ mu, const double *__restrict__ lam,
    const T *__restrict__ ulin, const T *__restrict__ state, T mshift_rho, const T *__restrict__ v,
    T *__restrict__ y, int mask, PUpd<T> pu, const int *__restrict__ skip) {
  using K = EK<P, Q, T>;
  if (skip && *skip) return;
  const T beta = PU ? (T)*pu.beta : T(0);
  SDME_SETUP_A
  constexpr int QQQ = Q * Q * Q;
  constexpr bool PIPE = !REC && K::PIPE;
  const T *__restrict__ sp = state + (size_t)(s.valid ? s.e : 0) * 10 * QQQ + s.t2;
  // one-slab prefetch: the first slab is requested before the gather
  T Gn[10];
  if (!REC && !PIPE) {
#pragma unroll
    for (int k = 0; k < 10; k++) Gn[k] = sp[k * QQQ];
  }
  // material of the element (s.e is a valid index also for idle slabs),
  // requested with the gather and converted after the forward pass
  const double mud = mu[s.e], lad = lam[s.e];
  if constexpr (PU) {
    PuReq<K, T> q;
    tile_request_pu<K>(m, s, pu, v, q);
    SDME_SETUP_B
    tile_store_pu<K>(m, s, s_row, pu, q, beta, mask != 0, tile);
    __syncthreads();
  } else {
    SDME_REQUEST((REC ? ulin : v))
    SDME_SETUP_B
    SDME_STORE((REC ? false : mask != 0))
  }
  T XU[3][3][K::n];
  if (REC) {
    forward_lds<K, T, true>(sB, sD, tile, st, s, XU);
    __syncthreads();  // the tile is refilled with v below
    gather_tile<K>(m, s, s_row, v, mask != 0, tile);
    __syncthreads();
  }
  // named buffers: the first DEPTH slabs are requested once the gather has
  // completed (memory waits are in order, so earlier requests would be
  // waited for by the gather) and stay in flight through the forward
  // contractions, which wait only on LDS; the empty asm keeps the compiler
  // from moving the loads down to their first use.
  constexpr int DEPTH = K::DEPTH;
  T Ga[10], Gc[10], Gb[10];
  if (PIPE) {
#pragma unroll
    for (int k = 0; k < 10; k++) Ga[k] = sp[k * QQQ];
    __builtin_amdgcn_sched_barrier(0);
    const int o1 = min(1, Q - 1) * K::QQ;
#pragma unroll
    for (int k = 0; k < 10; k++) Gc[k] = sp[k * QQQ + o1];
    if constexpr (DEPTH == 3) {
      __builtin_amdgcn_sched_barrier(0);
      const int o2 = min(2, Q - 1) * K::QQ;
#pragma unroll
      for (int k = 0; k < 10; k++) Gb[k] = sp[k * QQQ + o2];
    }
    asm volatile("" ::: "memory");
  }
  T X[3][3][K::n];
  forward_lds<K, T, true>(sB, sD, tile, st, s, X);
  const T mue = s.valid ? (T)mud : T(0), lae = s.valid ? (T)lad : T(0);
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ;
  T A[3][3][K::n];
  zero_acc<K>(A);
  // linearised stress at Gauss point (i1, i2, q3) from G = F^-1, c1 (the
  // quadrature weight enters through the coefficients, dP being linear in
  // mu, c1 and lam):
  // dP = mu dF + c1 (G dF G)^T + lam tr(G dF) G^T, one row at a time,
  // accumulated at once into the transposed xi3 contraction (few live
  // temporaries)
  // With the fused direction update the FP64 kernel also forms p^T A p as
  // the sum of the element energies sum_q grad p : flux (+ s rho w detJ |p|^2):
  // p is zero on constrained DOFs, so this equals p^T (A p) of the masked
  // operator and replaces a streaming dot over p and A p (measured -2.5 % per
  // FP64 PCG iteration; in FP32 the extra work in the operator cost more than
  // the 0.03 ms dot it saves, +0.5 %).
  constexpr bool FUSED_PAP = SDME_FUSED_PAP && sizeof(T) == 8;
  T energy = T(0);
  auto point = [&](int q3, const T *G, T c1) {
    T dF[9];
    grad_at<K, T>(m, s_tab, q3, X, dF);
    T val[3];
    if (MASS) value_at<K, T>(s_tab, q3, X, val);
    T Am[9];
#pragma unroll
    for (int I = 0; I < 3; I++)
#pragma unroll
      for (int L = 0; L < 3; L++)
        Am[I * 3 + L] = G[I * 3 + 0] * dF[0 * 3 + L] + G[I * 3 + 1] * dF[1 * 3 + L] +
                        G[I * 3 + 2] * dF[2 * 3 + L];
    const T wq = w12 * sW[q3];
    const T wmu = wq * mue, wc1 = wq * c1;
    const T trl = (wq * lae) * (Am[0] + Am[4] + Am[8]);
    T bq[K::n], dq[K::n];
    lds_row<K::n>(sB + q3 * K::NP, bq);
    lds_row<K::n>(sD + 2 * K::DS + q3 * K::NP, dq);
#pragma unroll
    for (int i = 0; i < 3; i++) {
      T fr[3];
#pragma unroll
      for (int J = 0; J < 3; J++) {
        T AG = Am[J * 3 + 0] * G[0 * 3 + i] + Am[J * 3 + 1] * G[1 * 3 + i] +
               Am[J * 3 + 2] * G[2 * 3 + i];
        fr[J] = wmu * dF[i * 3 + J] + wc1 * AG + trl * G[J * 3 + i];
      }
      const T mv = MASS ? mshift_rho * wq * val[i] : T(0);
      if constexpr (PU && FUSED_PAP) {
        T ei = dF[i * 3 + 0] * fr[0] + dF[i * 3 + 1] * fr[1] + dF[i * 3 + 2] * fr[2];
        if (MASS) ei += val[i] * mv;
        energy += ei;
      }
#pragma unroll
      for (int c = 0; c < K::n; c++) {
        A[i][2][c] += bq[c] * fr[0];
        A[i][1][c] += bq[c] * fr[1];
        A[i][0][c] += dq[c] * fr[2];
        if (MASS) A[i][0][c] += bq[c] * mv;
      }
    }
  };
  bool bad = false;
  if (REC) {
#pragma unroll 1
    for (int q3 = 0; q3 < Q; q3++) {
      T H[9];
      grad_at<K, T>(m, s_tab, q3, XU, H);
      Kin<T> kk;
      if (!kinematics(H, kk)) {
        bad = true;
        kk.lnJ = T(0);
#pragma unroll
        for (int i = 0; i < 9; i++) kk.G[i] = T(0);
      }
      point(q3, kk.G, mue - lae * kk.lnJ);
    }
  } else if (PIPE) {
    // Gauss-point slabs in groups of DEPTH with the named buffers (no
    // register rotation): slab q3 + DEPTH is requested into a buffer as soon
    // as slab q3 has used it, and each wait leaves the other buffers'
    // requests outstanding.  Requests past the column repeat its last slab
    // (min(., Q - 1)) so that every request is unconditional; the scheduling
    // barriers keep each request after the computation that frees its buffer.
#pragma unroll 1
    for (int q3 = 0; q3 < Q; q3 += DEPTH) {
      point(q3, Ga, Ga[9]);
      __builtin_amdgcn_sched_barrier(0);
      const int oa = min(q3 + DEPTH, Q - 1) * K::QQ;
#pragma unroll
      for (int k = 0; k < 10; k++) Ga[k] = sp[k * QQQ + oa];
      if (Q % DEPTH == 0 || q3 + 1 < Q) {
        point(q3 + 1, Gc, Gc[9]);
        __builtin_amdgcn_sched_barrier(0);
        const int oc = min(q3 + 1 + DEPTH, Q - 1) * K::QQ;
#pragma unroll
        for (int k = 0; k < 10; k++) Gc[k] = sp[k * QQQ + oc];
      }
      if constexpr (DEPTH == 3) {
        if (Q % 3 == 0 || q3 + 2 < Q) {
          point(q3 + 2, Gb, Gb[9]);
          __builtin_amdgcn_sched_barrier(0);
          const int ob = min(q3 + 2 + DEPTH, Q - 1) * K::QQ;
#pragma unroll
          for (int k = 0; k < 10; k++) Gb[k] = sp[k * QQQ + ob];
        }
      }
    }
  } else {
    // one slab prefetched while the current one is processed
#pragma unroll 1
    for (int q3 = 0; q3 < Q; q3++) {
      T G[10];
#pragma unroll
      for (int k = 0; k < 10; k++) G[k] = Gn[k];
      if (q3 + 1 < Q) {
#pragma unroll
        for (int k = 0; k < 10; k++) Gn[k] = sp[k * QQQ + (q3 + 1) * K::QQ];
      }
      point(q3, G, G[9]);
    }
  }
  if (REC && bad && s.valid) {
    atomicOr(m.flag, 1);
    atomicMin(m.flag + 1, s.e);
  }
  double dot = 0;
  transpose_all<K, T, true, false>(m, s, A, sBt, sDt, su, st, tile, s_face, s_row, y, mask != 0,
                                   (const T *)nullptr, dot);
  if constexpr (PU && FUSED_PAP) {
    __shared__ double s_red[(K::NT + 63) / 64];
    if (pu.pap)
      block_partial_t<K::NT>(s.valid ? (double)energy : 0.0, Reduce{pu.pap, nullptr, nullptr},
                             s_red);
  }
}

// ====================================================================== mass
// y = rho M v on affine hexahedra with one density: the element mass is
// rho detJ (Mq (x) Mq (x) Mq) with Mq[a][b] = sum_q w_q B[q][a] B[q][b] the 1D
// mass of the mesh's rule (the quadrature sum of rho N_a N_b over a
// tensor-product rule factors into these 1D sums), so the assembled mass is
// rho detJ times the Kronecker product of the assembled 1D masses: slot
// e P + l (0 <= l < P) of a direction takes sum_a Mq[l][a] v(e P + a) from
// element e and, at l = 0, also sum_a Mq[P][a] v((e - 1) P + a) from element
// e - 1.  A block owns the output box of KronDims and marches along z through
// its input planes: each plane is loaded once (x and y halos P, zero outside
// the mesh and, with mask, on constrained slots), filtered along x and y in
// LDS, and accumulated per z element in registers; every output slot is
// stored once (constrained ones as zero with mask).  RED also sums v . y over
// the block's unconstrained outputs into the block partial (v^T M v).
#ifndef SDME_KRON_XCD
#define SDME_KRON_XCD 1
#endif
template <int P, typename T, bool RED>
__global__ __launch_bounds__((KronDims<P, (int)sizeof(T)>::NT)) void k_mass(
    MeshK<T> m, T rs, const T *__restrict__ v, T *__restrict__ y, int mask, Reduce red,
    const int *__restrict__ skip, KronGrid g) {
  using D = KronDims<P, (int)sizeof(T)>;
  constexpr int n = D::n, NT = D::NT, EX = D::EX, TX = D::TX, RY = D::RY, GPE = D::GPE,
                IX = D::IX, IY = D::IY, IXP = D::IXP, TXP = D::TXP, NLD = D::NLD;
  constexpr int NXI = (EX * IY + NT - 1) / NT;  // x-pass items per thread
  constexpr bool MQR = D::MQR;
  if (skip && *skip) return;
  // input and x-filtered planes, two of each (plane z uses buffer z & 1)
  __shared__ __align__(16) T sIn[2][IY * IXP];
  __shared__ __align__(16) T sX[2][IY * TXP];
  __shared__ T sM[n * n];
  __shared__ double s_red[NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int b = blockIdx.x;
#if SDME_KRON_XCD
  {  // blocks b, b + 8, ... run on one XCD: give each XCD a contiguous range
    const int G = g.blocks(), per = G / 8, rem = G % 8, xcd = b % 8, k = b / 8;
    b = xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
  }
#endif
  const int xt = b % g.nxt;
  b /= g.nxt;
  const int yt = b % g.nyt;
  b /= g.nyt;
  const int zc = b % g.nzc, comp = b / g.nzc;
  const int ex0 = xt * D::EX, ey0 = yt * D::EY, ez_lo = zc * g.cz,
            ez_hi = min(m.nz, ez_lo + g.cz);
  const int x0 = ex0 * P, y0 = ey0 * P, Nx = m.Nx, Ny = m.Ny, Nz = m.Nz;
  const uint32_t mb = mask ? (m.bc >> comp) : 0u;
  if (tid < n * n) {
    const int Q = m.Q, a = tid / n, c = tid % n;
    const T *B = m.tab, *W = m.tab + 2 * Q * n;
    T acc = T(0);
    for (int q = 0; q < Q; q++) acc += W[q] * B[q * n + a] * B[q * n + c];
    sM[tid] = acc;
  }
  // the thread's input-plane slots: in-plane offset (-1: outside the mesh or
  // constrained on an x or y face with mask) and LDS position (-1: none)
  int off[NLD], lpos[NLD];
#pragma unroll
  for (int i = 0; i < NLD; i++) {
    const int idx = tid + i * NT, r = idx / IX, c = idx - r * IX;
    const int gx = x0 - P + c, gy = y0 - P + r;
    const bool ok = idx < IX * IY && gx >= 0 && gx < Nx && gy >= 0 && gy < Ny &&
                    !((mb & 1u) && gx == 0) && !((mb & 8u) && gx == Nx - 1) &&
                    !((mb & 64u) && gy == 0) && !((mb & 512u) && gy == Ny - 1);
    off[i] = ok ? gy * Nx + gx : -1;
    lpos[i] = idx < IX * IY ? r * IXP + c : -1;
  }
  // the thread's x-pass items (element je of the tile, row r): LDS offsets
  // of its input row segment and output, and what the element contributes
  // (bit 0: its own term, element < nx; bit 1: the vertex's element-(e - 1)
  // term, e > 0; none past the element index nx, which only owns the vertex)
  int xin[NXI], xout[NXI], xfl[NXI];
#pragma unroll
  for (int k = 0; k < NXI; k++) {
    // consecutive lanes take consecutive elements of a row (contiguous LDS
    // segments)
    const int it = tid + k * NT, r = it / EX, je = it - r * EX, e = ex0 + je;
    const bool act = it < EX * IY && e <= m.nx;
    xin[k] = r * IXP + je * P;
    xout[k] = r * TXP + je * P;
    xfl[k] = act ? ((e < m.nx ? 1 : 0) | (e > 0 ? 2 : 0)) : 0;
  }
  const T *vp = v + (size_t)comp * m.Nn;
  const size_t plane_sz = (size_t)Nx * Ny;
  T pre[NLD];
  auto request = [&](int z) {
    const bool zok = !((mb & 4096u) && z == 0) && !((mb & 32768u) && z == Nz - 1);
    const T *pz = vp + (size_t)z * plane_sz;
#pragma unroll
    for (int i = 0; i < NLD; i++) pre[i] = (zok && off[i] >= 0) ? pz[off[i]] : T(0);
  };
  auto commit = [&](T *dst) {
#pragma unroll
    for (int i = 0; i < NLD; i++)
      if (lpos[i] >= 0) dst[lpos[i]] = pre[i];
  };
  __syncthreads();  // sM
  T mq[MQR ? n * n : 1];
  if constexpr (MQR) {
#pragma unroll
    for (int i = 0; i < n * n; i++) mq[i] = sM[i];
  }
  auto M = [&](int l, int a) -> T {
    if constexpr (MQR)
      return mq[l * n + a];
    else
      return sM[l * n + a];
  };
  // x pass: the P slots of the item's element in its row (in[0..P]: element
  // e - 1, in[P..2P]: element e)
  auto xpass = [&](const T *src, T *dst) {
#pragma unroll
    for (int k = 0; k < NXI; k++) {
      const int fl = xfl[k];
      if (!fl) continue;
      const T *in = src + xin[k];
      T u[2 * P + 1];  // slots of element e - 1 (0 .. P) and e (P .. 2P)
      if constexpr (D::VEC) {
        constexpr int VW = D::VW;
        using V = T __attribute__((ext_vector_type(VW)));
#pragma unroll
        for (int q = 0; q < 2 * P / VW; q++) {
          const V t = *reinterpret_cast<const V *>(in + q * VW);
#pragma unroll
          for (int c = 0; c < VW; c++) u[q * VW + c] = t[c];
        }
        u[2 * P] = in[2 * P];
      } else {
#pragma unroll
        for (int a = 0; a <= 2 * P; a++) u[a] = in[a];
      }
      T o[P];
#pragma unroll
      for (int l = 0; l < P; l++) o[l] = T(0);
      if (fl & 1) {
#pragma unroll
        for (int a = 0; a < n; a++) {
#pragma unroll
          for (int l = 0; l < P; l++) o[l] += M(l, a) * u[P + a];
        }
      }
      if (fl & 2) {
#pragma unroll
        for (int a = 0; a < n; a++) o[0] += M(P, a) * u[a];
      }
      T *out = dst + xout[k];
      if constexpr (D::VEC) {
        // past the element index nx only slot 0 is written
        constexpr int VW = D::VW;
        using V = T __attribute__((ext_vector_type(VW)));
        if (fl & 1) {
#pragma unroll
          for (int q = 0; q < P / VW; q++) {
            V t;
#pragma unroll
            for (int c = 0; c < VW; c++) t[c] = o[q * VW + c];
            *reinterpret_cast<V *>(out + q * VW) = t;
          }
        } else {
          out[0] = o[0];
        }
      } else {
        out[0] = o[0];
        if (fl & 1) {
#pragma unroll
          for (int l = 1; l < P; l++) out[l] = o[l];
        }
      }
    }
  };
  // y pass: wave wv owns rows l0 .. l0 + RY - 1 of element ey, lane = x slot
  const int gq = wv / GPE, ey = ey0 + gq, l0 = (wv % GPE) * RY;
  const int gx = x0 + lane;
  const int xcl = min(lane, TX - 1);
  const bool xok = lane < TX && gx < Nx;
  auto ypass = [&](const T *src, T (&w)[RY]) {
    const T *col = src + (gq * P) * TXP + xcl;  // rows of element ey - 1, then ey
#pragma unroll
    for (int j = 0; j < RY; j++) w[j] = T(0);
    if (ey < m.ny) {
#pragma unroll
      for (int a = 0; a < n; a++) {
        const T u = col[(P + a) * TXP];
#pragma unroll
        for (int j = 0; j < RY; j++) w[j] += M(l0 + j, a) * u;
      }
    }
    if (l0 == 0 && ey > 0 && ey <= m.ny) {
#pragma unroll
      for (int a = 0; a < n; a++) w[0] += M(P, a) * col[a * TXP];
    }
  };
  double dot = 0;
  // the thread's output rows: in-plane offset (-1: no output) and whether
  // the slot is constrained on an x or y face (with mask)
  int orow[RY];
  unsigned ocon = 0;
#pragma unroll
  for (int j = 0; j < RY; j++) {
    const int gy = y0 + gq * P + l0 + j;
    const bool ok = xok && gy < Ny && ey <= m.ny;
    orow[j] = ok ? gy * Nx + gx : -1;
    if (((mb & 1u) && gx == 0) || ((mb & 8u) && gx == Nx - 1) || ((mb & 64u) && gy == 0) ||
        ((mb & 512u) && gy == Ny - 1))
      ocon |= 1u << j;
  }
  T *yc = y + (size_t)comp * m.Nn;
  // outputs of row j of this wave at plane zo (val = accumulated sum)
  auto emit = [&](int zo, int j, T val) {
    if (orow[j] < 0) return;
    const bool con = ((ocon >> j) & 1u) || ((mb & 4096u) && zo == 0) ||
                     ((mb & 32768u) && zo == Nz - 1);
    const size_t gi = (size_t)zo * plane_sz + orow[j];
    const T o = con ? T(0) : val * rs;
    // non-temporal stores in FP64 (4 % faster at 47^3, P = 4; 2 % slower in FP32)
    if constexpr (sizeof(T) == 8)
      __builtin_nontemporal_store(o, yc + gi);
    else
      yc[gi] = o;
    if (RED && !con) dot += (double)vp[gi] * (double)o;
  };
  // z march over the planes z0 .. zlast of elements e_start .. ez_hi - 1
  // (e_start = ez_lo - 1 supplies the contribution of element ez_lo - 1 to
  // the chunk's first vertex plane).  Plane z = e P + a adds Mq[l][a] w to
  // the accumulators of element e; at a vertex plane element e - 1 is
  // complete: its planes are stored and the vertex starts element e.
  // One barrier per plane: plane z + 1 is stored to the other LDS buffer
  // before it, plane z + 2 requested after it.
  const int e_start = ez_lo > 0 ? ez_lo - 1 : 0, z0 = e_start * P, zlast = ez_hi * P;
  T w[RY], acc[RY][n], carry[RY];
#pragma unroll
  for (int j = 0; j < RY; j++) {
    carry[j] = T(0);
#pragma unroll
    for (int l = 0; l < n; l++) acc[j][l] = T(0);
  }
  request(z0);
  commit(sIn[0]);
  if (z0 + 1 <= zlast) request(z0 + 1);
  __syncthreads();
  for (int z = z0; z <= zlast; z++) {
    const int bf = (z - z0) & 1;
    xpass(sIn[bf], sX[bf]);
    if (z + 1 <= zlast) commit(sIn[bf ^ 1]);
    __syncthreads();
    if (z + 2 <= zlast) request(z + 2);
    ypass(sX[bf], w);
    const int a = z % P;
    if (a != 0) {
#pragma unroll
      for (int j = 0; j < RY; j++) {
#pragma unroll
        for (int l = 0; l < n; l++) acc[j][l] += sM[l * n + a] * w[j];
      }
    } else {
      // vertex plane: completes element z / P - 1 (none at z0), starts z / P
      const int e = z / P - 1;
      if (z > z0) {
#pragma unroll
        for (int j = 0; j < RY; j++) {
#pragma unroll
          for (int l = 0; l < n; l++) acc[j][l] += M(l, P) * w[j];
        }
        if (e >= ez_lo) {
#pragma unroll
          for (int l = 0; l < P; l++) {
#pragma unroll
            for (int j = 0; j < RY; j++) emit(e * P + l, j, acc[j][l]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < RY; j++) {
        carry[j] = z > z0 ? acc[j][P] : T(0);
#pragma unroll
        for (int l = 0; l < n; l++) acc[j][l] = M(l, 0) * w[j];
        acc[j][0] += carry[j];
      }
    }
  }
  if (ez_hi == m.nz) {  // the final vertex plane: element nz - 1 only
#pragma unroll
    for (int j = 0; j < RY; j++) emit(Nz - 1, j, carry[j]);
  }
  if (RED) block_partial_t<NT>(dot, red, s_red);
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
          if (m.stage)  // deterministic assembly: element vector, gathered afterwards
            m.stage[((size_t)s.e * 3 + i) * K::n3 + (c * n + s.i2) * n + s.i1] = val;
          else if (!(mask && is_constrained(m.bc, i, ix, iy, iz, m.Nx, m.Ny, m.Nz)))
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
  __shared__ double s_red[(K::NT + 63) / 64];
  SDME_SETUP_A
  const double mud = mu[s.e], lad = lam[s.e];  // requested with the gather
  SDME_SETUP_B
  gather_tile<K>(m, s, s_row, u, false, tile);
  __syncthreads();
  T X[3][3][K::n];
  forward_lds<K, T, true>(sB, sD, tile, st, s, X);
  T mue = s.valid ? mud : 0.0, lae = s.valid ? lad : 0.0;
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
      acc += w12 * sW[q3] * psi;
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
  __shared__ double s_part[K::NE][2][K::QQ];
  SDME_PROLOGUE(u, false)
  T XU[3][3][K::n], XW[3][3][K::n];
  forward_lds<K, T, true>(sB, sD, tile, st, s, XU);
  __syncthreads();
  gather_tile<K>(m, s, s_row, wv, false, tile);
  __syncthreads();
  forward_lds<K, T, true>(sB, sD, tile, st, s, XW);
  T w12 = sW[s.i1] * sW[s.i2] * m.detJ;
  double am = 0, al = 0;
#pragma unroll 1
  for (int q3 = 0; q3 < Q; q3++) {
    T H[9], Gw[9];
    grad_at<K, T>(m, s_tab, q3, XU, H);
    grad_at<K, T>(m, s_tab, q3, XW, Gw);
    Kin<T> kk;
    if (kinematics(H, kk)) {
      T wq = w12 * sW[q3];
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
// Each wrapper dispatches on the volume rule of the mesh: Q = P + 2
// Gauss-Legendre points or Q = P + 1 Gauss-Lobatto-Legendre points.
template <int P, int Q, typename T>
int launch_force_q(const MeshK<T> &m, const double *mu, const double *lam, const T *u, T *R,
                          T *state, int mask, hipStream_t st) {
  using K = EK<P, Q, T>;
  dim3 grid(blocks_for<K>(m.nx, m.ny, m.nz)), block(K::NT);
  if (R && state)
    hipLaunchKernelGGL((k_force<P, Q, T, true, true>), grid, block, 0, st, m, mu, lam, u, R, state, mask);
  else if (R)
    hipLaunchKernelGGL((k_force<P, Q, T, false, true>), grid, block, 0, st, m, mu, lam, u, R, state, mask);
  else
    hipLaunchKernelGGL((k_force<P, Q, T, true, false>), grid, block, 0, st, m, mu, lam, u, R, state, mask);
  if (R && m.stage && launch_stage_gather<T>(P, m, K::NE, K::TX, K::TILE, mask, R, nullptr, st))
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template <int P, typename T>
int launch_force_t(const MeshK<T> &m, const double *mu, const double *lam, const T *u, T *R,
                          T *state, int mask, hipStream_t st) {
  return m.Q == P + 1 ? launch_force_q<P, P + 1, T>(m, mu, lam, u, R, state, mask, st)
                      : launch_force_q<P, P + 2, T>(m, mu, lam, u, R, state, mask, st);
}

template <int P, int Q, typename T>
int launch_tangent_q(const MeshK<T> &m, const double *mu, const double *lam, const T *ulin,
                     const T *state, T msr, const T *v, T *y, int mask, const PUpd<T> *pu,
                     const int *skip, hipStream_t st) {
  using K = EK<P, Q, T>;
  dim3 grid(blocks_for<K>(m.nx, m.ny, m.nz)), block(K::NT);
  const bool mass = msr != T(0);
  const PUpd<T> none{nullptr, nullptr, nullptr, nullptr, nullptr};
  const PUpd<T> &u = pu ? *pu : none;
#define SDME_TAN(REC, MASS, PU)                                                                 \
  hipLaunchKernelGGL((k_tangent<P, Q, T, REC, MASS, PU>), grid, block, 0, st, m, mu, lam, ulin, \
                     state, msr, v, y, mask, u, skip)
  if (ulin) {
    if (pu) return -2;  // the fused update is provided for the stored-state operator
    if (mass) SDME_TAN(true, true, false); else SDME_TAN(true, false, false);
  } else if (pu) {
    if (mass) SDME_TAN(false, true, true); else SDME_TAN(false, false, true);
  } else {
    if (mass) SDME_TAN(false, true, false); else SDME_TAN(false, false, false);
  }
#undef SDME_TAN
  if (m.stage && launch_stage_gather<T>(P, m, K::NE, K::TX, K::TILE, mask, y, skip, st)) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template <int P, typename T>
int launch_tangent_t(const MeshK<T> &m, const double *mu, const double *lam, const T *ulin,
                     const T *state, T msr, const T *v, T *y, int mask, const PUpd<T> *pu,
                     const int *skip, hipStream_t st) {
  return m.Q == P + 1 ? launch_tangent_q<P, P + 1, T>(m, mu, lam, ulin, state, msr, v, y, mask, pu, skip, st)
                      : launch_tangent_q<P, P + 2, T>(m, mu, lam, ulin, state, msr, v, y, mask, pu, skip, st);
}

// Mass-kernel grid: z chunks sized so that the grid fits in the blocks the
// device holds at once (occupancy x compute units, queried once per
// instantiation on the current device).
// (The capacity is taken on the device current at the first launch and kept
// for the process: the library runs on one GPU model.)
template <int P, typename T>
KronGrid mass_grid_t(const MeshK<T> &m) {
  static const int cap = [] {
    int nb = 0, cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mass<P, T, false>,
                                                     KronDims<P, (int)sizeof(T)>::NT, 0) !=
            hipSuccess)
      return 1024;
    return nb * cus > 0 ? nb * cus : 1024;
  }();
  return kron_grid<KronDims<P, (int)sizeof(T)>>(m.nx, m.ny, m.nz, cap);
}
template <int P, typename T>
int mass_blocks_t(const MeshK<T> &m) {
  return mass_grid_t<P, T>(m).blocks();
}

template <int P, typename T>
int launch_mass_t(const MeshK<T> &m, T rho, const T *v, T *y, int mask, Reduce red, int do_red,
                  const int *skip, hipStream_t st) {
  using D = KronDims<P, (int)sizeof(T)>;
  const KronGrid g = mass_grid_t<P, T>(m);
  const T rs = rho * m.detJ;
  if (do_red)
    hipLaunchKernelGGL((k_mass<P, T, true>), dim3(g.blocks()), dim3(D::NT), 0, st, m, rs, v, y,
                       mask, red, skip, g);
  else
    hipLaunchKernelGGL((k_mass<P, T, false>), dim3(g.blocks()), dim3(D::NT), 0, st, m, rs, v, y,
                       mask, red, skip, g);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int P, int Q, typename T>
int launch_diag_q(const MeshK<T> &m, const double *mu, const double *lam, const T *state,
                         T msr, T *d, int mask, hipStream_t st) {
  using K = EK<P, Q, T>;
  static_assert(3 * K::n * K::n * Q <= K::SE, "diag LDS layout");
  dim3 grid(blocks_for<K>(m.nx, m.ny, m.nz)), block(K::NT);
  hipLaunchKernelGGL((k_diag<P, Q, T>), grid, block, 0, st, m, mu, lam, state, msr, d, mask);
  if (m.stage && launch_stage_gather_elem<T>(P, m, mask, d, st)) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template <int P, typename T>
int launch_diag_t(const MeshK<T> &m, const double *mu, const double *lam, const T *state,
                         T msr, T *d, int mask, hipStream_t st) {
  return m.Q == P + 1 ? launch_diag_q<P, P + 1, T>(m, mu, lam, state, msr, d, mask, st)
                      : launch_diag_q<P, P + 2, T>(m, mu, lam, state, msr, d, mask, st);
}

template <int P, int Q>
int launch_energy_q(const MeshK<double> &m, const double *mu, const double *lam,
                           const double *u, Reduce red, hipStream_t st) {
  using K = EK<P, Q, double>;
  dim3 grid(blocks_for<K>(m.nx, m.ny, m.nz)), block(K::NT);
  hipLaunchKernelGGL((k_energy<P, Q>), grid, block, 0, st, m, mu, lam, u, red);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template <int P>
int launch_energy_t(const MeshK<double> &m, const double *mu, const double *lam,
                           const double *u, Reduce red, hipStream_t st) {
  return m.Q == P + 1 ? launch_energy_q<P, P + 1>(m, mu, lam, u, red, st)
                      : launch_energy_q<P, P + 2>(m, mu, lam, u, red, st);
}

template <int P, int Q>
int launch_matgrad_q(const MeshK<double> &m, const double *u, const double *w, double scale,
                            double *gm, double *gl, hipStream_t st) {
  using K = EK<P, Q, double>;
  dim3 grid(blocks_for<K>(m.nx, m.ny, m.nz)), block(K::NT);
  hipLaunchKernelGGL((k_matgrad<P, Q>), grid, block, 0, st, m, u, w, scale, gm, gl);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template <int P>
int launch_matgrad_t(const MeshK<double> &m, const double *u, const double *w, double scale,
                            double *gm, double *gl, hipStream_t st) {
  return m.Q == P + 1 ? launch_matgrad_q<P, P + 1>(m, u, w, scale, gm, gl, st)
                      : launch_matgrad_q<P, P + 2>(m, u, w, scale, gm, gl, st);
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
                                              double *, int, const PUpd<double> *, const int *,
                                              hipStream_t);
template int launch_tangent_t<SDME_P, float>(const MeshK<float> &, const double *, const double *,
                                             const float *, const float *, float, const float *,
                                             float *, int, const PUpd<float> *, const int *,
                                             hipStream_t);
template int mass_blocks_t<SDME_P, double>(const MeshK<double> &);
template int mass_blocks_t<SDME_P, float>(const MeshK<float> &);
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
