// C-ABI entry points of libsdme: context, operators and the solver/driver
// loops (host side; every arithmetic step runs in the kernels of
// elem_kernels.hip and vec_kernels.hip).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "sdme.h"
#include "sdme_internal.h"
#include "sdme_launch.h"

using namespace sdme;

#ifndef SDME_FUSED_PAP
#define SDME_FUSED_PAP 1
#endif

// Offsets of the parts of the context's device block, and its size.
struct BlockPlan {
  size_t o_tm64 = 0, o_tm32 = 0, o_t64 = 0, o_t32 = 0, o_flag = 0, o_pcg = 0, o_part = 0,
         o_cnt = 0, o_res = 0, o_stage = 0, stage_bytes = 0, dev_bytes = 0, host_bytes = 0;
};
// Host block: PcgDev[2] at 0, double[16] at 1024, int at 2048.
constexpr size_t HOST_BLOCK_BYTES = 4096;

struct sdme_ctx {
  sdme_mesh_desc d;
  int P, Q, n;
  int64_t Nn, E, nqp;
  Basis basis;
  void *dev_block = nullptr;
  double *tab64 = nullptr;
  float *tab32 = nullptr;
  int *flag = nullptr;
  PcgDev *pcg = nullptr;  // [2]: outer/FP64 and inner/FP32
  double *partials = nullptr;
  unsigned *counter = nullptr;
  double *results = nullptr;  // [16]
  void *host_block = nullptr;
  BlockPlan plan;
  PcgDev *h_pcg = nullptr;
  double *h_res = nullptr;
  int *h_flag = nullptr;
  int64_t jac_element = -1;  // from the last read of the status words
  MeshK<double> m64;
  MeshK<float> m32;
  // the meshes of the mass operator: the same as m64, m32, or (mass_rule 1)
  // with the Gauss-Lobatto-Legendre rule of P+1 points and its own tables
  MeshK<double> mm64;
  MeshK<float> mm32;
  double *tabm64 = nullptr;
  float *tabm32 = nullptr;
  std::vector<double> tabm_host;
  bool dev_ready = false;
  // optional per-launch timing of the PCG operator (HIP events on the solve
  // stream): [0] FP64 operator, [1] FP32 operator
  bool prof = false;
  std::vector<hipEvent_t> ev;
  double prof_ms[2] = {0, 0};
  int64_t prof_count[2] = {0, 0};
  std::vector<double> tab_host;
  std::vector<float> tab32_host, tabm32_host;
};

namespace {

constexpr int CHUNK = 16;  // PCG iterations enqueued between convergence reads

inline hipStream_t S(void *s) { return (hipStream_t)s; }

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

Reduce red_at(sdme_ctx *c, int slot) { return Reduce{c->partials, c->counter, c->results + slot}; }

// roctx range around a driver phase (Newton iteration, time step, linear
// solve): host-side markers that rocprofv3 --marker-trace records beside the
// kernels; without a profiler attached the calls return at once.
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};

template <typename T>
const MeshK<T> &mk(const sdme_ctx *c);
template <typename T>
const MeshK<T> &mkm(const sdme_ctx *c);
template <>
const MeshK<double> &mkm<double>(const sdme_ctx *c) { return c->mm64; }
template <>
const MeshK<float> &mkm<float>(const sdme_ctx *c) { return c->mm32; }
template <>
const MeshK<double> &mk<double>(const sdme_ctx *c) { return c->m64; }
template <>
const MeshK<float> &mk<float>(const sdme_ctx *c) { return c->m32; }

// bump allocator over the caller's workspace
struct Bump {
  char *base;
  size_t cap, off = 0;
  bool ok = true;
  Bump(void *b, size_t c) : base((char *)b), cap(c) {}
  template <typename T>
  T *get(int64_t count) {
    size_t bytes = ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
    if (!base || off + bytes > cap) {
      ok = false;
      off += bytes;
      return nullptr;
    }
    T *p = (T *)(base + off);
    off += bytes;
    return p;
  }
};

int dev_err(hipError_t e) { return e == hipSuccess ? SDME_OK : SDME_EDEVICE; }
int lerr(int r) { return r == 0 ? SDME_OK : (r == -2 ? SDME_EINVAL : SDME_EDEVICE); }

bool valid_prec(int p) { return p == SDME_FP64 || p == SDME_FP32; }

// Status words on the device: flag[0] = 1 once det F <= 0 was met at a
// Gauss point, flag[1] = the smallest index of an element where it was
// (INT_MAX: none).  read_flag keeps that element for sdme_jac_element.
int read_flag(sdme_ctx *c, hipStream_t st) {
  if (hipMemcpyAsync(c->h_flag, c->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return SDME_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return SDME_EDEVICE;
  c->jac_element = (c->h_flag[0] && c->h_flag[1] != INT_MAX) ? c->h_flag[1] : -1;
  return c->h_flag[0] ? SDME_EJAC : SDME_OK;
}

int clear_flag(sdme_ctx *c, hipStream_t st) {
  return lerr(launch_fill<int>(c->flag, 0, 1, st) || launch_fill<int>(c->flag + 1, INT_MAX, 1, st)
                  ? -1
                  : 0);
}

// ||x||^2 and x.y in double (synchronises); returns via out[0] = x.y, out[1] = y.y
template <typename T>
int dot2(sdme_ctx *c, const T *x, const T *y, int64_t n, double out[2], hipStream_t st) {
  if (launch_dot2<T>(x, y, n, red_at(c, 0), st)) return SDME_EDEVICE;
  if (hipMemcpyAsync(c->h_res, c->results, 2 * sizeof(double), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return SDME_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return SDME_EDEVICE;
  out[0] = c->h_res[0];
  out[1] = c->h_res[1];
  return SDME_OK;
}

// Operator descriptor for the PCG: tangent from stored state (kind 0), tangent
// recomputed from u_lin (kind 1) or mass (kind 2).
template <typename T>
struct Op {
  int kind;
  const T *state;
  const T *ulin;
  T msr;  // mass_shift * rho
  T rho;
  // kind 3 (condensed system, FP64): the operator whose interior modes are
  // condensed (0 tangent, 2 mass), the inverted interior blocks and two
  // scratch vectors
  int inner = 0;
  const double *Kinv = nullptr;
  double *t = nullptr, *z = nullptr;
};

template <typename T>
int apply_op(sdme_ctx *c, const sdme_material *mat, const Op<T> &op, const T *v, T *y, Reduce red,
             int do_red, const int *skip, hipStream_t st, const PUpd<T> *pu = nullptr) {
  if (op.kind == 3) {
    // Schur complement of the interior modes applied to v (zero on every
    // interior slot): t = A v; z = v with z_I = -inv(A_II) t_I (the interior
    // response, Eq. Schur_split2); y = A z, restricted to the other slots
    // (Eq. Schur_split1)
    if constexpr (sizeof(T) == 8) {
      const int64_t N = 3 * c->Nn;
      Op<T> in = op;
      in.kind = op.inner;
      if (launch_fill<double>(op.t, 0.0, N, st) ||
          apply_op<T>(c, mat, in, v, op.t, red, 0, skip, st) ||
          launch_convert<double, double>(op.z, v, 1.0, N, st) ||
          launch_interior_apply(c->P, c->m64, op.Kinv, op.t, op.z, -1.0, skip, st) ||
          apply_op<T>(c, mat, in, op.z, y, red, 0, skip, st) ||
          launch_interior_set(c->P, c->m64, y, 0.0, skip, st))
        return -1;
      return 0;
    }
    return -2;
  }
  if (op.kind == 2) return launch_mass<T>(c->P, mkm<T>(c), op.rho, v, y, 1, red, do_red, skip, st);
  if (do_red) return -2;
  return launch_tangent<T>(c->P, mk<T>(c), mat->mu, mat->lam, op.kind == 1 ? op.ulin : nullptr,
                           op.kind == 0 ? op.state : nullptr, op.msr, v, y, 1, pu, skip, st);
}

// Residual replacement ("reliable updates") of the mixed-precision CG: the
// FP32 iteration keeps its search direction while the solution is accumulated
// in FP64 and the FP32 residual is periodically replaced by the true FP64
// residual b - A64 x64 (defect correction inside one Krylov sequence).
struct Replace {
  const Op<double> *op64;
  double *x64, *r64, *Ap64;
  const double *bm;
  double delta;
  int count;
};

int do_replace(sdme_ctx *c, const sdme_material *mat, Replace &rep, float *x32, float *r32,
               const float *d32, float *p32, PcgDev *s, bool update_p, hipStream_t st) {
  int64_t N = 3 * c->Nn;
  if (launch_add_scaled_f(rep.x64, x32, 1.0, N, st) || launch_fill<float>(x32, 0.0f, N, st) ||
      launch_fill<double>(rep.Ap64, 0.0, N, st))
    return SDME_EDEVICE;
  Reduce none{c->partials, c->counter, c->results + 8};
  if (apply_op<double>(c, mat, *rep.op64, rep.x64, rep.Ap64, none, 0, nullptr, st) ||
      launch_axpbypcz(rep.r64, 1.0, rep.bm, 0.0, -1.0, rep.Ap64, N, st) ||
      launch_pcg_replace(r32, rep.r64, d32, p32, s, rep.delta, N, red_at(c, 2), update_p, st))
    return SDME_EDEVICE;
  rep.count++;
  return SDME_OK;
}

// Jacobi PCG in precision T on vectors of type T: b masked on input, x out.
// The operator's p^T A p comes from a separate streaming dot product.  With
// a second direction buffer p2 and the stored-state operator, the update
// p = z + beta p is fused into the operator's gather (p and p2 alternate),
// and x is updated every other iteration with both directions.
template <typename T>
int pcg_core(sdme_ctx *c, const sdme_material *mat, const Op<T> &op, const T *b, T *x, const T *d,
             double rtol, int maxit, T *r, T *p, T *Ap, int slot, int *iters, double *rel,
             hipStream_t st, Replace *rep = nullptr, T *p2 = nullptr) {
  int64_t N = 3 * c->Nn;
  PcgDev *s = c->pcg + slot;
  if (launch_fill<T>(x, T(0), N, st) || launch_fill<T>(Ap, T(0), N, st) ||
      launch_convert<T, T>(r, b, 1.0, N, st))
    return SDME_EDEVICE;
  if (launch_pcg_init<T>(r, d, p, s, rtol, maxit, rep ? rep->delta : 0.0, N, red_at(c, 2), st))
    return SDME_EDEVICE;
  Reduce none{c->partials, c->counter, c->results + 8};
  const bool fused = p2 != nullptr && op.kind == 0;
  // p^T A p formed by the FP64 fused operator (element energies)
  const bool fused_pap = fused && SDME_FUSED_PAP && sizeof(T) == 8;
  const int op_blocks =
      elem_blocks(c->P, mk<T>(c).Q, (int)sizeof(T), c->d.nx, c->d.ny, c->d.nz, true);
  T *pb[2] = {p, p2};
  int par = 0;  // pb[par] holds the current search direction
  for (;;) {
    if (hipMemcpyAsync(c->h_pcg + slot, s, sizeof(PcgDev), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SDME_EDEVICE;
    int done = c->h_pcg[slot].done;
    // launched iterations past a stop return at once, so the direction
    // buffers alternate with the iterations that ran
    if (fused) par = c->h_pcg[slot].iters & 1;
    // complete a deferred x update (pb[par] is the last direction) before a
    // residual replacement reads x, at the end, and at every chunk boundary
    if (c->h_pcg[slot].xpend && launch_pcg_xflush<T>(x, pb[par], s, N, st))
      return SDME_EDEVICE;
    if constexpr (sizeof(T) == 4) {
      if (rep && (done == 5 || done == 1)) {
        // the FP32 residual met the replacement or the stop threshold: replace
        // it by the FP64 defect; stop only if that defect meets the tolerance
        if (rep->count >= 1000) return SDME_ENOCONV;
        int rc = do_replace(c, mat, *rep, x, r, d, pb[par], s, !fused, st);
        if (rc) return rc;
        if (hipMemcpyAsync(c->h_pcg + slot, s, sizeof(PcgDev), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return SDME_EDEVICE;
        done = c->h_pcg[slot].done;  // 1: FP64 defect converged, 3: non-finite, 0: go on
      }
    }
    if (done) break;
    int it0 = c->h_pcg[slot].iters;
    for (int j = 0; j < CHUNK; j++) {
      if (c->prof && hipEventRecord(c->ev[2 * j], st) != hipSuccess) return SDME_EDEVICE;
      T *pc = pb[par];
      if (fused) {
        // p_new = z + beta p_old formed in the operator's gather
        PUpd<T> pu{r, d, pb[par ^ 1], &s->beta, fused_pap ? c->partials : nullptr};
        if (apply_op<T>(c, mat, op, pc, Ap, none, 0, &s->done, st, &pu)) return SDME_EDEVICE;
        par ^= 1;
        pc = pb[par];
      } else if (apply_op<T>(c, mat, op, pc, Ap, none, 0, &s->done, st)) {
        return SDME_EDEVICE;
      }
      if (c->prof && hipEventRecord(c->ev[2 * j + 1], st) != hipSuccess) return SDME_EDEVICE;
      // p^T A p: block partials of the element energies written by the FP64
      // fused operator, else a separate streaming dot over p and A p
      if (fused_pap) {
        if (launch_pcg_pap_fin(s, red_at(c, 6), op_blocks, st)) return SDME_EDEVICE;
      } else if (launch_pcg_pap<T>(pc, Ap, s, N, red_at(c, 6), st)) {
        return SDME_EDEVICE;
      }
      // fused: pb[par ^ 1] still holds the previous direction (the next
      // operator overwrites it), so the x update can lag one iteration
      if (launch_pcg_update<T>(x, r, pc, Ap, d, s, N, red_at(c, 4), st,
                               fused ? (const T *)pb[par ^ 1] : nullptr))
        return SDME_EDEVICE;
      if (!fused && launch_pcg_pupdate<T>(pc, r, d, s, N, st)) return SDME_EDEVICE;
    }
    if (c->prof) {
      // count only the iterations that ran (later ones return at once)
      if (hipMemcpyAsync(c->h_pcg + slot, s, sizeof(PcgDev), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return SDME_EDEVICE;
      int ran = c->h_pcg[slot].iters - it0;
      int k = sizeof(T) == 8 ? 0 : 1;
      for (int j = 0; j < ran && j < CHUNK; j++) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, c->ev[2 * j], c->ev[2 * j + 1]) != hipSuccess)
          return SDME_EDEVICE;
        c->prof_ms[k] += ms;
        c->prof_count[k] += 1;
      }
    }
  }
  const PcgDev &h = c->h_pcg[slot];
  *iters = h.iters;
  *rel = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
  switch (h.done) {
    case 1: return SDME_OK;
    case 2: return SDME_EBREAKDOWN;
    case 3: return SDME_ENAN;
    default: return SDME_ENOCONV;
  }
}

// Workspace plan of a linear solve with given precision.
struct LinWs {
  double *d64 = nullptr, *r64 = nullptr, *p64 = nullptr, *q64 = nullptr, *Ap64 = nullptr,
         *bm = nullptr;
  float *d32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *Ap32 = nullptr,
        *e32 = nullptr, *b32 = nullptr;
  float *state32 = nullptr;
};

void plan_lin(sdme_ctx *c, int prec, bool need_state32, Bump &b, LinWs &w) {
  int64_t N = 3 * c->Nn;
  w.d64 = b.get<double>(N);
  w.r64 = b.get<double>(N);
  w.p64 = b.get<double>(N);
  w.q64 = b.get<double>(N);
  w.Ap64 = b.get<double>(N);
  w.bm = b.get<double>(N);
  if (prec == SDME_FP32) {
    w.d32 = b.get<float>(N);
    w.r32 = b.get<float>(N);
    w.p32 = b.get<float>(N);
    w.q32 = b.get<float>(N);
    w.Ap32 = b.get<float>(N);
    w.e32 = b.get<float>(N);
    w.b32 = b.get<float>(N);
    if (need_state32) w.state32 = b.get<float>(c->nqp * 10);
  }
}

// Solve (K_T + shift M) x = b (or M x = b) given an FP64 stored state.
int solve_linear(sdme_ctx *c, const sdme_material *mat, int prec, const double *state64,
                 double shift, bool mass_only, const double *b, double *x, double rtol, int maxit,
                 double inner_rtol, LinWs &w, sdme_stats *stats, hipStream_t st,
                 int *its_out = nullptr) {
  Range range("sdme_pcg");
  int64_t N = 3 * c->Nn;
  int P = c->P;
  // masked right-hand side
  if (launch_convert<double, double>(w.bm, b, 1.0, N, st) || launch_bc<double>(w.bm, 0, c->m64, st))
    return SDME_EDEVICE;
  Op<double> op64{mass_only ? 2 : 0, state64, nullptr, shift * mat->rho, mat->rho};
  // FP64 diagonal
  if (launch_fill<double>(w.d64, 0.0, N, st)) return SDME_EDEVICE;
  if (launch_diag<double>(P, mass_only ? c->mm64 : c->m64, mat->mu, mat->lam,
                          mass_only ? nullptr : state64,
                          mass_only ? mat->rho : shift * mat->rho, w.d64, 1, st))
    return SDME_EDEVICE;
  if (launch_bc<double>(w.d64, 1, c->m64, st) || launch_recip(w.d64, N, st)) return SDME_EDEVICE;
  int its = 0;
  double rel = 0;
  if (prec == SDME_FP64) {
    int rc = pcg_core<double>(c, mat, op64, w.bm, x, w.d64, rtol, maxit, w.r64, w.p64, w.Ap64, 0,
                              &its, &rel, st, nullptr, w.q64);
    if (stats) {
      stats->iterations += its;
      stats->rel_residual = rel;
    }
    if (its_out) *its_out = its;
    return rc;
  }
  // mixed: FP32 PCG (FP32 state, operator and vectors, FP64 dots) with FP64
  // residual replacement and FP64 accumulation of the solution
  if (!mass_only && launch_convert<float, double>(w.state32, state64, 1.0, c->nqp * 10, st))
    return SDME_EDEVICE;
  if (launch_convert<float, double>(w.d32, w.d64, 1.0, N, st) ||
      launch_convert<float, double>(w.b32, w.bm, 1.0, N, st) || launch_fill<double>(x, 0.0, N, st))
    return SDME_EDEVICE;
  Op<float> op32{mass_only ? 2 : 0, w.state32, nullptr, (float)(shift * mat->rho), (float)mat->rho};
  Replace rep{&op64, x, w.r64, w.Ap64, w.bm, inner_rtol, 0};
  int rc = pcg_core<float>(c, mat, op32, w.b32, w.e32, w.d32, rtol, maxit, w.r32, w.p32, w.Ap32, 1,
                           &its, &rel, st, &rep, w.q32);
  // on an early stop the FP32 part accumulated since the last replacement
  // still belongs to the iterate
  if ((rc == SDME_EBREAKDOWN || rc == SDME_ENOCONV) && launch_add_scaled_f(x, w.e32, 1.0, N, st))
    return SDME_EDEVICE;
  if (stats) {
    stats->iterations += its;
    stats->outer += rep.count;
    stats->rel_residual = rel;
  }
  if (its_out) *its_out = its;
  return rc;
}

size_t lin_bytes(sdme_ctx *c, int prec, bool state32) {
  Bump b(nullptr, 0);
  LinWs w;
  plan_lin(c, prec, state32, b, w);
  return b.off;
}

}  // namespace


// Workspace of sdme_jacobi_pcg_noalloc: one array per device, resident for
// the life of the process.  Host code never uses the array's name as an
// address: each device's copy is located once with hipGetSymbolAddress (in
// sdme_bind, or at that entry point's first call on the device) and only that
// pointer is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SDME_NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES] = {};

// Address of the current device's scratch array (resolved once per device).
static int scratch_address(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return SDME_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SDME_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SDME_OK;
}

// Layout of the context's device block (tables, reduction partials, solver
// scalars) and host block (scalars read back by the drivers); both are
// allocated by the caller (sdme_context_bytes, sdme_bind).
static void plan_blocks(sdme_ctx *c) {
  const sdme_mesh_desc *d = &c->d;
  const int P = c->P;
  const int TS = (int)c->tab_host.size(), TSM = (int)c->tabm_host.size();
  int nblk = 0;
  for (int q : {c->Q, c->mm64.Q})
    for (int word : {4, 8})
      for (bool grad : {true, false})
        nblk = std::max(nblk, elem_blocks(P, q, word, d->nx, d->ny, d->nz, grad));
  if (nblk < 2 * VEC_BLOCKS) nblk = 2 * VEC_BLOCKS;
  int64_t fb = std::max(std::max(d->nx * d->ny, d->ny * d->nz), d->nx * d->nz);
  if (fb > nblk) nblk = (int)fb;
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t o = bytes;
    bytes += (b + 255) & ~(size_t)255;
    return o;
  };
  BlockPlan &b = c->plan;
  b.o_tm64 = take(sizeof(double) * TSM);
  b.o_tm32 = take(sizeof(float) * TSM);
  b.o_t64 = take(sizeof(double) * TS);
  b.o_t32 = take(sizeof(float) * TS);
  b.o_flag = take(2 * sizeof(int));
  b.o_pcg = take(2 * sizeof(PcgDev));
  b.o_part = take(sizeof(double) * 2 * (size_t)nblk);
  b.o_cnt = take(sizeof(unsigned) * 4);
  b.o_res = take(sizeof(double) * 16);
  // ordered assembly: staging for the largest output of an element launch
  // (element kernels' tiles, element vectors of the diagonal and the body
  // load; face-element vectors are smaller), in either precision
  b.stage_bytes = 0;
  if (d->assembly == SDME_ASSEMBLY_ORDERED) {
    const size_t n3 = (size_t)c->n * c->n * c->n;
    for (int word : {4, 8}) {
      size_t w = (size_t)c->E * 3 * n3;
      for (int q : {c->Q, c->mm64.Q})
        for (bool grad : {true, false})
          w = std::max(w, (size_t)elem_blocks(P, q, word, d->nx, d->ny, d->nz, grad) *
                              (size_t)elem_tile_words(P, q, word, grad));
      b.stage_bytes = std::max(b.stage_bytes, w * word);
    }
  }
  b.o_stage = take(b.stage_bytes);
  b.dev_bytes = bytes;
  b.host_bytes = HOST_BLOCK_BYTES;
  c->tab32_host.resize(TS);
  for (int i = 0; i < TS; i++) c->tab32_host[i] = (float)c->tab_host[i];
  c->tabm32_host.resize(TSM);
  for (int i = 0; i < TSM; i++) c->tabm32_host[i] = (float)c->tabm_host[i];
}

// Every entry point that touches the device requires bound memory.
static int ensure_device(sdme_ctx *c) { return c->dev_ready ? SDME_OK : SDME_EINVAL; }

// ======================================================================= API
extern "C" const char *sdme_status_string(int s) {
  switch (s) {
    case SDME_OK: return "ok";
    case SDME_EINVAL: return "invalid argument";
    case SDME_ENOMEM: return "workspace too small or allocation failed";
    case SDME_EDEVICE: return "HIP runtime error";
    case SDME_EEIG: return "basis eigensolve or factorisation failed";
    case SDME_EJAC: return "det F <= 0 at a Gauss point";
    case SDME_ENOCONV: return "iteration limit reached before tolerance";
    case SDME_EBREAKDOWN: return "CG breakdown (p^T A p <= 0)";
    case SDME_ENAN: return "non-finite value";
    default: return "unknown status";
  }
}

namespace {
// Tables of Dims<P, Q>: B, D, W, B*B, D*D, B*D at the Q points of the volume
// rule; Bf, Wf at the P+1 Gauss-Legendre points of the face rule.
bool build_tables(const Basis &basis, int P, int Q, std::vector<double> &tab) {
  const int n = P + 1;
  tab.assign(2 * Q * n + Q + 3 * Q * n + n * n + n, 0.0);
  std::vector<double> xq(Q), wq(Q), v(n), dv(n);
  if (!sdme::volume_rule(P, Q, xq.data(), wq.data())) return false;
  for (int q = 0; q < Q; q++) {
    basis.eval(xq[q], v.data(), dv.data());
    for (int s = 0; s < n; s++) {
      tab[q * n + s] = v[s];
      tab[Q * n + q * n + s] = dv[s];
      int o = 2 * Q * n + Q;
      tab[o + q * n + s] = v[s] * v[s];
      tab[o + Q * n + q * n + s] = dv[s] * dv[s];
      tab[o + 2 * Q * n + q * n + s] = v[s] * dv[s];
    }
    tab[2 * Q * n + q] = wq[q];
  }
  std::vector<double> xf(n), wf(n);
  sdme::gauss_legendre(n, xf.data(), wf.data());
  int of = 2 * Q * n + Q + 3 * Q * n;
  for (int i = 0; i < n; i++) {
    basis.eval(xf[i], v.data(), nullptr);
    for (int s = 0; s < n; s++) tab[of + i * n + s] = v[s];
    tab[of + n * n + i] = wf[i];
  }
  return true;
}
}  // namespace

extern "C" int sdme_create(const sdme_mesh_desc *d, sdme_ctx **out) {
  if (!d || !out) return SDME_EINVAL;
  *out = nullptr;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->P < 1 || d->P > 8 ||
      (d->Q != d->P + 2 && d->Q != d->P + 1) || d->mass_rule < 0 || d->mass_rule > 1 ||
      d->basis < 0 || d->basis > 4 || !(d->k >= 0 && d->k <= 1) || !(d->lambda_h >= 0) ||
      (d->assembly != SDME_ASSEMBLY_ATOMIC && d->assembly != SDME_ASSEMBLY_ORDERED) ||
      !(d->h[0] > 0 && d->h[1] > 0 && d->h[2] > 0) || (d->dirichlet >> 18) != 0)
    return SDME_EINVAL;
  int64_t Nx = (int64_t)d->nx * d->P + 1, Ny = (int64_t)d->ny * d->P + 1,
          Nz = (int64_t)d->nz * d->P + 1;
  int64_t Nn = Nx * Ny * Nz, E = (int64_t)d->nx * d->ny * d->nz;
  if (3 * Nn >= (int64_t)1 << 31 || E >= (int64_t)1 << 31) return SDME_EINVAL;
  sdme_ctx *c = new (std::nothrow) sdme_ctx();
  if (!c) return SDME_ENOMEM;
  c->d = *d;
  c->P = d->P;
  c->Q = d->Q;
  c->n = d->P + 1;
  c->Nn = Nn;
  c->E = E;
  c->nqp = E * d->Q * d->Q * d->Q;
  if (!c->basis.build(d->P, d->basis, d->k, d->lambda_h)) {
    delete c;
    return SDME_EEIG;
  }
  // tables: B, D, W, B*B, D*D, B*D at Q points; Bf, Wf at P+1 points
  int P = d->P, Q = d->Q, n = P + 1;
  std::vector<double> tab;
  if (!build_tables(c->basis, P, Q, tab) ||
      (d->mass_rule == 1 && !build_tables(c->basis, P, P + 1, c->tabm_host))) {
    delete c;
    return SDME_EEIG;
  }
  c->tab_host = tab;
  MeshK<double> &m = c->m64;
  m.nx = d->nx; m.ny = d->ny; m.nz = d->nz; m.E = (int)E;
  m.Nx = (int)Nx; m.Ny = (int)Ny; m.Nz = (int)Nz; m.Nn = (int)Nn; m.Q = Q;
  m.bc = d->dirichlet;
  for (int j = 0; j < 3; j++) m.ih[j] = 2.0 / d->h[j];
  m.detJ = d->h[0] * d->h[1] * d->h[2] / 8.0;
  m.tab = nullptr;
  m.flag = nullptr;
  m.stage = nullptr;
  MeshK<float> &f = c->m32;
  f.nx = m.nx; f.ny = m.ny; f.nz = m.nz; f.E = m.E;
  f.Nx = m.Nx; f.Ny = m.Ny; f.Nz = m.Nz; f.Nn = m.Nn; f.Q = m.Q;
  f.bc = m.bc;
  for (int j = 0; j < 3; j++) f.ih[j] = (float)m.ih[j];
  f.detJ = (float)m.detJ;
  f.tab = nullptr;
  f.flag = nullptr;
  f.stage = nullptr;
  c->mm64 = c->m64;
  c->mm32 = c->m32;
  if (!c->tabm_host.empty()) c->mm64.Q = c->mm32.Q = c->P + 1;
  plan_blocks(c);
  *out = c;
  return SDME_OK;
}

extern "C" int sdme_context_bytes(const sdme_ctx *c, size_t *dev_bytes, size_t *host_bytes) {
  if (!c || !dev_bytes || !host_bytes) return SDME_EINVAL;
  *dev_bytes = c->plan.dev_bytes;
  *host_bytes = c->plan.host_bytes;
  return SDME_OK;
}

extern "C" int sdme_jac_element(const sdme_ctx *c, int64_t *element) {
  if (!c || !element) return SDME_EINVAL;
  *element = c->jac_element;
  return SDME_OK;
}

extern "C" int sdme_bind(sdme_ctx *c, void *dev_block, size_t dev_bytes, void *host_block,
                         size_t host_bytes, void *stream) {
  if (!c || !dev_block || !host_block || dev_bytes < c->plan.dev_bytes ||
      host_bytes < c->plan.host_bytes || ((uintptr_t)dev_block & 255) != 0 ||
      ((uintptr_t)host_block & 7) != 0)
    return SDME_EINVAL;
  const BlockPlan &b = c->plan;
  hipStream_t st = S(stream);
  char *base = (char *)dev_block;
  c->dev_block = dev_block;
  c->host_block = host_block;
  c->tab64 = (double *)(base + b.o_t64);
  c->tabm64 = (double *)(base + b.o_tm64);
  c->tabm32 = (float *)(base + b.o_tm32);
  c->tab32 = (float *)(base + b.o_t32);
  c->flag = (int *)(base + b.o_flag);
  c->pcg = (PcgDev *)(base + b.o_pcg);
  c->partials = (double *)(base + b.o_part);
  c->counter = (unsigned *)(base + b.o_cnt);
  c->results = (double *)(base + b.o_res);
  c->h_pcg = (PcgDev *)host_block;
  c->h_res = (double *)((char *)host_block + 1024);
  c->h_flag = (int *)((char *)host_block + 2048);
  std::memset(host_block, 0, b.host_bytes);
  void *scr = nullptr;
  if (scratch_address(&scr)) return SDME_EDEVICE;  // library set-up on this device
  const size_t TS = c->tab_host.size(), TSM = c->tabm_host.size();
  // zero fill by a kernel (no memset node, so a caller may capture the
  // binding; the staging array is written before it is read and is left as
  // it is), then the tables, both on the caller's stream
  if (launch_fill<double>((double *)dev_block, 0.0, (int64_t)(b.o_stage / 8), st) ||
      hipMemcpyAsync(c->tab64, c->tab_host.data(), sizeof(double) * TS, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(c->tab32, c->tab32_host.data(), sizeof(float) * TS, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      (TSM && (hipMemcpyAsync(c->tabm64, c->tabm_host.data(), sizeof(double) * TSM,
                              hipMemcpyHostToDevice, st) != hipSuccess ||
               hipMemcpyAsync(c->tabm32, c->tabm32_host.data(), sizeof(float) * TSM,
                              hipMemcpyHostToDevice, st) != hipSuccess))) {
    c->dev_ready = false;
    return SDME_EDEVICE;
  }
  c->m64.tab = c->tab64;
  c->m64.flag = c->flag;
  c->m32.tab = c->tab32;
  c->m32.flag = c->flag;
  c->mm64.flag = c->mm32.flag = c->flag;
  c->mm64.tab = TSM ? c->tabm64 : c->tab64;
  c->mm32.tab = TSM ? c->tabm32 : c->tab32;
  // one staging array for both precisions: its users run one after another
  // on the call's stream
  double *stage64 = b.stage_bytes ? (double *)(base + b.o_stage) : nullptr;
  c->m64.stage = c->mm64.stage = stage64;
  c->m32.stage = c->mm32.stage = (float *)stage64;
  c->dev_ready = true;
  return SDME_OK;
}

extern "C" int sdme_profile(sdme_ctx *c, int enable, double ms_out[2], int64_t count_out[2]) {
  if (!c) return SDME_EINVAL;
  if (ms_out) {
    ms_out[0] = c->prof_ms[0];
    ms_out[1] = c->prof_ms[1];
  }
  if (count_out) {
    count_out[0] = c->prof_count[0];
    count_out[1] = c->prof_count[1];
  }
  if (enable && c->ev.empty()) {
    c->ev.resize(2 * CHUNK);
    for (auto &e : c->ev)
      if (hipEventCreate(&e) != hipSuccess) return SDME_EDEVICE;
  }
  c->prof = enable != 0;
  c->prof_ms[0] = c->prof_ms[1] = 0;
  c->prof_count[0] = c->prof_count[1] = 0;
  return SDME_OK;
}

extern "C" int sdme_destroy(sdme_ctx *c) {
  if (!c) return SDME_EINVAL;
  for (auto &e : c->ev) hipEventDestroy(e);
  // the device and host blocks belong to the caller
  delete c;
  return SDME_OK;
}

extern "C" int sdme_sizes(const sdme_ctx *c, int64_t out[4]) {
  if (!c || !out) return SDME_EINVAL;
  out[0] = c->Nn;
  out[1] = c->E;
  out[2] = c->nqp;
  out[3] = 10;
  return SDME_OK;
}

extern "C" int sdme_gather_indices(const sdme_ctx *c, int32_t *o) {
  if (!c || !o) return SDME_EINVAL;
  int P = c->P, n = c->n;
  const MeshK<double> &m = c->m64;
  for (int64_t e = 0; e < c->E; e++) {
    int ex = (int)(e % m.nx), ey = (int)((e / m.nx) % m.ny), ez = (int)(e / ((int64_t)m.nx * m.ny));
    int32_t *row = o + e * (int64_t)n * n * n;
    for (int cc = 0; cc < n; cc++)
      for (int b = 0; b < n; b++)
        for (int a = 0; a < n; a++)
          row[(cc * n + b) * n + a] =
              (int32_t)(((int64_t)(ez * P + cc) * m.Ny + (ey * P + b)) * m.Nx + (ex * P + a));
  }
  return SDME_OK;
}

extern "C" int sdme_dirichlet_flags(const sdme_ctx *c, uint8_t *o) {
  if (!c || !o) return SDME_EINVAL;
  const MeshK<double> &m = c->m64;
  for (int comp = 0; comp < 3; comp++)
    for (int64_t g = 0; g < c->Nn; g++) {
      int ix = (int)(g % m.Nx), iy = (int)((g / m.Nx) % m.Ny), iz = (int)(g / ((int64_t)m.Nx * m.Ny));
      uint32_t mm = m.bc >> comp;
      bool k = ((mm & 1u) && ix == 0) || (((mm >> 3) & 1u) && ix == m.Nx - 1) ||
               (((mm >> 6) & 1u) && iy == 0) || (((mm >> 9) & 1u) && iy == m.Ny - 1) ||
               (((mm >> 12) & 1u) && iz == 0) || (((mm >> 15) & 1u) && iz == m.Nz - 1);
      o[comp * c->Nn + g] = k ? 1 : 0;
    }
  return SDME_OK;
}

extern "C" int sdme_affine_field(const sdme_ctx *c, const double a[3], const double G[9],
                                 double *o) {
  if (!c || !a || !G || !o) return SDME_EINVAL;
  int P = c->P, n = c->n;
  std::vector<double> g1(n), gx(n);
  if (!c->basis.affine(g1.data(), gx.data())) return SDME_EEIG;
  const MeshK<double> &m = c->m64;
  const double *h = c->d.h;
  for (int ez = 0; ez < m.nz; ez++)
    for (int ey = 0; ey < m.ny; ey++)
      for (int ex = 0; ex < m.nx; ex++) {
        double Xc[3] = {c->d.origin[0] + (ex + 0.5) * h[0], c->d.origin[1] + (ey + 0.5) * h[1],
                        c->d.origin[2] + (ez + 0.5) * h[2]};
        for (int i = 0; i < 3; i++) {
          double c0 = a[i] + G[i * 3] * Xc[0] + G[i * 3 + 1] * Xc[1] + G[i * 3 + 2] * Xc[2];
          for (int cc = 0; cc < n; cc++)
            for (int b = 0; b < n; b++)
              for (int aa = 0; aa < n; aa++) {
                double v = c0 * g1[aa] * g1[b] * g1[cc] +
                           G[i * 3 + 0] * h[0] / 2 * gx[aa] * g1[b] * g1[cc] +
                           G[i * 3 + 1] * h[1] / 2 * g1[aa] * gx[b] * g1[cc] +
                           G[i * 3 + 2] * h[2] / 2 * g1[aa] * g1[b] * gx[cc];
                int64_t g = ((int64_t)(ez * P + cc) * m.Ny + (ey * P + b)) * m.Nx + (ex * P + aa);
                o[i * c->Nn + g] = v;
              }
        }
      }
  return SDME_OK;
}

// ------------------------------------------------------------------ operators
extern "C" int sdme_internal_force(sdme_ctx *c, const sdme_material *mat, int prec, const void *u,
                                   void *R, void *state, int flags, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u || !R || !valid_prec(prec)) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  int64_t N = 3 * c->Nn;
  int rc;
  if ((flags & SDME_CHECK_JAC) && (rc = clear_flag(c, st))) return rc;
  int mask = (flags & SDME_MASK_BC) ? 1 : 0;
  if (prec == SDME_FP64) {
    if (launch_fill<double>((double *)R, 0.0, N, st)) return SDME_EDEVICE;
    rc = lerr(launch_force<double>(c->P, c->m64, mat->mu, mat->lam, (const double *)u, (double *)R,
                                   (double *)state, mask, st));
  } else {
    if (launch_fill<float>((float *)R, 0.0f, N, st)) return SDME_EDEVICE;
    rc = lerr(launch_force<float>(c->P, c->m32, mat->mu, mat->lam, (const float *)u, (float *)R,
                                  (float *)state, mask, st));
  }
  if (rc) return rc;
  if (flags & SDME_CHECK_JAC) return read_flag(c, st);
  return SDME_OK;
}

extern "C" int sdme_linearize(sdme_ctx *c, const sdme_material *mat, int prec, const void *u,
                              void *state, int flags, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u || !state || !valid_prec(prec)) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  int rc;
  if ((flags & SDME_CHECK_JAC) && (rc = clear_flag(c, st))) return rc;
  if (prec == SDME_FP64)
    rc = lerr(launch_force<double>(c->P, c->m64, mat->mu, mat->lam, (const double *)u, nullptr,
                                   (double *)state, 0, st));
  else
    rc = lerr(launch_force<float>(c->P, c->m32, mat->mu, mat->lam, (const float *)u, nullptr,
                                  (float *)state, 0, st));
  if (rc) return rc;
  if (flags & SDME_CHECK_JAC) return read_flag(c, st);
  return SDME_OK;
}

extern "C" int sdme_tangent_apply(sdme_ctx *c, const sdme_material *mat, int prec,
                                  const void *u_lin, const void *state, double mass_shift,
                                  const void *v, void *y, int flags, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !v || !y || !valid_prec(prec) ||
      (u_lin == nullptr) == (state == nullptr) || !std::isfinite(mass_shift) ||
      (c->d.mass_rule && mass_shift != 0.0))
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  int64_t N = 3 * c->Nn;
  int mask = (flags & SDME_MASK_BC) ? 1 : 0;
  int rc;
  if ((flags & SDME_CHECK_JAC) && (rc = clear_flag(c, st))) return rc;
  Reduce none{c->partials, c->counter, c->results + 8};
  if (prec == SDME_FP64) {
    if (launch_fill<double>((double *)y, 0.0, N, st)) return SDME_EDEVICE;
    rc = lerr(launch_tangent<double>(c->P, c->m64, mat->mu, mat->lam, (const double *)u_lin,
                                     (const double *)state, mass_shift * mat->rho,
                                     (const double *)v, (double *)y, mask, nullptr, nullptr, st));
  } else {
    if (launch_fill<float>((float *)y, 0.0f, N, st)) return SDME_EDEVICE;
    rc = lerr(launch_tangent<float>(c->P, c->m32, mat->mu, mat->lam, (const float *)u_lin,
                                    (const float *)state, (float)(mass_shift * mat->rho),
                                    (const float *)v, (float *)y, mask, nullptr, nullptr, st));
  }
  if (rc) return rc;
  if ((flags & SDME_CHECK_JAC) && u_lin) return read_flag(c, st);
  return SDME_OK;
}

extern "C" int sdme_mass_apply(sdme_ctx *c, double rho, int prec, const void *v, void *y,
                               int flags, void *stream) {
  if (!c || !v || !y || !valid_prec(prec) || !std::isfinite(rho)) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  int mask = (flags & SDME_MASK_BC) ? 1 : 0;
  Reduce none{c->partials, c->counter, c->results + 8};
  // the mass kernel writes every slot of y (no zero fill first)
  if (prec == SDME_FP64)
    return lerr(launch_mass<double>(c->P, c->mm64, rho, (const double *)v, (double *)y, mask, none,
                                    0, nullptr, st));
  return lerr(launch_mass<float>(c->P, c->mm32, (float)rho, (const float *)v, (float *)y, mask,
                                 none, 0, nullptr, st));
}

extern "C" int sdme_jacobi_diag(sdme_ctx *c, const sdme_material *mat, int prec,
                                const void *state, double mass_shift, void *d, int flags,
                                void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !state || !d || !valid_prec(prec) ||
      (c->d.mass_rule && mass_shift != 0.0))
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  int64_t N = 3 * c->Nn;
  int mask = (flags & SDME_MASK_BC) ? 1 : 0;
  if (prec == SDME_FP64) {
    if (launch_fill<double>((double *)d, 0.0, N, st)) return SDME_EDEVICE;
    if (launch_diag<double>(c->P, c->m64, mat->mu, mat->lam, (const double *)state,
                            mass_shift * mat->rho, (double *)d, mask, st))
      return SDME_EDEVICE;
    if (mask && launch_bc<double>((double *)d, 1, c->m64, st)) return SDME_EDEVICE;
    return SDME_OK;
  }
  if (launch_fill<float>((float *)d, 0.0f, N, st)) return SDME_EDEVICE;
  if (launch_diag<float>(c->P, c->m32, mat->mu, mat->lam, (const float *)state,
                         (float)(mass_shift * mat->rho), (float *)d, mask, st))
    return SDME_EDEVICE;
  if (mask && launch_bc<float>((float *)d, 1, c->m32, st)) return SDME_EDEVICE;
  return SDME_OK;
}

extern "C" int sdme_strain_energy(sdme_ctx *c, const sdme_material *mat, const double *u,
                                  double *out, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u || !out) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  if (launch_energy(c->P, c->m64, mat->mu, mat->lam, u, red_at(c, 10), st)) return SDME_EDEVICE;
  if (hipMemcpyAsync(c->h_res, c->results + 10, sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SDME_EDEVICE;
  *out = c->h_res[0];
  return SDME_OK;
}

extern "C" int sdme_face_traction(sdme_ctx *c, int face, const double t[3], double scale,
                                  double *f, void *stream) {
  if (!c || !t || !f || face < 0 || face > 5) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  return lerr(launch_face(c->P, c->m64, 0, face, t, scale, 0, 0, 0, nullptr, f,
                          red_at(c, 11), 0, S(stream)));
}

extern "C" int sdme_penalty_plane(sdme_ctx *c, const sdme_contact *ct, const double *u, double *f,
                                  double *energy, void *stream) {
  if (!c || !ct || !u || !f || !(ct->eps >= 0)) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  int rc = lerr(launch_face(c->P, c->m64, 1, 4, nullptr, 1.0, ct->eps, ct->z0, c->d.origin[2], u,
                            f, red_at(c, 11), energy ? 1 : 0, st));
  if (rc || !energy) return rc;
  if (hipMemcpyAsync(c->h_res, c->results + 11, sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SDME_EDEVICE;
  *energy = c->h_res[0];
  return SDME_OK;
}

extern "C" int sdme_quadrature_points(const sdme_ctx *c, int face, double *o) {
  if (!c || !o || face < -1 || face > 5) return SDME_EINVAL;
  const sdme_mesh_desc &d = c->d;
  const int ne[3] = {d.nx, d.ny, d.nz};
  if (face < 0) {
    const int Q = c->Q, Q3 = Q * Q * Q;
    std::vector<double> x(Q), w(Q);
    sdme::volume_rule(c->P, Q, x.data(), w.data());
    for (int64_t e = 0; e < c->E; e++) {
      const int ei[3] = {(int)(e % d.nx), (int)((e / d.nx) % d.ny),
                         (int)(e / ((int64_t)d.nx * d.ny))};
      for (int q = 0; q < Q3; q++) {
        const int qi[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
        for (int k = 0; k < 3; k++)
          o[((size_t)k * c->E + e) * Q3 + q] =
              d.origin[k] + d.h[k] * (ei[k] + 0.5 * (1.0 + x[qi[k]]));
      }
    }
    return SDME_OK;
  }
  const int dir = face / 2, side = face % 2, t1 = dir == 0 ? 1 : 0, t2 = dir == 2 ? 1 : 2;
  const int nq = c->P + 1, nfe = ne[t1] * ne[t2];
  std::vector<double> x(nq), w(nq);
  sdme::gauss_legendre(nq, x.data(), w.data());
  for (int fe = 0; fe < nfe; fe++) {
    const int i = fe % ne[t1], j = fe / ne[t1];
    for (int p = 0; p < nq * nq; p++) {
      const int pi = p % nq, pj = p / nq;
      double X[3];
      X[dir] = d.origin[dir] + (side ? ne[dir] * d.h[dir] : 0.0);
      X[t1] = d.origin[t1] + d.h[t1] * (i + 0.5 * (1.0 + x[pi]));
      X[t2] = d.origin[t2] + d.h[t2] * (j + 0.5 * (1.0 + x[pj]));
      for (int k = 0; k < 3; k++) o[((size_t)k * nfe + fe) * nq * nq + p] = X[k];
    }
  }
  return SDME_OK;
}

extern "C" int sdme_body_load(sdme_ctx *c, const double *b, double *f, void *stream) {
  if (!c || !b || !f) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  return lerr(launch_body_load(c->P, c->m64, b, f, S(stream)));
}

extern "C" int sdme_face_load(sdme_ctx *c, int face, const double *t, double *f, void *stream) {
  if (!c || !t || !f || face < 0 || face > 5) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  return lerr(launch_face_load(c->P, c->m64, face, t, f, S(stream)));
}

extern "C" int sdme_l2_error(sdme_ctx *c, const double *u, const double *g, double *out,
                             void *stream) {
  if (!c || !u || !g || !out) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  // 3 partials per block: at most VEC_BLOCKS blocks (the partials buffer
  // holds at least 4 VEC_BLOCKS doubles)
  if (launch_l2_error(c->P, c->m64, u, g, c->partials, VEC_BLOCKS, c->results + 13, st))
    return SDME_EDEVICE;
  if (hipMemcpyAsync(c->h_res, c->results + 13, 3 * sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SDME_EDEVICE;
  for (int k = 0; k < 3; k++) out[k] = std::sqrt(c->h_res[k]);
  return SDME_OK;
}

extern "C" int sdme_material_grad_accumulate(sdme_ctx *c, const double *u, const double *w,
                                             double scale, double *gm, double *gl, void *stream) {
  if (!c || !u || !w || !gm || !gl || !std::isfinite(scale)) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  return lerr(launch_matgrad(c->P, c->m64, u, w, scale, gm, gl, S(stream)));
}

extern "C" int sdme_axpby(sdme_ctx *c, int64_t n, double alpha, const double *x, double beta,
                          double *y, void *stream) {
  if (!c || n < 0 || (n > 0 && (!x || !y))) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  if (n == 0) return SDME_OK;
  return lerr(launch_axpby(y, alpha, x, beta, n, S(stream)));
}

extern "C" int sdme_misfit(sdme_ctx *c, const double *u, const double *target, double *lam,
                           double *J, void *stream) {
  if (!c || !u || !target || !lam || !J) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  int64_t N = 3 * c->Nn;
  if (launch_axpbypcz(lam, 1.0, u, 0.0, -1.0, target, N, st) || launch_bc<double>(lam, 0, c->m64, st))
    return SDME_EDEVICE;
  double dd[2];
  int rc = dot2<double>(c, lam, lam, N, dd, st);
  if (rc) return rc;
  *J = 0.5 * dd[1];
  return SDME_OK;
}

// -------------------------------------------------------------------- solvers
extern "C" int sdme_workspace_bytes(const sdme_ctx *cc, int op, int prec, size_t *bytes) {
  if (!cc || !bytes || !valid_prec(prec)) return SDME_EINVAL;
  sdme_ctx *c = const_cast<sdme_ctx *>(cc);
  int64_t N = 3 * c->Nn;
  size_t st64 = ((size_t)c->nqp * 10 * sizeof(double) + 255) & ~(size_t)255;
  size_t vec = ((size_t)N * sizeof(double) + 255) & ~(size_t)255;
  switch (op) {
    case SDME_OP_PCG:
      *bytes = st64 + lin_bytes(c, prec, true);
      break;
    case SDME_OP_NEWTON:
      *bytes = st64 + 4 * vec + lin_bytes(c, prec, true);
      break;
    case SDME_OP_NEWMARK:
      *bytes = st64 + 7 * vec + lin_bytes(c, prec, true);
      break;
    case SDME_OP_CONDENSED: {
      const int nI = interior_size(c->P);
      *bytes = st64 + ((size_t)c->E * nI * nI * sizeof(double) + 255 & ~(size_t)255) + 8 * vec;
      break;
    }
    case SDME_OP_EXPLICIT:
    case SDME_OP_ADJOINT:
      *bytes = 6 * vec + 2 * (((size_t)N * sizeof(float) + 255) & ~(size_t)255) +
               lin_bytes(c, SDME_FP64, false);
      break;
    default:
      return SDME_EINVAL;
  }
  return SDME_OK;
}

extern "C" int sdme_jacobi_pcg(sdme_ctx *c, const sdme_material *mat, int prec, const double *u_lin,
                               double shift, int mass_only, const double *b, double *x, double rtol,
                               int maxit, double inner_rtol, sdme_stats *stats, void *ws,
                               size_t ws_bytes, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !b || !x || !valid_prec(prec) ||
      (!mass_only && !u_lin) || !(rtol > 0) || maxit < 1 || !(inner_rtol > 0 && inner_rtol < 1) ||
      (c->d.mass_rule && !mass_only && shift != 0.0))
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  Timer tm;
  hipStream_t st = S(stream);
  Bump bp(ws, ws_bytes);
  double *state64 = bp.get<double>(c->nqp * 10);
  LinWs w;
  plan_lin(c, prec, true, bp, w);
  if (!bp.ok) return SDME_ENOMEM;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int rc = SDME_OK;
  if (!mass_only) {
    if (!(rc = clear_flag(c, st))) {
      if (launch_force<double>(c->P, c->m64, mat->mu, mat->lam, u_lin, nullptr, state64, 0, st))
        rc = SDME_EDEVICE;
      else
        rc = read_flag(c, st);
    }
  }
  if (!rc)
    rc = solve_linear(c, mat, prec, state64, shift, mass_only != 0, b, x, rtol, maxit, inner_rtol,
                      w, stats, st);
  if (hipStreamSynchronize(st) != hipSuccess) rc = SDME_EDEVICE;
  if (stats) {
    stats->status = rc;
    stats->time_ms = tm.ms();
  }
  return rc;
}


extern "C" int sdme_jacobi_pcg_noalloc(sdme_ctx *c, const sdme_material *mat, int prec,
                                       const double *u_lin, double shift, int mass_only,
                                       const double *b, double *x, double rtol, int maxit,
                                       double inner_rtol, sdme_stats *stats, void *stream) {
  if (!c || !valid_prec(prec)) return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  size_t need = 0;
  if (int rc_ = sdme_workspace_bytes(c, SDME_OP_PCG, prec, &need)) return rc_;
  if (need > (size_t)SDME_NOALLOC_SCRATCH_BYTES) return SDME_ENOMEM;
  void *ws = nullptr;
  if (int rc_ = scratch_address(&ws)) return rc_;
  // every workspace buffer is written before it is read, so the contents
  // left by an earlier call need no clearing
  return sdme_jacobi_pcg(c, mat, prec, u_lin, shift, mass_only, b, x, rtol, maxit, inner_rtol,
                         stats, ws, (size_t)SDME_NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" int sdme_condensed_sizes(const sdme_ctx *c, int64_t out[3]) {
  if (!c || !out) return SDME_EINVAL;
  const MeshK<double> &m = c->m64;
  int64_t fixed = 0;
  for (int comp = 0; comp < 3; comp++)
    for (int iz = 0; iz < m.Nz; iz++)
      for (int iy = 0; iy < m.Ny; iy++)
        for (int ix = 0; ix < m.Nx; ix++) {
          uint32_t b = c->d.dirichlet >> comp;
          if (((b & 1u) && ix == 0) || (((b >> 3) & 1u) && ix == m.Nx - 1) ||
              (((b >> 6) & 1u) && iy == 0) || (((b >> 9) & 1u) && iy == m.Ny - 1) ||
              (((b >> 12) & 1u) && iz == 0) || (((b >> 15) & 1u) && iz == m.Nz - 1))
            fixed++;
        }
  const int64_t nI = interior_size(c->P);
  out[1] = c->E * nI;
  out[0] = 3 * c->Nn - fixed - out[1];
  out[2] = nI;
  return SDME_OK;
}

extern "C" int sdme_condensed_pcg(sdme_ctx *c, const sdme_material *mat, const double *u_lin,
                                  double shift, int mass_only, const double *b, double *x,
                                  double rtol, int maxit, sdme_stats *stats, void *ws,
                                  size_t ws_bytes, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !b || !x || (!mass_only && !u_lin) ||
      !(rtol > 0) || maxit < 1 || c->d.mass_rule != 0 || !std::isfinite(shift))
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  Timer tm;
  hipStream_t st = S(stream);
  const int64_t N = 3 * c->Nn;
  const int P = c->P, nI = interior_size(P);
  Bump bp(ws, ws_bytes);
  double *state64 = bp.get<double>(c->nqp * 10);
  double *Kinv = bp.get<double>((int64_t)c->E * nI * nI);
  double *bm = bp.get<double>(N), *d = bp.get<double>(N), *r = bp.get<double>(N),
         *p = bp.get<double>(N), *Ap = bp.get<double>(N), *t = bp.get<double>(N),
         *z = bp.get<double>(N), *g = bp.get<double>(N);
  if (!bp.ok) return SDME_ENOMEM;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int rc = SDME_OK;
  const double msr = mass_only ? mat->rho : shift * mat->rho;
  const double *state = mass_only ? nullptr : state64;
  // linearisation state, interior blocks and their inverses
  if (!(rc = clear_flag(c, st))) {
    if (!mass_only &&
        launch_force<double>(P, c->m64, mat->mu, mat->lam, u_lin, nullptr, state64, 0, st))
      rc = SDME_EDEVICE;
    else if (!mass_only)
      rc = read_flag(c, st);
  }
  if (!rc && (launch_interior_block(P, c->m64, mat->mu, mat->lam, state, msr, Kinv, st) ||
              launch_interior_invert(P, (int)c->E, Kinv, c->flag, st)))
    rc = SDME_EDEVICE;
  if (!rc && read_flag(c, st)) rc = SDME_EBREAKDOWN;  // an interior block not SPD
  // Jacobi preconditioner: the diagonal of the operator on the remaining slots
  if (!rc && (launch_fill<double>(d, 0.0, N, st) ||
              launch_diag<double>(P, c->m64, mat->mu, mat->lam, state, msr, d, 1, st) ||
              launch_bc<double>(d, 1, c->m64, st) ||
              launch_interior_set(P, c->m64, d, 1.0, nullptr, st) || launch_recip(d, N, st)))
    rc = SDME_EDEVICE;
  Op<double> op{3, state, nullptr, mass_only ? 0.0 : msr, mat->rho};
  op.inner = mass_only ? 2 : 0;
  op.Kinv = Kinv;
  op.t = t;
  op.z = z;
  Op<double> in = op;
  in.kind = op.inner;
  Reduce none{c->partials, c->counter, c->results + 8};
  // condensed right-hand side g = b - A_{.I} inv(A_II) b_I off the interiors
  if (!rc && (launch_convert<double, double>(bm, b, 1.0, N, st) ||
              launch_bc<double>(bm, 0, c->m64, st) || launch_fill<double>(z, 0.0, N, st) ||
              launch_interior_apply(P, c->m64, Kinv, bm, z, 1.0, nullptr, st) ||
              launch_fill<double>(t, 0.0, N, st) ||
              apply_op<double>(c, mat, in, z, t, none, 0, nullptr, st) ||
              launch_axpbypcz(g, 1.0, bm, 0.0, -1.0, t, N, st) ||
              launch_interior_set(P, c->m64, g, 0.0, nullptr, st)))
    rc = SDME_EDEVICE;
  int its = 0;
  double rel = 0;
  if (!rc)
    rc = pcg_core<double>(c, mat, op, g, x, d, rtol, maxit, r, p, Ap, 0, &its, &rel, st);
  // interior modes from the boundary solution (Eq. Schur_split2)
  if ((rc == SDME_OK || rc == SDME_ENOCONV) &&
      (launch_fill<double>(t, 0.0, N, st) ||
       apply_op<double>(c, mat, in, x, t, none, 0, nullptr, st) ||
       launch_axpbypcz(t, 1.0, bm, -1.0, 0.0, t, N, st) ||
       launch_interior_apply(P, c->m64, Kinv, t, x, 1.0, nullptr, st)))
    rc = SDME_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) rc = SDME_EDEVICE;
  if (stats) {
    stats->iterations = its;
    stats->rel_residual = rel;
    stats->status = rc;
    stats->time_ms = tm.ms();
  }
  return rc;
}

namespace {

// Newton loop shared by the static solve and the Newmark step.  The residual
// is psi = f - R(u) - M (shift (u - u_n) - c2 v_n - c3 a_n) when dyn != 0.
struct Dyn {
  const double *u_n, *v_n, *a_n;
  double b1, b2, b3;
};

int newton_loop(sdme_ctx *c, const sdme_material *mat, int prec, double *u, const double *f_ext,
                const Dyn *dyn, double newton_rtol, double pcg_rtol, int max_newton, int max_pcg,
                sdme_stats *stats, void *ws, size_t ws_bytes, hipStream_t st) {
  int64_t N = 3 * c->Nn;
  Bump bp(ws, ws_bytes);
  double *state64 = bp.get<double>(c->nqp * 10);
  double *R = bp.get<double>(N), *psi = bp.get<double>(N), *du = bp.get<double>(N),
         *acc = bp.get<double>(N);
  LinWs w;
  plan_lin(c, prec, true, bp, w);
  if (!bp.ok) return SDME_ENOMEM;
  double psi0 = -1, nrm = 0;
  int rc = SDME_OK;
  double shift = dyn ? dyn->b1 : 0.0;
  // Damped Newton: when the updated state inverts an element (det F <= 0),
  // the last increment is halved (u -= alpha du, alpha halved), up to 20
  // times per Newton iteration.
  double alpha = 1.0;
  int halvings = 0;
  for (int k = 0;; k++) {
    Range range("sdme_newton_iteration");
    if ((rc = clear_flag(c, st))) return rc;
    if (launch_fill<double>(R, 0.0, N, st) ||
        launch_force<double>(c->P, c->m64, mat->mu, mat->lam, u, R, state64, 1, st))
      return SDME_EDEVICE;
    if ((rc = read_flag(c, st))) {
      if (rc != SDME_EJAC || k == 0 || halvings >= 20) return rc;
      alpha *= 0.5;
      halvings++;
      if (stats) stats->halvings++;
      if (launch_axpby(u, -alpha, du, 1.0, N, st)) return SDME_EDEVICE;
      k--;
      continue;
    }
    alpha = 1.0;
    halvings = 0;
    // psi = f - R
    if (f_ext) {
      if (launch_axpbypcz(psi, 1.0, f_ext, 0.0, -1.0, R, N, st)) return SDME_EDEVICE;
    } else {
      if (launch_axpbypcz(psi, -1.0, R, 0.0, 0.0, nullptr, N, st)) return SDME_EDEVICE;
    }
    if (dyn) {
      // acc = b1 (u - u_n) - b2 v_n - b3 a_n ; psi -= M acc
      if (launch_axpbypcz(acc, dyn->b1, u, 0.0, -dyn->b1, dyn->u_n, N, st) ||
          launch_axpbypcz(acc, -dyn->b2, dyn->v_n, 1.0, -dyn->b3, dyn->a_n, N, st) ||
          launch_fill<double>(du, 0.0, N, st))
        return SDME_EDEVICE;
      Reduce none{c->partials, c->counter, c->results + 8};
      if (launch_mass<double>(c->P, c->mm64, mat->rho, acc, du, 1, none, 0, nullptr, st))
        return SDME_EDEVICE;
      if (launch_axpby(psi, -1.0, du, 1.0, N, st)) return SDME_EDEVICE;
    }
    if (launch_bc<double>(psi, 0, c->m64, st)) return SDME_EDEVICE;
    double dd[2];
    if ((rc = dot2<double>(c, psi, psi, N, dd, st))) return rc;
    nrm = std::sqrt(dd[1]);
    if (!std::isfinite(nrm)) return SDME_ENAN;
    if (psi0 < 0) psi0 = nrm;
    if (stats) stats->newton_rel = psi0 > 0 ? nrm / psi0 : 0.0;
    if (nrm <= newton_rtol * psi0 || nrm == 0.0) break;
    if (k >= max_newton) return SDME_ENOCONV;
    int lin_its = 0;
    rc = solve_linear(c, mat, prec, state64, shift, false, psi, du, pcg_rtol, max_pcg, 1e-2, w,
                      stats, st, &lin_its);
    // Non-positive curvature met inside PCG (an iterate where K_T is not
    // positive definite): take the CG iterate reached before it as the
    // increment (truncated Newton-CG); the next Newton iteration re-linearises.
    if (rc == SDME_EBREAKDOWN && lin_its > 0) rc = SDME_OK;
    if (rc) return rc;
    if (launch_axpby(u, 1.0, du, 1.0, N, st)) return SDME_EDEVICE;
    if (stats) stats->newton++;
  }
  return SDME_OK;
}

}  // namespace

extern "C" int sdme_newton_static(sdme_ctx *c, const sdme_material *mat, int prec, double *u,
                                  const double *f_ext, double newton_rtol, double pcg_rtol,
                                  int max_newton, int max_pcg, sdme_stats *stats, void *ws,
                                  size_t ws_bytes, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u || !valid_prec(prec) || !(newton_rtol > 0) ||
      !(pcg_rtol > 0) || max_newton < 0 || max_pcg < 1)
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  Timer tm;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int rc = newton_loop(c, mat, prec, u, f_ext, nullptr, newton_rtol, pcg_rtol, max_newton, max_pcg,
                       stats, ws, ws_bytes, S(stream));
  if (stats) {
    stats->status = rc;
    stats->time_ms = tm.ms();
  }
  return rc;
}

extern "C" int sdme_newmark_newton_step(sdme_ctx *c, const sdme_material *mat, int prec, double *u,
                                        double *v, double *a, const double *f_next, double dt,
                                        double beta, double gamma, double newton_rtol,
                                        double pcg_rtol, int max_newton, int max_pcg,
                                        sdme_stats *stats, void *ws, size_t ws_bytes,
                                        void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u || !v || !a || !valid_prec(prec) || !(dt > 0) ||
      c->d.mass_rule ||
      !(beta > 0) || !(gamma > 0) || !(newton_rtol > 0) || !(pcg_rtol > 0) || max_newton < 0 ||
      max_pcg < 1)
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  Timer tm;
  hipStream_t st = S(stream);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int64_t N = 3 * c->Nn;
  size_t need = 0, total = 0;
  sdme_workspace_bytes(c, SDME_OP_NEWTON, prec, &need);
  sdme_workspace_bytes(c, SDME_OP_NEWMARK, prec, &total);
  if (!ws || ws_bytes < total) return SDME_ENOMEM;
  // copies of the step-n state live at the end of the workspace
  char *tail = (char *)ws + need;
  size_t vb = ((size_t)N * 8 + 255) & ~(size_t)255;
  double *un = (double *)tail, *vn = (double *)(tail + vb), *an = (double *)(tail + 2 * vb);
  if (launch_convert<double, double>(un, u, 1.0, N, st) ||
      launch_convert<double, double>(vn, v, 1.0, N, st) ||
      launch_convert<double, double>(an, a, 1.0, N, st))
    return SDME_EDEVICE;
  Dyn dyn{un, vn, an, 1.0 / (beta * dt * dt), 1.0 / (beta * dt), 1.0 / (2.0 * beta) - 1.0};
  int rc = newton_loop(c, mat, prec, u, f_next, &dyn, newton_rtol, pcg_rtol, max_newton, max_pcg,
                       stats, ws, need, st);
  if (rc == SDME_OK) {
    // a = b1 (u - un) - b2 vn - b3 an ; v = vn + dt ((1-gamma) an + gamma a)
    if (launch_axpbypcz(a, dyn.b1, u, 0.0, -dyn.b1, un, N, st) ||
        launch_axpbypcz(a, -dyn.b2, vn, 1.0, -dyn.b3, an, N, st) ||
        launch_bc<double>(a, 0, c->m64, st) ||
        launch_axpbypcz(v, dt * gamma, a, 1.0, dt * (1.0 - gamma), an, N, st) ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = SDME_EDEVICE;
  }
  if (stats) {
    stats->status = rc;
    stats->time_ms = tm.ms();
  }
  return rc;
}

namespace {

// f = P - R(u) + f_c(u), masked; precision of R selectable.
int explicit_force(sdme_ctx *c, const sdme_material *mat, int prec_force, const double *u,
                   const double *f_ext, const sdme_contact *ct, double *f, double *R, float *u32,
                   float *R32, hipStream_t st) {
  int64_t N = 3 * c->Nn;
  int rc = clear_flag(c, st);
  if (rc) return rc;
  if (prec_force == SDME_FP32) {
    if (launch_convert<float, double>(u32, u, 1.0, N, st) || launch_fill<float>(R32, 0.0f, N, st) ||
        launch_force<float>(c->P, c->m32, mat->mu, mat->lam, u32, R32, nullptr, 0, st) ||
        launch_convert<double, float>(R, R32, 1.0, N, st))
      return SDME_EDEVICE;
  } else {
    if (launch_fill<double>(R, 0.0, N, st) ||
        launch_force<double>(c->P, c->m64, mat->mu, mat->lam, u, R, nullptr, 0, st))
      return SDME_EDEVICE;
  }
  if (f_ext) {
    if (launch_axpbypcz(f, 1.0, f_ext, 0.0, -1.0, R, N, st)) return SDME_EDEVICE;
  } else if (launch_axpbypcz(f, -1.0, R, 0.0, 0.0, nullptr, N, st)) {
    return SDME_EDEVICE;
  }
  if (ct && launch_face(c->P, c->m64, 1, 4, nullptr, 1.0, ct->eps, ct->z0, c->d.origin[2], u, f,
                        red_at(c, 11), 0, st))
    return SDME_EDEVICE;
  if (launch_bc<double>(f, 0, c->m64, st)) return SDME_EDEVICE;
  return read_flag(c, st);
}

struct ExWs {
  double *R, *f, *a, *t1, *t2, *t3;
  float *u32, *R32;
  LinWs lin;
};

bool plan_ex(sdme_ctx *c, void *ws, size_t bytes, ExWs &w) {
  int64_t N = 3 * c->Nn;
  Bump bp(ws, bytes);
  w.R = bp.get<double>(N);
  w.f = bp.get<double>(N);
  w.a = bp.get<double>(N);
  w.t1 = bp.get<double>(N);
  w.t2 = bp.get<double>(N);
  w.t3 = bp.get<double>(N);
  w.u32 = bp.get<float>(N);
  w.R32 = bp.get<float>(N);
  plan_lin(c, SDME_FP64, false, bp, w.lin);
  return bp.ok;
}

}  // namespace

extern "C" int sdme_explicit_step(sdme_ctx *c, const sdme_material *mat, int prec_force,
                                  const double *u_prev, const double *u_cur, double *u_next,
                                  const double *v0, const double *f_ext, double dt,
                                  const sdme_contact *ct, double mass_rtol, sdme_stats *stats,
                                  void *ws, size_t ws_bytes, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u_cur || !u_next || !valid_prec(prec_force) ||
      !(dt > 0) || !(mass_rtol > 0) || (!u_prev && !v0) || !(mat->rho > 0))
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  Range range("sdme_explicit_step");
  Timer tm;
  hipStream_t st = S(stream);
  ExWs w;
  if (!plan_ex(c, ws, ws_bytes, w)) return SDME_ENOMEM;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int64_t N = 3 * c->Nn;
  int rc = explicit_force(c, mat, prec_force, u_cur, f_ext, ct, w.f, w.R, w.u32, w.R32, st);
  if (!rc) {
    sdme_stats ms;
    std::memset(&ms, 0, sizeof(ms));
    rc = solve_linear(c, mat, SDME_FP64, nullptr, 0.0, true, w.f, w.a, mass_rtol, 100000, 1e-4,
                      w.lin, &ms, st);
    if (stats) stats->mass_iterations += ms.iterations;
  }
  if (!rc) {
    if (u_prev) {
      // u_next = 2 u_cur - u_prev + dt^2 a
      if (launch_axpbypcz(w.t1, 2.0, u_cur, 0.0, -1.0, u_prev, N, st) ||
          launch_axpbypcz(w.t1, dt * dt, w.a, 1.0, 0.0, nullptr, N, st) ||
          launch_convert<double, double>(u_next, w.t1, 1.0, N, st))
        rc = SDME_EDEVICE;
    } else {
      // start: u_next = u_cur + dt v0 + dt^2/2 a
      if (launch_axpbypcz(w.t1, 1.0, u_cur, 0.0, dt, v0, N, st) ||
          launch_axpbypcz(w.t1, 0.5 * dt * dt, w.a, 1.0, 0.0, nullptr, N, st) ||
          launch_convert<double, double>(u_next, w.t1, 1.0, N, st))
        rc = SDME_EDEVICE;
    }
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = SDME_EDEVICE;
  }
  if (stats) {
    stats->status = rc;
    stats->time_ms = tm.ms();
  }
  return rc;
}

extern "C" int sdme_energies(sdme_ctx *c, const sdme_material *mat, const double *u_prev,
                             const double *u_cur, const double *u_next, double dt,
                             const sdme_contact *ct, double out[3], void *ws, size_t ws_bytes,
                             void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u_prev || !u_cur || !u_next || !out || !(dt > 0))
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  ExWs w;
  if (!plan_ex(c, ws, ws_bytes, w)) return SDME_ENOMEM;
  int64_t N = 3 * c->Nn;
  // v = (u_next - u_prev) / (2 dt); KE = 1/2 v^T M v (fused element-local dot)
  if (launch_axpbypcz(w.t1, 0.5 / dt, u_next, 0.0, -0.5 / dt, u_prev, N, st) ||
      launch_fill<double>(w.t2, 0.0, N, st) ||
      launch_mass<double>(c->P, c->mm64, mat->rho, w.t1, w.t2, 0, red_at(c, 12), 1, nullptr, st) ||
      launch_fin2(red_at(c, 12), mass_blocks<double>(c->P, c->mm64), st))
    return SDME_EDEVICE;
  if (hipMemcpyAsync(c->h_res, c->results + 12, sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SDME_EDEVICE;
  out[0] = 0.5 * c->h_res[0];
  int rc = sdme_strain_energy(c, mat, u_cur, &out[1], stream);
  if (rc) return rc;
  out[2] = 0.0;
  if (ct) {
    if (launch_fill<double>(w.t3, 0.0, N, st)) return SDME_EDEVICE;
    rc = sdme_penalty_plane(c, ct, u_cur, w.t3, &out[2], stream);
  }
  return rc;
}

extern "C" int sdme_lambda_max(sdme_ctx *c, const sdme_material *mat, const double *u_lin,
                               const sdme_contact *ct, const double *x0, int iters,
                               double mass_rtol, double *lam_out, void *ws, size_t ws_bytes,
                               void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u_lin || !x0 || iters < 1 || !lam_out ||
      !(mass_rtol > 0))
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  hipStream_t st = S(stream);
  int64_t N = 3 * c->Nn;
  ExWs w;
  Bump bp(ws, ws_bytes);
  double *state = bp.get<double>(c->nqp * 10);
  if (!bp.ok || !plan_ex(c, (char *)ws + bp.off, ws_bytes - bp.off, w)) return SDME_ENOMEM;
  int rc = clear_flag(c, st);
  if (rc) return rc;
  if (launch_force<double>(c->P, c->m64, mat->mu, mat->lam, u_lin, nullptr, state, 0, st))
    return SDME_EDEVICE;
  if ((rc = read_flag(c, st))) return rc;
  double *x = w.t1, *y = w.t2, *mx = w.t3;
  if (launch_convert<double, double>(x, x0, 1.0, N, st) || launch_bc<double>(x, 0, c->m64, st))
    return SDME_EDEVICE;
  Reduce none{c->partials, c->counter, c->results + 8};
  double lam = 0;
  for (int it = 0; it < iters; it++) {
    // y = (K_T + K_c) x ; lam = x^T y / x^T M x
    if (launch_fill<double>(y, 0.0, N, st) ||
        launch_tangent<double>(c->P, c->m64, mat->mu, mat->lam, nullptr, state, 0.0, x, y, 1,
                               nullptr, nullptr, st))
      return SDME_EDEVICE;
    if (ct && launch_face(c->P, c->m64, 2, 4, nullptr, 1.0, ct->eps, 0, 0, x, y, red_at(c, 11), 0, st))
      return SDME_EDEVICE;
    if (launch_bc<double>(y, 0, c->m64, st) || launch_fill<double>(mx, 0.0, N, st) ||
        launch_mass<double>(c->P, c->mm64, mat->rho, x, mx, 1, none, 0, nullptr, st))
      return SDME_EDEVICE;
    double a[2], b[2];
    if ((rc = dot2<double>(c, x, y, N, a, st)) || (rc = dot2<double>(c, x, mx, N, b, st))) return rc;
    lam = a[0] / b[0];
    // x = M^-1 y normalised
    sdme_stats ms;
    std::memset(&ms, 0, sizeof(ms));
    rc = solve_linear(c, mat, SDME_FP64, nullptr, 0.0, true, y, w.a, mass_rtol, 100000, 1e-4,
                      w.lin, &ms, st);
    if (rc) return rc;
    if ((rc = dot2<double>(c, w.a, w.a, N, a, st))) return rc;
    if (!(a[1] > 0)) break;
    if (launch_axpbypcz(x, 1.0 / std::sqrt(a[1]), w.a, 0.0, 0.0, nullptr, N, st)) return SDME_EDEVICE;
  }
  *lam_out = lam;
  return SDME_OK;
}

extern "C" int sdme_explicit_adjoint_step(sdme_ctx *c, const sdme_material *mat, const double *u_n,
                                          const double *lam_next, const double *lam_next2,
                                          double *lam_out, double dt, int first, double mass_rtol,
                                          double *g_mu, double *g_lam, sdme_stats *stats,
                                          void *ws, size_t ws_bytes, void *stream) {
  if (!c || !mat || !mat->mu || !mat->lam || !u_n || !lam_next || !g_mu || !g_lam || !(dt > 0) ||
      !(mass_rtol > 0) || (!first && (!lam_next2 || !lam_out)))
    return SDME_EINVAL;
  if (int rc_ = ensure_device(c)) return rc_;
  Timer tm;
  hipStream_t st = S(stream);
  ExWs w;
  if (!plan_ex(c, ws, ws_bytes, w)) return SDME_ENOMEM;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int64_t N = 3 * c->Nn;
  sdme_stats ms;
  std::memset(&ms, 0, sizeof(ms));
  // w = M^-1 lam_next
  int rc = solve_linear(c, mat, SDME_FP64, nullptr, 0.0, true, lam_next, w.a, mass_rtol, 100000,
                        1e-4, w.lin, &ms, st);
  if (stats) stats->mass_iterations = ms.iterations;
  if (!rc) {
    double scale = first ? -0.5 * dt * dt : -dt * dt;
    if (launch_matgrad(c->P, c->m64, u_n, w.a, scale, g_mu, g_lam, st)) rc = SDME_EDEVICE;
  }
  if (!rc && !first) {
    Reduce none{c->partials, c->counter, c->results + 8};
    // t = K_T(u_n) w ; lam_out = 2 lam_next - dt^2 t - lam_next2
    if ((rc = clear_flag(c, st)) == SDME_OK) {
      if (launch_fill<double>(w.t1, 0.0, N, st) ||
          launch_tangent<double>(c->P, c->m64, mat->mu, mat->lam, u_n, nullptr, 0.0, w.a, w.t1, 1,
                                 nullptr, nullptr, st) ||
          launch_axpbypcz(w.t2, 2.0, lam_next, 0.0, -1.0, lam_next2, N, st) ||
          launch_axpbypcz(w.t2, -dt * dt, w.t1, 1.0, 0.0, nullptr, N, st) ||
          launch_bc<double>(w.t2, 0, c->m64, st) ||
          launch_convert<double, double>(lam_out, w.t2, 1.0, N, st))
        rc = SDME_EDEVICE;
      if (!rc) rc = read_flag(c, st);
    }
  }
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = SDME_EDEVICE;
  if (stats) {
    stats->status = rc;
    stats->time_ms = tm.ms();
  }
  return rc;
}
