/*
 * libsdme -- SDME high-order FEM hot path for AMD MI355X (gfx950).
 *
 * Element-by-element neo-Hookean internal force and tangent-stiffness action
 * on structured tensor-product hexahedra, evaluated at Gauss points with the
 * one-dimensional SDME bases of Dias, Suzuki, Valente & Bittencourt,
 * "Simulation of non-linear structural elastodynamic and impact problems using
 * minimum energy and simultaneous diagonalization high-order bases"
 * (arXiv 2104.13466), plus the Jacobi-preconditioned CG, static Newton,
 * Newmark-Newton and central-difference drivers built on them.
 *
 * Conventions (all entry points):
 *  - Plain C ABI.  Every function returns an int status (SDME_OK = 0 or a
 *    negative SDME_E* code); no exception or abort crosses the boundary.
 *    Arguments are validated on the host before any launch.
 *  - The caller owns all memory; the library allocates and frees no device
 *    or pinned memory.  "dev" pointers are device (HBM) pointers, "host"
 *    pointers host memory, both owned by the caller.  A context is a small
 *    host object (sdme_create / sdme_destroy); its device block (basis
 *    tables, reduction partials and solver scalars, O(number of elements)
 *    bytes) and host block (scalars the drivers read back) are allocated by
 *    the caller at the sizes sdme_context_bytes reports and attached with
 *    sdme_bind before the first call that touches the device.  Large scratch
 *    (solver vectors, linearisation state) is passed in by the caller as a
 *    workspace of at least sdme_workspace_bytes() bytes.
 *  - Vectors are structure-of-arrays [3][Nn]: component c of global slot g at
 *    index c*Nn + g.  The structured slot grid has Nd = nd*P+1 slots per
 *    direction, numbered x fastest: g = (iz*Ny + iy)*Nx + ix.  Element
 *    (ex,ey,ez) with local mode (a,b,c) (tensor indices of Eq.
 *    ProdTensorialHexaedro) owns slot (ex*P+a, ey*P+b, ez*P+c); element index
 *    e = (ez*ny + ey)*nx + ex, local index l = (c*(P+1) + b)*(P+1) + a.
 *  - prec selects the storage and arithmetic type of the vectors passed as
 *    void*: SDME_FP64 -> double, SDME_FP32 -> float.  Reductions (dot
 *    products, energies) always accumulate in double.
 *  - stream is a hipStream_t passed as void* (NULL = default stream).  Calls
 *    are asynchronous on that stream unless documented as synchronising
 *    (solvers and drivers read convergence scalars back and return after the
 *    solve; their stats are valid on return).  Calls on one context share
 *    its device block (reduction partials, solver scalars, status words and,
 *    with SDME_ASSEMBLY_ORDERED, the staging array): they must not overlap,
 *    i.e. issue them on one stream or order the streams; the host object is
 *    not thread-safe.
 *  - Dirichlet DOFs (faces/components set in sdme_mesh_desc.dirichlet) carry
 *    their prescribed values inside displacement vectors.  With
 *    SDME_MASK_BC, operators treat constrained DOFs of their input direction
 *    as zero and write zero to constrained outputs.
 */
#ifndef SDME_H
#define SDME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define SDME_OK 0
#define SDME_EINVAL (-1)      /* bad argument (checked before any launch)     */
#define SDME_ENOMEM (-2)      /* workspace too small / allocation failed      */
#define SDME_EDEVICE (-3)     /* HIP runtime error                            */
#define SDME_EEIG (-4)        /* basis eigensolve / factorisation failed      */
#define SDME_EJAC (-5)        /* det F <= 0 at a Gauss point                  */
#define SDME_ENOCONV (-6)     /* iteration limit reached before tolerance     */
#define SDME_EBREAKDOWN (-7)  /* CG breakdown: p^T A p <= 0                   */
#define SDME_ENAN (-8)        /* non-finite value in a residual or scalar     */

const char *sdme_status_string(int status);

/* ------------------------------------------------------------- 1D bases */
#define SDME_BASIS_NODAL 0   /* Lagrange on GLL points (Eq. lagrangian)           */
#define SDME_BASIS_MODAL 1   /* standard Jacobi(1,1) modal "ST" (Eq. BasePadrao1D) */
#define SDME_BASIS_SDME_M 2  /* SD + minimum energy in the L2 norm                */
#define SDME_BASIS_SDME_K 3  /* SD + minimum energy in the energy norm            */
#define SDME_BASIS_SDME_H 4  /* SD + minimum energy in the norm of K + lambda M   */

/*
 * sdme_basis_build -- construct a 1D basis of order P (Section 2) and tabulate
 * it at the Q Gauss-Legendre points.
 *   SD step (Eqs. diagMassa, L, diagL, Y, ParametroK) with parameter k in
 *   [0,1]; ME step (Eqs. ExtensaoMEmassa, alphaMassa, alphaRigidez, alphaKN)
 *   with lambda_h for SDME-H.  Internal modes are ordered by ascending
 *   eigenvalue Lambda_S and signed so that their derivative at xi = -1 is
 *   positive.  Slot order: 0 = left vertex mode, 1..P-1 internal, P = right
 *   vertex mode.
 * Outputs (host, row-major, any may be NULL):
 *   x[Q], w[Q]          Gauss points and weights on [-1,1]
 *   B[Q][P+1], D[Q][P+1] values and derivatives of the slots at x
 *   M1, K1 [(P+1)^2]    1D mass and stiffness in slot order
 *   lambda_s[P-1]       eigenvalues Lambda_S (SDME kinds; zeros otherwise)
 * Limits: 1 <= P <= 10, P+1 <= Q <= 16, 0 <= k <= 1, lambda_h >= 0.
 * Errors: SDME_EINVAL for limits, SDME_EEIG if an eigensolve or Cholesky
 * factorisation fails.
 */
int sdme_basis_build(int P, int Q, int kind, double k, double lambda_h, double *x, double *w,
                     double *B, double *D, double *M1, double *K1, double *lambda_s);

/* Evaluate the same basis at npts arbitrary points (host arrays
 * V[npts][P+1], dV[npts][P+1]; dV may be NULL). */
int sdme_basis_eval(int P, int kind, double k, double lambda_h, int npts, const double *pts,
                    double *V, double *dV);

/* ------------------------------------------------------------ mesh/context */
typedef struct sdme_ctx sdme_ctx;

typedef struct {
  int nx, ny, nz;     /* hexahedra per direction (>= 1)                       */
  int P;              /* polynomial order, 1..8                               */
  int Q;              /* volume points per direction: P+2 (Gauss-Legendre) or  */
                      /* P+1 (Gauss-Lobatto-Legendre; with the nodal basis    */
                      /* collocated: diagonal mass)                           */
  int basis;          /* SDME_BASIS_*                                          */
  double k;           /* SD parameter k (Eq. Y), paper value 0.5               */
  double lambda_h;    /* SDME-H parameter lambda (Eq. EffectiveStiffness_lambda), paper 100 */
  double h[3];        /* element edge lengths (affine boxes)                   */
  double origin[3];   /* coordinates of the box corner                         */
  uint32_t dirichlet; /* bit (face*3 + comp): faces 0 x=0, 1 x=max, 2 y=0, 3 y=max, 4 z=0, 5 z=max */
  int mass_rule;      /* 0: the mass with the volume rule (consistent);        */
                      /* 1: the mass with the Gauss-Lobatto-Legendre rule of   */
                      /* P+1 points (diagonal for the nodal basis: the          */
                      /* Lagrange diagonal-mass variant of Section 5.2), used by */
                      /* sdme_mass_apply, mass solves, explicit steps, energies */
                      /* and sdme_lambda_max; the mass-shifted operators        */
                      /* (mass_shift != 0, Newmark) then return SDME_EINVAL     */
  int assembly;       /* SDME_ASSEMBLY_ATOMIC: element contributions to shared  */
                      /* slots are added with hardware atomics (the order of    */
                      /* the additions, and so the last bits of the sums, may   */
                      /* differ between runs); SDME_ASSEMBLY_ORDERED: they are  */
                      /* staged and added in ascending element order (the       */
                      /* assembly over elements of Section 2), so every result, */
                      /* PCG and Newton iterates included, repeats bit for bit; */
                      /* the device block then also holds the staging array     */
} sdme_mesh_desc;

#define SDME_ASSEMBLY_ATOMIC 0
#define SDME_ASSEMBLY_ORDERED 1

/* Create a context for a structured box mesh (host only).  The basis is
 * built on the host (sdme_basis_build) at once; its tables are uploaded to
 * the caller's device block by sdme_bind (host-only queries such as
 * sdme_sizes and sdme_gather_indices need no binding).  Meshes need
 * 3*Nn < 2^31.  Errors: SDME_EINVAL, SDME_EEIG. */
int sdme_create(const sdme_mesh_desc *desc, sdme_ctx **out);
/* Releases the host object only: the caller frees the blocks it bound, once
 * the work it queued on them has completed. */
int sdme_destroy(sdme_ctx *ctx);

/* Sizes of the memory a context needs from the caller: *dev_bytes of device
 * memory (basis tables of the volume and mass rules in FP64 and FP32, the
 * Jacobian flag, PCG scalars, per-block reduction partials and, with
 * SDME_ASSEMBLY_ORDERED, the staging array: the larger of the element
 * kernels' output tiles and 3 (P+1)^3 words per element, in FP64) and *host_bytes
 * of host memory (solver scalars copied back by the drivers).  Host-only.
 * Errors: SDME_EINVAL. */
int sdme_context_bytes(const sdme_ctx *ctx, size_t *dev_bytes, size_t *host_bytes);

/* Attach caller-owned memory to a context and upload its basis tables:
 * dev_block (device, at least dev_bytes, 256-byte aligned) is zero-filled by
 * a kernel and the tables are copied into it with hipMemcpyAsync, both on
 * stream; host_block (host, at least host_bytes, 8-byte aligned; pinned
 * memory keeps the drivers' read-backs asynchronous copies) is cleared at
 * once.  The context keeps both pointers (it does not own them) until it is
 * destroyed or bound again.  Every entry point that touches the device returns
 * SDME_EINVAL on a context that was never bound.  Errors: SDME_EINVAL (sizes,
 * alignment, NULL), SDME_EDEVICE. */
int sdme_bind(sdme_ctx *ctx, void *dev_block, size_t dev_bytes, void *host_block,
              size_t host_bytes, void *stream);

/* The element named by the last SDME_EJAC: the smallest index of an element
 * with det F <= 0 at a Gauss point in the last call that checked the
 * Jacobian (SDME_CHECK_JAC, the Newton drivers), or -1 when that call found
 * none.  Host-only; element index e = (ez ny + ey) nx + ex.  Errors:
 * SDME_EINVAL (NULL). */
int sdme_jac_element(const sdme_ctx *ctx, int64_t *element);

/* out[0] = Nn (slots per component), out[1] = E (elements),
 * out[2] = Gauss points (E*Q^3), out[3] = words of linearisation state per
 * Gauss point (10: F^-1 and mu - lambda ln J). */
int sdme_sizes(const sdme_ctx *ctx, int64_t out[4]);

/* Element-to-global map: host_out[e*(P+1)^3 + l] = global slot (Eq.
 * ProdTensorialHexaedro indices; topological association of Section 2). */
int sdme_gather_indices(const sdme_ctx *ctx, int32_t *host_out);

/* host_out[c*Nn + g] = 1 if DOF (c,g) is constrained, else 0. */
int sdme_dirichlet_flags(const sdme_ctx *ctx, uint8_t *host_out);

/* Coefficients of the affine field u(X) = a + G X (G row-major 3x3) in the
 * tensor-product basis, written to host_out[3*Nn] (the expansion is exact: the
 * 1D expansions of 1 and xi, combined per element with X = Xc + (h/2) xi). */
int sdme_affine_field(const sdme_ctx *ctx, const double a[3], const double G[9],
                      double *host_out);

/* --------------------------------------------------------------- operators */
#define SDME_FP64 0
#define SDME_FP32 1

#define SDME_MASK_BC 1   /* zero constrained inputs (direction) and outputs   */
#define SDME_CHECK_JAC 2 /* synchronise and return SDME_EJAC if det F <= 0    */

/* Per-element Lame parameters (device, double[E]) and density. */
typedef struct {
  const double *mu;
  const double *lam;
  double rho;
} sdme_material;

/*
 * sdme_internal_force -- R(u) = sum_e sum_q w_q detJ P(F) : grad N
 * (second term of Eq. material virtual work; compressible neo-Hookean,
 * Eq. hyperelastic strain energy / second Piola-Kirchhoff relation, with
 * P = F S).  u, R: dev [3][Nn] of type prec; R is overwritten.
 * state (dev, nullable): if given, the linearisation state of u is written,
 * layout [E][10][Q^3] of type prec (F^-1 row-major, then mu - lambda ln J).
 * flags: SDME_MASK_BC masks R on constrained DOFs (u is never masked);
 * SDME_CHECK_JAC synchronises and reports det F <= 0.
 */
int sdme_internal_force(sdme_ctx *ctx, const sdme_material *mat, int prec, const void *u,
                        void *R, void *state, int flags, void *stream);

/* Write only the linearisation state of u (see sdme_internal_force). */
int sdme_linearize(sdme_ctx *ctx, const sdme_material *mat, int prec, const void *u,
                   void *state, int flags, void *stream);

/*
 * sdme_tangent_apply -- y = (K_T(u_lin) + mass_shift * M) v, K_T the
 * derivative of R (linearisation, Eq. directional derivative / effective
 * stiffness) and M the consistent mass rho int N N (so mass_shift = b1 gives
 * the Newmark matrix b1 M + K_T).  Exactly one of u_lin (recompute F at every
 * Gauss point) and state (stored linearisation from sdme_linearize) is
 * non-NULL.  v, y: dev [3][Nn] of type prec; y is overwritten.
 */
int sdme_tangent_apply(sdme_ctx *ctx, const sdme_material *mat, int prec, const void *u_lin,
                       const void *state, double mass_shift, const void *v, void *y, int flags,
                       void *stream);

/* y = rho M v (consistent mass, inertia term of Eq. material virtual work). */
int sdme_mass_apply(sdme_ctx *ctx, double rho, int prec, const void *v, void *y, int flags,
                    void *stream);

/* d = diag(K_T + mass_shift M) from a stored linearisation state (Jacobi
 * preconditioner of the element-by-element diagonal PCG, Section 5).  With
 * SDME_MASK_BC constrained entries are set to 1. */
int sdme_jacobi_diag(sdme_ctx *ctx, const sdme_material *mat, int prec, const void *state,
                     double mass_shift, void *d, int flags, void *stream);

/* Strain energy sum_e sum_q w_q detJ Psi(F(u)) -> *host_out (synchronises). */
int sdme_strain_energy(sdme_ctx *ctx, const sdme_material *mat, const double *u,
                       double *host_out, void *stream);

/* Dead traction t (reference configuration) on a box face: f += scale *
 * int_face N t dA, surface Gauss rule with P+1 points per direction.  f: dev
 * double [3][Nn], accumulated. */
int sdme_face_traction(sdme_ctx *ctx, int face, const double t[3], double scale, double *f,
                       void *stream);

/* Rigid plane z = z0 (normal +z) below face z=0: gap g = Z + u_z - z0 at the
 * face Gauss points (P+1 per direction, the paper's contact rule), penalty
 * force f_z += int N eps max(-g,0) dA (accumulated into f).  If energy_host is
 * non-NULL the penalty energy 1/2 eps int min(g,0)^2 dA is returned there
 * (synchronises). */
typedef struct {
  double eps; /* penalty per unit area */
  double z0;  /* plane height          */
} sdme_contact;

int sdme_penalty_plane(sdme_ctx *ctx, const sdme_contact *c, const double *u, double *f,
                       double *energy_host, void *stream);

/* ------------------------------------------- loads given at quadrature points
 * For the fabricated-solution problems of Section 5 (body force and boundary
 * tractions computed from a prescribed displacement field; their work enters
 * the virtual-work statement of Section 3 with the reference-configuration
 * volume and face measures).
 *
 * sdme_quadrature_points -- physical coordinates of the quadrature points,
 * written to host_out (host double, no device access): face = -1: the volume
 * Gauss points, [3][E][Q^3] with q = q1 + Q (q2 + Q q3) and element
 * e = (ez ny + ey) nx + ex; face = 0..5: the face Gauss points of the face
 * rule (P+1 points per direction), [3][nfe][(P+1)^2] with face element
 * fe = j ne1 + i and point p = pj (P+1) + pi, where (i, pi) run along the
 * face's first tangential direction (y for faces 0, 1; x otherwise) and
 * (j, pj) along the second (z for faces 0..3; y for faces 4, 5); nfe =
 * ne1 * ne2.  Errors: SDME_EINVAL. */
int sdme_quadrature_points(const sdme_ctx *ctx, int face, double *host_out);

/* sdme_body_load -- f += sum_e sum_q w_q detJ N_a(X_q) b(X_q) for every slot
 * a: b dev double [3][E][Q^3] (body force per unit reference volume at the
 * volume Gauss points, layout of sdme_quadrature_points), f dev double
 * [3][Nn], accumulated (atomics; not masked).  Errors: SDME_EINVAL. */
int sdme_body_load(sdme_ctx *ctx, const double *b, double *f, void *stream);

/* sdme_face_load -- f += int_face N_a t dA with t dev double [3][nfe][(P+1)^2]
 * (traction per unit reference area at the face Gauss points, layout of
 * sdme_quadrature_points).  Accumulated, not masked.  Errors: SDME_EINVAL. */
int sdme_face_load(sdme_ctx *ctx, int face, const double *t, double *f, void *stream);

/* sdme_l2_error -- host_out[c] = ( sum_e sum_q w_q detJ (u_h,c(X_q) -
 * g_c(X_q))^2 )^(1/2) for c = 0, 1, 2: the L2 norm over the box of the
 * difference between the field with coefficients u (dev double [3][Nn]) and
 * the values g (dev double [3][E][Q^3] at the volume quadrature points), by
 * the volume rule of the mesh (Q points per direction).  Deterministic (block
 * partials summed in block order).  Synchronises.  Errors: SDME_EINVAL,
 * SDME_EDEVICE. */
int sdme_l2_error(sdme_ctx *ctx, const double *u, const double *g, double *host_out,
                  void *stream);

/* Sensitivity of R to the element Lame parameters contracted with w:
 * g_mu[e] += scale * sum_q w_q detJ (F - F^-T) : grad w,
 * g_lam[e] += scale * sum_q w_q detJ lnJ F^-T : grad w  (dev double[E]). */
int sdme_material_grad_accumulate(sdme_ctx *ctx, const double *u, const double *w, double scale,
                                  double *g_mu, double *g_lam, void *stream);

/* ----------------------------------------------------------------- solvers */
typedef struct {
  int status;         /* SDME_OK or error                                     */
  int iterations;     /* PCG iterations (all inner iterations in mixed mode)  */
  int outer;          /* FP64 defect-correction sweeps (mixed mode)           */
  int newton;         /* Newton iterations                                    */
  int mass_iterations;/* PCG iterations of mass solves (explicit, adjoint)    */
  int halvings;       /* Newton increments halved because the updated state   */
                      /* inverted an element (damped Newton)                  */
  double rel_residual;/* final ||b - A x|| / ||b|| (FP64)                      */
  double newton_rel;  /* final ||psi|| / ||psi_0||                             */
  double time_ms;     /* wall time of the call                                */
} sdme_stats;

#define SDME_OP_PCG 0
#define SDME_OP_NEWTON 1
#define SDME_OP_NEWMARK 2
#define SDME_OP_EXPLICIT 3
#define SDME_OP_ADJOINT 4
#define SDME_OP_CONDENSED 5

/* Workspace bytes needed by a solver/driver entry point with the given prec
 * (SDME_FP64 or SDME_FP32 = mixed FP32 inner / FP64 outer). */
int sdme_workspace_bytes(const sdme_ctx *ctx, int op, int prec, size_t *bytes);

/*
 * sdme_jacobi_pcg -- solve (K_T(u_lin) + mass_shift M) x = b on the free DOFs
 * by conjugate gradients with the diagonal preconditioner (the paper's CGD /
 * element-by-element diagonal PCG, Section 5).  b, x: dev double [3][Nn]
 * (x overwritten, zero on constrained DOFs; b masked internally).  Stops when
 * ||b - A x||_2 <= rtol ||b||_2.
 * prec = SDME_FP64: FP64 vectors, state and operator.
 * prec = SDME_FP32: mixed precision -- the CG iteration runs in FP32 (FP32
 * state, operator and vectors, FP64 dots) while the solution is accumulated
 * in FP64; each time the FP32 residual has dropped by the factor inner_rtol
 * (and when it reaches rtol) it is replaced by the FP64 defect
 * r = b - A x computed with the FP64 operator, keeping the search direction
 * (residual replacement / reliable updates).  The stop test uses the FP64
 * defect.  stats->outer counts the replacements; the drivers use 1e-2.
 * mass_only != 0 solves with the mass matrix alone (K_T omitted, u_lin unused).
 * Synchronises.  Errors: SDME_ENOCONV (maxit), SDME_EBREAKDOWN, SDME_EJAC,
 * SDME_ENOMEM (ws_bytes too small).
 */
int sdme_jacobi_pcg(sdme_ctx *ctx, const sdme_material *mat, int prec, const double *u_lin,
                    double mass_shift, int mass_only, const double *b, double *x, double rtol,
                    int maxit, double inner_rtol, sdme_stats *stats, void *ws, size_t ws_bytes,
                    void *stream);

/*
 * Static condensation of the element-interior modes (Section 4, Eqs.
 * Eq:Matrix_form_schur1, Schur_split1, Schur_split2 and
 * Eq:Newmark_Matrix_form_schur1; Section 5.2 counts the remaining DOFs).
 * An interior mode has all three tensor indices internal; it belongs to one
 * element, so the interior unknowns of A x = b (A = K_T + mass_shift M, or
 * the mass alone) are eliminated element by element:
 *   S x_B = g,  S = A_BB - sum_e A_BI inv(A_II) A_IB,  g = b_B - A_BI inv(A_II) b_I,
 *   x_I = inv(A_II) (b_I - A_IB x_B).
 *
 * sdme_condensed_sizes -- host only: out[0] = free DOFs of the condensed
 * system (not interior, not constrained), out[1] = interior DOFs
 * (3 E (P-1)^3), out[2] = interior block size per element (3 (P-1)^3).
 */
int sdme_condensed_sizes(const sdme_ctx *ctx, int64_t out[3]);

/*
 * sdme_condensed_pcg -- solve A x = b (as sdme_jacobi_pcg, FP64) through the
 * condensed system: the interior blocks A_II of every element are formed from
 * the linearisation at u_lin at the Gauss points and inverted (dense, batched,
 * workspace E (3 (P-1)^3)^2 doubles), S is applied matrix-free (two operator
 * actions and one interior solve per iteration) and solved by CG with the
 * diagonal of A on the remaining DOFs as preconditioner (it omits the Schur
 * correction of the diagonal), then the interior modes are recovered.  Stops
 * when ||g - S x_B||_2 <= rtol ||g||_2.  x: dev double [3][Nn], overwritten.
 * Workspace: sdme_workspace_bytes(ctx, SDME_OP_CONDENSED, SDME_FP64).
 * Requires the consistent mass (mass_rule 0).  stats->iterations counts the
 * condensed CG iterations.  Synchronises.  Errors: SDME_EINVAL, SDME_ENOMEM,
 * SDME_EJAC, SDME_EBREAKDOWN (an interior block or S not positive definite),
 * SDME_ENOCONV, SDME_EDEVICE.
 */
int sdme_condensed_pcg(sdme_ctx *ctx, const sdme_material *mat, const double *u_lin,
                       double mass_shift, int mass_only, const double *b, double *x, double rtol,
                       int maxit, sdme_stats *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * sdme_jacobi_pcg_noalloc -- sdme_jacobi_pcg with the workspace taken from a
 * device-resident scratch array of SDME_NOALLOC_SCRATCH_BYTES bytes inside
 * the library (one per device, held until the process ends) instead of a
 * caller buffer: for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * The call allocates nothing; the context must be bound (sdme_bind).
 * Arguments, results and errors as sdme_jacobi_pcg, plus SDME_ENOMEM when the
 * solve needs more than SDME_NOALLOC_SCRATCH_BYTES
 * (sdme_workspace_bytes(ctx, SDME_OP_PCG, prec) tells beforehand; the 32 MiB
 * hold, at P = 4, about 2.5e5 DOF in FP64 and 1.6e5 DOF in mixed precision).  All calls on one device
 * share that device's array: calls that overlap in time on one device (from
 * several host threads or streams) race and must not be made.
 */
#define SDME_NOALLOC_SCRATCH_BYTES (32u << 20)
int sdme_jacobi_pcg_noalloc(sdme_ctx *ctx, const sdme_material *mat, int prec,
                            const double *u_lin, double mass_shift, int mass_only,
                            const double *b, double *x, double rtol, int maxit, double inner_rtol,
                            sdme_stats *stats, void *stream);

/*
 * sdme_newton_static -- Newton-Raphson for R(u) = f_ext (Section 3, the
 * linearised virtual work with the effective stiffness K_T), f_ext nullable
 * (= 0): K_T(u) du = psi = f_ext - R(u) by sdme_jacobi_pcg (inner_rtol 1e-2
 * when prec = SDME_FP32), u += du, until ||psi||_2 <= newton_rtol ||psi_0||_2.
 * u: dev double [3][Nn], in/out (prescribed values on constrained DOFs are
 * kept).  If an update inverts an element (det F <= 0) the increment is halved
 * (up to 20 times).  If PCG meets non-positive curvature (K_T not positive
 * definite at an iterate) after at least one iteration, the CG iterate reached
 * so far is taken as du (truncated Newton-CG).  Synchronises.  Errors:
 * SDME_ENOCONV (max_newton or max_pcg), SDME_EJAC, SDME_EBREAKDOWN (at the
 * first PCG iteration), SDME_ENOMEM.
 */
int sdme_newton_static(sdme_ctx *ctx, const sdme_material *mat, int prec, double *u,
                       const double *f_ext, double newton_rtol, double pcg_rtol, int max_newton,
                       int max_pcg, sdme_stats *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * sdme_newmark_newton_step -- one Newmark step (Section 4, implicit time
 * integration) with Newton iterations:
 *   psi = P_{n+1} - R(u) - M (b1 (u - u_n) - b2 v_n - b3 a_n),
 *   (b1 M + K_T) du = psi,  b1 = 1/(beta dt^2), b2 = 1/(beta dt),
 *   b3 = 1/(2 beta) - 1;  then a_{n+1} = b1 (u - u_n) - b2 v_n - b3 a_n,
 *   v_{n+1} = v_n + dt ((1-gamma) a_n + gamma a_{n+1}).
 * u, v, a: dev double [3][Nn], in (step n) / out (step n+1).  f_next
 * nullable.  Predictor u = u_n; damping and truncation as in
 * sdme_newton_static.  Synchronises.
 */
int sdme_newmark_newton_step(sdme_ctx *ctx, const sdme_material *mat, int prec, double *u,
                             double *v, double *a, const double *f_next, double dt, double beta,
                             double gamma, double newton_rtol, double pcg_rtol, int max_newton,
                             int max_pcg, sdme_stats *stats, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * sdme_explicit_step -- central difference (Section 4, explicit time
 * integration, Eq. Motion_explicit2): u_next = 2 u_cur - u_prev + dt^2 a with
 * M a = P - R(u_cur) + f_c(u_cur) solved by Jacobi-PCG on the mass matrix to
 * mass_rtol (f_ext and contact nullable).  prec_force selects the precision
 * of the internal-force evaluation (the update and mass solve are FP64).
 * If u_prev == NULL the start step is taken: u_next = u_cur + dt v0 +
 * dt^2/2 a_0 with v0 passed in place of u_prev through v0_if_start.
 * Synchronises (mass solve).
 */
int sdme_explicit_step(sdme_ctx *ctx, const sdme_material *mat, int prec_force,
                       const double *u_prev, const double *u_cur, double *u_next,
                       const double *v0_if_start, const double *f_ext, double dt,
                       const sdme_contact *contact, double mass_rtol, sdme_stats *stats, void *ws,
                       size_t ws_bytes, void *stream);

/* Energies at step n: out[0] = 1/2 v^T M v with v = (u_next - u_prev)/(2 dt),
 * out[1] = strain energy of u_cur, out[2] = penalty energy (0 without
 * contact).  Synchronises. */
int sdme_energies(sdme_ctx *ctx, const sdme_material *mat, const double *u_prev,
                  const double *u_cur, const double *u_next, double dt,
                  const sdme_contact *contact, double out_host[3], void *ws, size_t ws_bytes,
                  void *stream);

/* Largest eigenvalue of M^-1 (K_T(u_lin) + K_c) by power iteration from the
 * caller's start vector x0 (dev double [3][Nn]); K_c is the penalty
 * stiffness eps int N_z N_z dA on face z=0 when contact != NULL (all face
 * points taken as active).  Used for the CFL step dt = cfl * 2 / sqrt(lambda).
 * Synchronises. */
int sdme_lambda_max(sdme_ctx *ctx, const sdme_material *mat, const double *u_lin,
                    const sdme_contact *contact, const double *x0, int iters, double mass_rtol,
                    double *lambda_host, void *ws, size_t ws_bytes, void *stream);

/*
 * sdme_explicit_adjoint_step -- one step of the discrete adjoint of the
 * unloaded central-difference rollout (no contact) for J = 1/2 ||u_K - u*||^2:
 *   w = M^-1 lam_next;
 *   g_mu, g_lam += scale * dR(u_n)/d(mu, lam)^T w, scale = -dt^2 (n >= 1) or
 *   -dt^2/2 (n = 0, first != 0);
 *   if !first: lam_out = 2 lam_next - dt^2 K_T(u_n) w - lam_next2.
 * All vectors dev double [3][Nn]; g_mu, g_lam dev double [E].  Synchronises.
 */
int sdme_explicit_adjoint_step(sdme_ctx *ctx, const sdme_material *mat, const double *u_n,
                               const double *lam_next, const double *lam_next2, double *lam_out,
                               double dt, int first, double mass_rtol, double *g_mu,
                               double *g_lam, sdme_stats *stats, void *ws, size_t ws_bytes,
                               void *stream);

/* Per-launch timing of the PCG operator (the tangent or mass action inside
 * sdme_jacobi_pcg and the drivers), by HIP events recorded on the solve stream
 * around each operator launch that runs.  Returns in ms_out/count_out the
 * totals accumulated since the previous call ([0] FP64 operator, [1] FP32
 * operator; either may be NULL), then resets them and switches recording on
 * (enable != 0) or off.  Host-only bookkeeping; events are created on first
 * enable. */
int sdme_profile(sdme_ctx *ctx, int enable, double ms_out[2], int64_t count_out[2]);

/* lam_out = mask (u - target); *J_host = 1/2 ||lam_out||^2 (synchronises). */
int sdme_misfit(sdme_ctx *ctx, const double *u, const double *target, double *lam_out,
                double *J_host, void *stream);

/* y = alpha x + beta y on dev double [n] (vector update used by drivers). */
int sdme_axpby(sdme_ctx *ctx, int64_t n, double alpha, const double *x, double beta, double *y,
               void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SDME_H */
