"""ORACLE -- test infrastructure only.

Fabricated-solution loads and errors (Section 5), as plain definitions:
* quadrature points of the volume rule (Q per direction) and of the face rule
  (P+1 per direction) on a structured box;
* the body force b = -Div P(F(u*)) of a prescribed field u*, by fourth-order
  central differences: F = I + grad u* from differences of u*, the first
  Piola-Kirchhoff stress P = F S with S = mu (I - C^-1) + lambda ln J C^-1
  (the neo-Hookean law of Section 3), and Div P from differences of P;
* the traction t = P N on a face with outward normal N;
* the consistent loads f_a = sum_e sum_q w_q detJ N_a(X_q) b(X_q) and
  f_a = sum_face-elements sum_p w_p dA N_a(X_p) t(X_p), element by element with
  the full tensor-product shape functions (no sum factorisation);
* the L2 error (sum_e sum_q w_q detJ (u_h(X_q) - g(X_q))^2)^(1/2) per component.
The static example of Section 5.1 (u* = (1.9 sin x - x, 0, 0), unit cube,
E = 1000, nu = 0.3, x = 0 clamped, tractions of u* on the other faces) is
solved with the oracle's Newton-Raphson and Jacobi PCG.
"""
import numpy as np

from . import basis as ob
from . import fem
from . import solvers as osv


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


# --------------------------------------------------------------- points
def volume_points(mesh, origin=(0.0, 0.0, 0.0)):
    """(3, E, Q^3): Gauss point q = q1 + Q (q2 + Q q3) of element
    e = (ez ny + ey) nx + ex at X_d = origin_d + h_d (e_d + (1 + x_{q_d}) / 2)."""
    Q = mesh.Q
    x, _ = ob.volume_rule(mesh.P, Q)
    out = np.zeros((3, mesh.E, Q ** 3))
    for e in range(mesh.E):
        ei = (e % mesh.nx, (e // mesh.nx) % mesh.ny, e // (mesh.nx * mesh.ny))
        for q3 in range(Q):
            for q2 in range(Q):
                for q1 in range(Q):
                    q = q1 + Q * (q2 + Q * q3)
                    qi = (q1, q2, q3)
                    for d in range(3):
                        out[d, e, q] = origin[d] + mesh.h[d] * (ei[d] + 0.5 * (1 + x[qi[d]]))
    return out


def _face_dirs(face):
    d = face // 2
    t1, t2 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
    return d, face % 2, t1, t2


def face_points(mesh, face, origin=(0.0, 0.0, 0.0)):
    """(3, nfe, (P+1)^2): face element fe = j ne[t1] + i, point p = pj nq + pi,
    (i, pi) along the first tangential direction t1, (j, pj) along t2."""
    d, side, t1, t2 = _face_dirs(face)
    ne = (mesh.nx, mesh.ny, mesh.nz)
    nq = mesh.P + 1
    x, _ = ob.gauss_legendre(nq)
    nfe = ne[t1] * ne[t2]
    out = np.zeros((3, nfe, nq * nq))
    for fe in range(nfe):
        i, j = fe % ne[t1], fe // ne[t1]
        for pj in range(nq):
            for pi in range(nq):
                p = pj * nq + pi
                out[d, fe, p] = origin[d] + (ne[d] * mesh.h[d] if side else 0.0)
                out[t1, fe, p] = origin[t1] + mesh.h[t1] * (i + 0.5 * (1 + x[pi]))
                out[t2, fe, p] = origin[t2] + mesh.h[t2] * (j + 0.5 * (1 + x[pj]))
    return out


# ------------------------------------------------------------ mechanics
def piola(F, lam, mu):
    """First Piola-Kirchhoff stress of the neo-Hookean law, F (..., 3, 3)."""
    C = np.swapaxes(F, -1, -2) @ F
    Ci = np.linalg.inv(C)
    lnJ = np.log(np.linalg.det(F))
    S = mu * (np.eye(3) - Ci) + lam * lnJ[..., None, None] * Ci
    return F @ S


_D4 = ((-2, 1.0 / 12), (-1, -8.0 / 12), (1, 8.0 / 12), (2, -1.0 / 12))  # f' ~ sum c f(x + k d) / d


def deformation_gradient(ufun, X, delta=1e-3):
    """F = I + grad u at points X (3, N), fourth-order central differences."""
    N = X.shape[1]
    F = np.tile(np.eye(3), (N, 1, 1))
    for J in range(3):
        for k, c in _D4:
            Xs = X.copy()
            Xs[J] += k * delta
            F[:, :, J] += c * ufun(Xs).T / delta
    return F


def body_force(ufun, X, lam, mu, delta=1e-3):
    """b = -Div P(F(u*)) at points X (3, N)."""
    b = np.zeros_like(X)
    for J in range(3):
        for k, c in _D4:
            Xs = X.copy()
            Xs[J] += k * delta
            Pk = piola(deformation_gradient(ufun, Xs, delta), lam, mu)
            b -= c * Pk[:, :, J].T / delta
    return b


def traction(ufun, face, X, lam, mu, delta=1e-3):
    """t = P N at points X (3, N) of face `face` (outward normal N)."""
    d, side = face // 2, face % 2
    N = np.zeros(3)
    N[d] = 1.0 if side else -1.0
    P = piola(deformation_gradient(ufun, X, delta), lam, mu)
    return (P @ N).T


# ---------------------------------------------------------------- loads
def _tensor_shape(B1, B2, B3):
    """N[(q1,q2,q3) flattened with q1 fastest, (a,b,c) with a fastest]."""
    return np.einsum("ia,jb,kc->kjicba", B1, B2, B3).reshape(
        B1.shape[0] * B2.shape[0] * B3.shape[0], -1)


def body_load(mesh, b):
    """f (3 Nn) with f_a,i = sum_e sum_q w_q detJ N_a(X_q) b_i(X_q); b (3, E, Q^3)."""
    gm = mesh.gather_map()
    Nsh = _tensor_shape(mesh.B, mesh.B, mesh.B)
    wq = np.einsum("i,j,k->kji", mesh.w, mesh.w, mesh.w).reshape(-1) * np.prod(mesh.h) / 8
    f = np.zeros((3, mesh.Nn))
    for e in range(mesh.E):
        for i in range(3):
            np.add.at(f[i], gm[e], Nsh.T @ (wq * b[i, e]))
    return f.reshape(-1)


def face_load(mesh, face, Bf, t):
    """f (3 Nn) with f_a,i = sum over face elements and face Gauss points of
    w_pi w_pj dA N_a t_i; Bf[p][s] the 1D basis at the P+1 face Gauss points,
    t (3, nfe, (P+1)^2)."""
    d, side, t1, t2 = _face_dirs(face)
    ne = (mesh.nx, mesh.ny, mesh.nz)
    P, n = mesh.P, mesh.P + 1
    xf, wf = ob.gauss_legendre(n)
    dA = mesh.h[t1] * mesh.h[t2] / 4
    N2 = np.einsum("ia,jb->jiba", Bf, Bf).reshape(n * n, n * n)  # [p=(pj,pi)][(b,a)]
    w2 = np.einsum("i,j->ji", wf, wf).reshape(-1) * dA
    f = np.zeros((3, mesh.Nz, mesh.Ny, mesh.Nx))
    for fe in range(ne[t1] * ne[t2]):
        i, j = fe % ne[t1], fe // ne[t1]
        for k in range(3):
            val = (N2.T @ (w2 * t[k, fe])).reshape(n, n)  # [b][a]
            for bb in range(n):
                for a in range(n):
                    s = [0, 0, 0]
                    s[t1] = i * P + a
                    s[t2] = j * P + bb
                    s[d] = (ne[d] * P) if side else 0
                    f[k, s[2], s[1], s[0]] += val[bb, a]
    return f.reshape(-1)


def l2_error(mesh, u, g):
    """(sum_e sum_q w_q detJ (u_h,c(X_q) - g_c(X_q))^2)^(1/2), c = 0, 1, 2."""
    gm = mesh.gather_map()
    Nsh = _tensor_shape(mesh.B, mesh.B, mesh.B)
    wq = np.einsum("i,j,k->kji", mesh.w, mesh.w, mesh.w).reshape(-1) * np.prod(mesh.h) / 8
    U = u.reshape(3, -1)
    err = np.zeros(3)
    for e in range(mesh.E):
        for c in range(3):
            d = Nsh @ U[c, gm[e]] - g[c, e]
            err[c] += wq @ (d * d)
    return np.sqrt(err)


# ------------------------------------------------- static example (Sec. 5.1)
E_STATIC, NU_STATIC = 1000.0, 0.3


def static_field(X):
    out = np.zeros_like(X)
    out[0] = 1.9 * np.sin(X[0]) - X[0]
    return out


def static_mesh(P, kind, n=2, Q=None):
    """(mesh, face table Bf) of the unit cube with n^3 hexahedra (volume rule
    of Q points per direction, default P + 2)."""
    Q = P + 2 if Q is None else Q
    b, x, w, B, D = ob.build(P, Q, kind)
    m = fem.Mesh(n, n, n, P, Q, np.full(3, 1.0 / n), B, D, w)
    xf, _ = ob.gauss_legendre(P + 1)
    Bf, _ = b.eval(xf)
    return m, Bf


def static_loads(mesh, Bf):
    lam, mu = lame(E_STATIC, NU_STATIC)
    Xv = volume_points(mesh)
    bv = np.stack([body_force(static_field, Xv[:, e], lam, mu) for e in range(mesh.E)], axis=1)
    f = body_load(mesh, bv)
    for face in range(1, 6):
        Xf = face_points(mesh, face)
        tf = np.stack([traction(static_field, face, Xf[:, k], lam, mu)
                       for k in range(Xf.shape[1])], axis=1)
        f += face_load(mesh, face, Bf, tf)
    return f


def static_solve(P, kind, pcg_rtol=1e-10, max_pcg=5000):
    """Newton-Raphson to 1e-8 from u = 0 with x = 0 clamped; returns (u, hist,
    L2 errors per component)."""
    mesh, Bf = static_mesh(P, kind)
    lam, mu = lame(E_STATIC, NU_STATIC)
    mask = osv.dirichlet_mask(mesh, 0o7)
    pb = osv.Problem(mesh, np.full(mesh.E, mu), np.full(mesh.E, lam), 1.0, mask)
    u, hist = osv.newton_static(pb, np.zeros(3 * mesh.Nn), static_loads(mesh, Bf), 1e-8, pcg_rtol,
                                max_pcg=max_pcg)
    err = l2_error(mesh, u, static_field(volume_points(mesh)))
    return u, hist, err


# ---------------------------------------- transient example (Sec. 5.2, wave)
RHO_WAVE = 1.0


def wave_field(X, t):
    """u* = (sin(pi x / 2) sin(2 pi t), 0, 0) (Eq. eq:large_field)."""
    out = np.zeros_like(X)
    out[0] = np.sin(0.5 * np.pi * X[0]) * np.sin(2.0 * np.pi * t)
    return out


def quartic_field(X, t):
    """u* = (x^4 sin(2 pi t), 0, 0) (Section 5.2, implicit time integration)."""
    out = np.zeros_like(X)
    out[0] = X[0] ** 4 * np.sin(2.0 * np.pi * t)
    return out


_D2 = ((-2, -1.0 / 12), (-1, 16.0 / 12), (0, -30.0 / 12), (1, 16.0 / 12), (2, -1.0 / 12))


def time_derivative(ufun_t, X, t, order, tau=1e-3):
    """First or second derivative in t of ufun_t(X, t), fourth-order central
    differences."""
    st = _D4 if order == 1 else _D2
    out = np.zeros_like(X)
    for k, c in st:
        out += c * ufun_t(X, t + k * tau)
    return out / (tau if order == 1 else tau * tau)


def dynamic_body_force(ufun_t, X, t, lam, mu, rho, delta=1e-3):
    """b = rho d2u*/dt2 - Div P(F(u*)) at points X (3, N) and time t."""
    return (rho * time_derivative(ufun_t, X, t, 2) +
            body_force(lambda Y: ufun_t(Y, t), X, lam, mu, delta))


def wave_loads(mesh, Bf, t, field=wave_field):
    lam, mu = lame(E_STATIC, NU_STATIC)
    Xv = volume_points(mesh)
    bv = dynamic_body_force(field, Xv.reshape(3, -1), t, lam, mu, RHO_WAVE)
    f = body_load(mesh, bv.reshape(Xv.shape))
    for face in range(1, 6):
        Xf = face_points(mesh, face)
        tf = traction(lambda Y: field(Y, t), face, Xf.reshape(3, -1), lam, mu)
        f += face_load(mesh, face, Bf, tf.reshape(Xf.shape))
    return f


def _wave_problem(P, kind, Q=None, lumped=False, field=wave_field):
    """Mesh, face table, problem and projected initial velocity of the wave
    example; lumped: the mass with the Gauss-Lobatto-Legendre rule of P+1
    points (diagonal for the nodal basis), the rest with the mesh's rule."""
    mesh, Bf = static_mesh(P, kind, Q=Q)
    lam, mu = lame(E_STATIC, NU_STATIC)
    mask = osv.dirichlet_mask(mesh, 0o7)
    pb = osv.Problem(mesh, np.full(mesh.E, mu), np.full(mesh.E, lam), RHO_WAVE, mask)
    if lumped:
        mm, _ = static_mesh(P, kind, Q=P + 1)
        pbm = osv.Problem(mm, pb.mu, pb.lam, RHO_WAVE, mask)
        pb.M, pb.mass_diag, pb.mass_solve = pbm.M, pbm.mass_diag, pbm.mass_solve
    Xv = volume_points(mesh)
    vq = time_derivative(field, Xv, 0.0, 1)
    # the initial velocity: L2 projection of du*/dt(0) (rho M v0 = rho int N v*)
    v0, _ = pb.mass_solve(RHO_WAVE * body_load(mesh, vq), 1e-13)
    return mesh, Bf, pb, v0


def wave_explicit(P, kind, dt, nsteps, mass_rtol=1e-12, Q=None, lumped=False):
    """Central differences (start step of Section 4) from u = 0 and the
    projected initial velocity; returns (u_nsteps, L2 errors at t = nsteps dt)
    (errors by the P + 2 point Gauss-Legendre rule)."""
    mesh, Bf, pb, v0 = _wave_problem(P, kind, Q, lumped)
    u_cur = np.zeros(3 * mesh.Nn)
    u_prev = osv.explicit_start(pb, u_cur, v0, wave_loads(mesh, Bf, 0.0), dt, mass_rtol)
    for n in range(nsteps):
        f = wave_loads(mesh, Bf, n * dt) if n else wave_loads(mesh, Bf, 0.0)
        u_prev, u_cur = u_cur, osv.explicit_step(pb, u_prev, u_cur, f, dt, mass_rtol)
    # the error by the Gauss-Legendre rule of P + 2 points, whatever the
    # rule of the run
    emesh, _ = static_mesh(P, kind)
    err = l2_error(emesh, u_cur, wave_field(volume_points(emesh), nsteps * dt))
    return u_cur, err


def wave_newmark(P, kind, dt, nsteps, newton_rtol=1e-8, pcg_rtol=1e-8, field=wave_field):
    """Newmark (beta = 1/4, gamma = 1/2) with Newton from u = 0, the projected
    initial velocity and a_0 = M^-1 (f_0 - R(0)); returns (u, L2 errors,
    Newton iterations, PCG iterations per step)."""
    mesh, Bf, pb, v = _wave_problem(P, kind, field=field)
    u = np.zeros(3 * mesh.Nn)
    a, _ = pb.mass_solve(wave_loads(mesh, Bf, 0.0, field) - pb.R(u), 1e-13)
    newton, pcg_its = 0, []
    for n in range(nsteps):
        f = wave_loads(mesh, Bf, (n + 1) * dt, field)
        u, v, a, nk, its = osv.newmark_step(pb, u, v, a, f, dt, newton_rtol, pcg_rtol)
        newton += nk
        pcg_its += its
    err = l2_error(mesh, u, field(volume_points(mesh), nsteps * dt))
    return u, err, newton, pcg_its
