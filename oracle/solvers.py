"""ORACLE -- test infrastructure only.

Textbook FP64 drivers on top of the direct element loops of ``oracle/fem.c``:
Dirichlet masks, the affine-field expansion, preconditioned conjugate gradients
with the diagonal (Jacobi) preconditioner, static Newton-Raphson, the Newmark
step with Newton iterations (Section 4, implicit time integration), the central
difference scheme (Section 4, explicit time integration) with a rigid-plane
penalty, energies, and the discrete adjoint of a central-difference rollout.

Readings (paper silent or garbled; also listed in the design notes):
* Newmark coefficients: the standard beta = 1/4, gamma = 1/2 scheme,
  a_{n+1} = (u_{n+1}-u_n)/(beta dt^2) - v_n/(beta dt) - (1/(2 beta)-1) a_n,
  v_{n+1} = v_n + dt((1-gamma) a_n + gamma a_{n+1}).  The printed b-coefficients
  and g1 = 0.5, g2 = 0.25 contradict the stated unconditional stability.
* Newton and CG tolerances are relative: ||psi_k|| <= tol ||psi_0||,
  ||r|| <= tol ||b||.
* The linearised system reads K^ du = psi with psi = P - R - M a (the printed
  equation "psi + du^T K^ Delta" is garbled).
* Dirichlet DOFs carry their prescribed values in u; increments, residuals and
  accelerations are zero there.
"""
import numpy as np


# ----------------------------------------------------------------- problem setup
def dirichlet_mask(mesh, bits):
    """1.0 on free DOFs, 0.0 on DOFs of face f, component c with bit f*3+c set
    (faces 0:x=0 1:x=max 2:y=0 3:y=max 4:z=0 5:z=max); SoA [3][Nn]."""
    m = np.ones((3, mesh.Nz, mesh.Ny, mesh.Nx))
    for f in range(6):
        for c in range(3):
            if not (bits >> (f * 3 + c)) & 1:
                continue
            d, side = f // 2, f % 2
            idx = [slice(None)] * 3
            n_d = (mesh.Nx, mesh.Ny, mesh.Nz)[d]
            idx[2 - d] = n_d - 1 if side else 0
            m[(c,) + tuple(idx)] = 0.0
    return m.reshape(-1)


def affine_field(mesh, basis, origin, a, G):
    """Coefficients of u(X) = a + G X, expanded exactly in the tensor-product
    basis: on each element X = Xc + (h/2) xi, so u is the sum of a constant and
    three linear-in-one-direction terms, each a tensor product of the 1D
    expansions of 1 and xi."""
    g1, gx = basis.affine_coeffs()
    P, n = mesh.P, mesh.P + 1
    a = np.asarray(a, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64).reshape(3, 3)
    h = mesh.h
    u = np.zeros((3, mesh.Nz, mesh.Ny, mesh.Nx))
    t_c = np.einsum("c,b,a->cba", g1, g1, g1)
    t_x = np.einsum("c,b,a->cba", g1, g1, gx)
    t_y = np.einsum("c,b,a->cba", g1, gx, g1)
    t_z = np.einsum("c,b,a->cba", gx, g1, g1)
    for ez in range(mesh.nz):
        for ey in range(mesh.ny):
            for ex in range(mesh.nx):
                Xc = np.asarray(origin) + (np.array([ex, ey, ez]) + 0.5) * h
                for i in range(3):
                    c0 = a[i] + G[i] @ Xc
                    blk = (c0 * t_c + G[i, 0] * h[0] / 2 * t_x + G[i, 1] * h[1] / 2 * t_y +
                           G[i, 2] * h[2] / 2 * t_z)
                    u[i, ez * P:ez * P + n, ey * P:ey * P + n, ex * P:ex * P + n] = blk
    return u.reshape(-1)


# ------------------------------------------------------------------------- PCG
def pcg(apply, b, d, rtol, maxit, x0=None):
    """Conjugate gradients with the diagonal preconditioner z = r / d.
    Stops when ||r||_2 <= rtol ||b||_2.  Returns (x, iterations, ||r||/||b||)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x) if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = r / d
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * nb and it < maxit:
        Ap = apply(p)
        pAp = p @ Ap
        if pAp <= 0:
            raise ArithmeticError("CG breakdown: p^T A p <= 0")
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        z = r / d
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, np.linalg.norm(r) / nb


class Problem:
    """Mesh + material + Dirichlet mask with masked operators."""

    def __init__(self, mesh, mu, lam, rho, mask):
        self.mesh, self.mu, self.lam, self.rho, self.mask = mesh, mu, lam, rho, mask

    def R(self, u):
        return self.mesh.internal_force(self.mu, self.lam, u)

    def A(self, ulin, cm):
        m = self.mask
        return lambda v: m * self.mesh.tangent_apply(self.mu, self.lam, ulin, m * v, cm)

    def diag(self, ulin, cm):
        return np.where(self.mask > 0, self.mesh.tangent_diag(self.mu, self.lam, ulin, cm), 1.0)

    def M(self, v):
        m = self.mask
        return m * self.mesh.mass_apply(self.rho, m * v)

    def mass_diag(self):
        # diag(rho M): the tangent diagonal with zero Lame parameters at u = 0
        return np.where(self.mask > 0, self.mesh.tangent_diag(
            np.zeros(self.mesh.E), np.zeros(self.mesh.E), np.zeros(3 * self.mesh.Nn), self.rho), 1.0)

    def mass_solve(self, f, rtol):
        x, its, _ = pcg(self.M, self.mask * f, self.mass_diag(), rtol, 10000)
        return x, its


# --------------------------------------------------------------- static Newton
def newton_static(pb, u0, f_ext, newton_rtol, pcg_rtol, max_newton=20, max_pcg=100000):
    """Newton-Raphson for R(u) = f_ext: K_T(u) du = psi, psi = f_ext - R(u)."""
    u = u0.copy()
    hist = []
    psi0 = None
    for k in range(max_newton + 1):
        psi = pb.mask * (f_ext - pb.R(u))
        npsi = np.linalg.norm(psi)
        psi0 = npsi if psi0 is None else psi0
        hist.append(npsi)
        if npsi <= newton_rtol * psi0 or k == max_newton:
            break
        du, its, _ = pcg(pb.A(u, 0.0), psi, pb.diag(u, 0.0), pcg_rtol, max_pcg)
        hist.append(("pcg", its))
        u += du
    return u, hist


# -------------------------------------------------------------------- Newmark
def newmark_coeffs(dt, beta=0.25, gamma=0.5):
    return 1.0 / (beta * dt * dt), 1.0 / (beta * dt), 1.0 / (2.0 * beta) - 1.0


def newmark_step(pb, u_n, v_n, a_n, f_next, dt, newton_rtol, pcg_rtol, beta=0.25, gamma=0.5,
                 max_newton=20, max_pcg=100000):
    """One Newmark step with Newton iterations on
    psi = P_{n+1} - R(u) - M (b1 (u - u_n) - b2 v_n - b3 a_n),
    (b1 M + K_T) du = psi (Section 4, implicit time integration)."""
    b1, b2, b3 = newmark_coeffs(dt, beta)
    u = u_n.copy()
    psi0 = None
    newton_its, pcg_its = 0, []
    for k in range(max_newton + 1):
        acc = pb.mask * (b1 * (u - u_n) - b2 * v_n - b3 * a_n)
        psi = pb.mask * (f_next - pb.R(u) - pb.M(acc))
        npsi = np.linalg.norm(psi)
        psi0 = npsi if psi0 is None else psi0
        if npsi <= newton_rtol * psi0 or k == max_newton:
            break
        du, its, _ = pcg(pb.A(u, b1 * pb.rho), psi, pb.diag(u, b1 * pb.rho), pcg_rtol, max_pcg)
        pcg_its.append(its)
        u += du
        newton_its += 1
    a = pb.mask * (b1 * (u - u_n) - b2 * v_n - b3 * a_n)
    v = v_n + dt * ((1.0 - gamma) * a_n + gamma * a)
    return u, v, a, newton_its, pcg_its


# ------------------------------------------------------------ central difference
class Contact:
    """Rigid plane z = z0 below face z=0, penalty eps, surface rule (Bf, wf)."""

    def __init__(self, eps, z0, origin_z, Bf, wf):
        self.eps, self.z0, self.origin_z, self.Bf, self.wf = eps, z0, origin_z, Bf, wf

    def force(self, mesh, u):
        f = mesh.vec()
        e = mesh.penalty_plane(self.eps, self.z0, self.origin_z, self.Bf, self.wf, u, f)
        return f, e


def explicit_accel(pb, u, f_ext, mass_rtol, contact=None):
    """a = M^-1 (P - R(u) + f_c(u)) on free DOFs (Eq. Motion_explicit1)."""
    f = f_ext - pb.R(u)
    if contact is not None:
        fc, _ = contact.force(pb.mesh, u)
        f = f + fc
    a, _ = pb.mass_solve(f, mass_rtol)
    return a


def explicit_start(pb, u0, v0, f0, dt, mass_rtol, contact=None):
    """u_{-1} = u_0 - dt v_0 + dt^2/2 a_0 with a_0 = M^-1 psi_0."""
    a0 = explicit_accel(pb, u0, f0, mass_rtol, contact)
    return u0 - dt * v0 + 0.5 * dt * dt * a0


def explicit_step(pb, u_prev, u_cur, f_ext, dt, mass_rtol, contact=None):
    """u_{n+1} = 2 u_n - u_{n-1} + dt^2 M^-1 (P_n - R(u_n)) (Eq. Motion_explicit2)."""
    a = explicit_accel(pb, u_cur, f_ext, mass_rtol, contact)
    return 2.0 * u_cur - u_prev + dt * dt * a


def energies(pb, u_prev, u_cur, u_next, dt, contact=None):
    """(kinetic, strain, contact) at step n with v_n = (u_{n+1}-u_{n-1})/(2 dt)."""
    v = (u_next - u_prev) / (2.0 * dt)
    ke = 0.5 * v @ pb.M(v)
    se = pb.mesh.strain_energy(pb.mu, pb.lam, u_cur)
    ce = 0.0
    if contact is not None:
        _, ce = contact.force(pb.mesh, u_cur)
    return ke, se, ce


# --------------------------------------------------------------------- adjoint
def rollout(pb, u0, v0, dt, K, mass_rtol):
    """States u_0..u_K of the central-difference scheme without load."""
    zero = np.zeros_like(u0)
    a0 = explicit_accel(pb, u0, zero, mass_rtol)
    us = [u0, u0 + dt * v0 + 0.5 * dt * dt * a0]
    for n in range(1, K):
        us.append(explicit_step(pb, us[n - 1], us[n], zero, dt, mass_rtol))
    return us


def misfit(pb, uK, target):
    r = pb.mask * (uK - target)
    return 0.5 * r @ r


def adjoint_gradient(pb, u0, v0, dt, K, target, mass_rtol):
    """dJ/dmu_e, dJ/dlam_e of J = 1/2 ||u_K - u*||^2 through K central-difference
    steps.  Reverse recursion with w_{n+1} = M^-1 lam_{n+1}:
      lam_n = 2 lam_{n+1} - dt^2 K_T(u_n) w_{n+1} - lam_{n+2},
      dJ/dtheta = -dt^2 sum_{n>=1} w_{n+1}^T dR(u_n)/dtheta
                  - dt^2/2 w_1^T dR(u_0)/dtheta."""
    us = rollout(pb, u0, v0, dt, K, mass_rtol)
    g_mu = np.zeros(pb.mesh.E)
    g_lam = np.zeros(pb.mesh.E)
    lam_n1 = pb.mask * (us[K] - target)  # lam_K
    lam_n2 = np.zeros_like(lam_n1)         # lam_{K+1}
    for n in range(K - 1, -1, -1):
        w, _ = pb.mass_solve(lam_n1, mass_rtol)  # w_{n+1}
        scale = -dt * dt if n >= 1 else -0.5 * dt * dt
        pb.mesh.material_grad(us[n], w, scale, g_mu, g_lam)
        if n >= 1:
            Kw = pb.A(us[n], 0.0)(w)
            lam_n = 2.0 * lam_n1 - dt * dt * Kw - lam_n2
            lam_n2, lam_n1 = lam_n1, pb.mask * lam_n
    return g_mu, g_lam, 0.5 * np.sum((pb.mask * (us[K] - target)) ** 2)
