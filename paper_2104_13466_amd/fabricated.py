"""Fabricated-solution problems (Section 5): a prescribed displacement field
u*, and the body force and face tractions that make it the exact solution of
the neo-Hookean equilibrium problem of Section 3 (total Lagrangian, loads per
unit reference volume and area).  This module holds problem data only: closed
forms evaluated at points the library supplies (``Context.quadrature_points``);
the loads are assembled by the library (``body_load``, ``face_load``) and the
error by ``l2_error``.

Static large-strain example of Section 5.1 (unit cube, 2x2x2 hexahedra,
E = 1000, nu = 0.3): u* = (1.9 sin x - x, 0, 0).  Then F = diag(J, 1, 1) with
J = 1.9 cos x, and the first Piola-Kirchhoff stress of the neo-Hookean law
S = mu (I - C^-1) + lambda ln J C^-1, P = F S is diagonal:
    P11 = mu (J - 1/J) + lambda ln J / J,   P22 = P33 = lambda ln J,
all functions of x alone.  Body force b = -Div P = (-dP11/dx, 0, 0) with
dP11/dx = (mu (1 + 1/J^2) + lambda (1 - ln J) / J^2) J'(x), J' = -1.9 sin x;
traction t = P N on a face with outward normal N.

Boundary conditions (the paper states only the field): the face x = 0 is
clamped (u* = 0 there; this reproduces the paper's DOF counts 3 (2P+1)^2 2P
for this mesh), every other face carries the traction of u*.
"""
import numpy as np

from . import inputs

E_MOD, NU = 1000.0, 0.3
DIRICHLET_X0 = 0o7  # face 0 (x = 0), all three components


def lame():
    """(lambda, mu) of the static example."""
    return inputs.lame(E_MOD, NU)


# ------------------------------------------------------------ uniaxial fields
# Both examples are uniaxial, u* = (w(x, t), 0, 0): F = diag(J, 1, 1) with
# J = 1 + w_x, and P is diagonal with P11 = mu (J - 1/J) + lambda ln J / J,
# P22 = P33 = lambda ln J; b = rho w_tt - (dP11/dJ) w_xx e_x with
# dP11/dJ = mu (1 + 1/J^2) + lambda (1 - ln J) / J^2.
#   static (Section 5.1):      w = 1.9 sin x - x
#   wave (Section 5.2, Eq. eq:large_field): w = sin(pi x / 2) sin(2 pi t),
#       t in [0, 0.25], rho = 1, explicit and Newmark integration
#   quartic (Section 5.2, implicit time integration): w = x^4 sin(2 pi t),
#       t in [0, 0.025], Newmark integration
RHO = 1.0
FIELDS = ("static", "wave", "quartic")


def _w(name, x, t):
    """(w, w_x, w_xx, w_t, w_tt) of the field."""
    if name == "static":
        z = np.zeros_like(x)
        return 1.9 * np.sin(x) - x, 1.9 * np.cos(x) - 1.0, -1.9 * np.sin(x), z, z
    if name == "wave":
        k, om = 0.5 * np.pi, 2.0 * np.pi
        sx, cx, st, ct = np.sin(k * x), np.cos(k * x), np.sin(om * t), np.cos(om * t)
        return sx * st, k * cx * st, -k * k * sx * st, om * sx * ct, -om * om * sx * st
    if name == "quartic":
        om = 2.0 * np.pi
        st, ct = np.sin(om * t), np.cos(om * t)
        return (x ** 4 * st, 4.0 * x ** 3 * st, 12.0 * x ** 2 * st, om * x ** 4 * ct,
                -om * om * x ** 4 * st)
    raise ValueError(name)


def _piola(J):
    lam, mu = lame()
    lnJ = np.log(J)
    return (mu * (J - 1.0 / J) + lam * lnJ / J, lam * lnJ,
            mu * (1.0 + 1.0 / J ** 2) + lam * (1.0 - lnJ) / J ** 2)


def field_u(name, X, t=0.0):
    """u* at points X (3, ...) -> (3, ...)."""
    out = np.zeros_like(X)
    out[0] = _w(name, X[0], t)[0]
    return out


def field_v(name, X, t=0.0):
    """du*/dt at points X."""
    out = np.zeros_like(X)
    out[0] = _w(name, X[0], t)[3]
    return out


def body_force(name, X, t=0.0):
    """b = rho d2u*/dt2 - Div P(u*) at points X (3, ...) -> (3, ...)."""
    w, wx, wxx, wt, wtt = _w(name, X[0], t)
    _, _, dP = _piola(1.0 + wx)
    out = np.zeros_like(X)
    out[0] = RHO * wtt - dP * wxx
    return out


def traction(name, face, X, t=0.0):
    """t = P(u*) N on face `face` (0..5: x=0, x=max, y=0, y=max, z=0, z=max)
    at points X (3, ...) -> (3, ...)."""
    d, side = face // 2, face % 2
    P11, P22, _ = _piola(1.0 + _w(name, X[0], t)[1])
    out = np.zeros_like(X)
    out[d] = (1.0 if side else -1.0) * (P11 if d == 0 else P22)
    return out


def loads(ctx, name, f, t=0.0):
    """Assemble the external load of the field at time t into f (device
    double [3 Nn], accumulated): body force over the box and tractions on the
    five faces other than the clamped x = 0."""
    import torch
    b = torch.as_tensor(body_force(name, ctx.quadrature_points(), t), device=f.device)
    ctx.body_load(b.contiguous(), f)
    for face in range(1, 6):
        tr = torch.as_tensor(traction(name, face, ctx.quadrature_points(face), t), device=f.device)
        ctx.face_load(face, tr.contiguous(), f)
    torch.cuda.synchronize()


def exact_at_gauss_points(ctx, name, t=0.0, device="cuda"):
    """u* at the volume Gauss points (3, E, Q^3), on the device."""
    import torch
    return torch.as_tensor(field_u(name, ctx.quadrature_points(), t), device=device).contiguous()


def static_u(X):
    return field_u("static", X)


def static_body_force(X):
    return body_force("static", X)


def static_traction(face, X):
    return traction("static", face, X)


def static_loads(ctx, f):
    loads(ctx, "static", f)


def static_exact_at_gauss_points(ctx, device="cuda"):
    return exact_at_gauss_points(ctx, "static", 0.0, device)


# ------------------------------------------------ transient drivers (wave)
def _projection(ctx, mat, name, t, prec):
    """Coefficients of the L2 projection of du*/dt (t) (mass solve)."""
    import torch
    b = torch.zeros(3 * ctx.Nn, dtype=torch.float64, device="cuda")
    vq = torch.as_tensor(field_v(name, ctx.quadrature_points(), t), device="cuda").contiguous()
    ctx.body_load(vq, b)
    x = torch.zeros_like(b)
    ctx.jacobi_pcg(mat, prec, b, x, mass_only=True, rtol=1e-13, maxit=100000)
    return x


def wave_explicit(ctx, mat, dt, nsteps, prec_force, mass_rtol=1e-12, name="wave"):
    """Central differences from u = 0 and the projected initial velocity of
    the field, external load of the field at every step; returns (u at
    t = nsteps dt, total mass-PCG iterations)."""
    import torch
    from .sdme import FP64
    N = 3 * ctx.Nn
    us = [torch.zeros(N, dtype=torch.float64, device="cuda") for _ in range(3)]
    f = torch.zeros(N, dtype=torch.float64, device="cuda")
    v0 = _projection(ctx, mat, name, 0.0, FP64)
    mass_its = 0
    for n in range(nsteps):
        f.zero_()
        loads(ctx, name, f, n * dt)
        prev, cur, nxt = us[(n + 2) % 3], us[n % 3], us[(n + 1) % 3]
        st = ctx.explicit_step(mat, prec_force, None if n == 0 else prev, cur, nxt, dt,
                               v0=v0 if n == 0 else None, f_ext=f, mass_rtol=mass_rtol)
        mass_its += st["mass_iterations"]
    return us[nsteps % 3], mass_its


def wave_newmark(ctx, mat, dt, nsteps, prec, newton_rtol=1e-8, pcg_rtol=1e-8, name="wave"):
    """Newmark (beta = 1/4, gamma = 1/2) with Newton from u = 0, the projected
    initial velocity and a_0 = M^-1 (f_0 - R(0)); returns (u at t = nsteps dt,
    Newton iterations, PCG iterations)."""
    import torch
    from .sdme import FP64, MASK_BC
    N = 3 * ctx.Nn
    u = torch.zeros(N, dtype=torch.float64, device="cuda")
    v = _projection(ctx, mat, name, 0.0, FP64)
    f = torch.zeros_like(u)
    loads(ctx, name, f, 0.0)
    R = torch.zeros_like(u)
    ctx.internal_force(mat, FP64, u, R, flags=MASK_BC)
    ctx.axpby(1.0, f, -1.0, R)
    a = torch.zeros_like(u)
    ctx.jacobi_pcg(mat, FP64, R, a, mass_only=True, rtol=1e-13, maxit=100000)
    newton = pcg = 0
    for n in range(nsteps):
        f.zero_()
        loads(ctx, name, f, (n + 1) * dt)
        st = ctx.newmark_newton_step(mat, prec, u, v, a, f, dt, newton_rtol=newton_rtol,
                                     pcg_rtol=pcg_rtol)
        newton += st["newton"]
        pcg += st["iterations"]
    return u, newton, pcg
