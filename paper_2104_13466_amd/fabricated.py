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


def static_u(X):
    """u* at points X (3, ...) -> (3, ...)."""
    x = X[0]
    out = np.zeros_like(X)
    out[0] = 1.9 * np.sin(x) - x
    return out


def _stresses(x):
    lam, mu = lame()
    J = 1.9 * np.cos(x)
    lnJ = np.log(J)
    return J, lnJ, mu * (J - 1.0 / J) + lam * lnJ / J, lam * lnJ


def static_body_force(X):
    """b = -Div P(u*) at points X (3, ...) -> (3, ...)."""
    lam, mu = lame()
    x = X[0]
    J, lnJ, _, _ = _stresses(x)
    dJ = -1.9 * np.sin(x)
    out = np.zeros_like(X)
    out[0] = -(mu * (1.0 + 1.0 / J ** 2) + lam * (1.0 - lnJ) / J ** 2) * dJ
    return out


def static_traction(face, X):
    """t = P(u*) N on face `face` (0..5: x=0, x=max, y=0, y=max, z=0, z=max)
    at points X (3, ...) -> (3, ...)."""
    d, side = face // 2, face % 2
    sgn = 1.0 if side else -1.0
    _, _, P11, P22 = _stresses(X[0])
    out = np.zeros_like(X)
    out[d] = sgn * (P11 if d == 0 else P22)
    return out


def static_loads(ctx, f):
    """Assemble the static example's external load into f (device double
    [3 Nn], accumulated): body force over the box and tractions on the five
    faces other than the clamped x = 0."""
    import torch
    b = torch.as_tensor(static_body_force(ctx.quadrature_points()), device=f.device).contiguous()
    ctx.body_load(b, f)
    for face in range(1, 6):
        t = torch.as_tensor(static_traction(face, ctx.quadrature_points(face)),
                            device=f.device).contiguous()
        ctx.face_load(face, t, f)
    torch.cuda.synchronize()


def static_exact_at_gauss_points(ctx, device="cuda"):
    """u* at the volume Gauss points (3, E, Q^3), on the device."""
    import torch
    return torch.as_tensor(static_u(ctx.quadrature_points()), device=device).contiguous()
