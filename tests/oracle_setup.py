"""Test helper: build oracle meshes and problems from workload parameters."""
import numpy as np

from oracle import basis as ob
from oracle import fem
from oracle import solvers as osv
from paper_2104_13466_amd import inputs


def make(n, L, P, Q=None, kind=ob.SDME_H, E=1.0e3, nu=0.3, rho=1.0, dirichlet=0, k=0.5,
         lam_h=100.0, mu=None, lam=None):
    Q = P + 2 if Q is None else Q
    basis, x, w, B, D = ob.build(P, Q, kind, k=k, lam=lam_h)
    h = [L[i] / n[i] for i in range(3)]
    mesh = fem.Mesh(n[0], n[1], n[2], P, Q, h, B, D, w)
    lam0, mu0 = inputs.lame(E, nu)
    mu = np.full(mesh.E, mu0) if mu is None else np.asarray(mu, dtype=np.float64)
    lam = np.full(mesh.E, lam0) if lam is None else np.asarray(lam, dtype=np.float64)
    mask = osv.dirichlet_mask(mesh, dirichlet)
    return osv.Problem(mesh, mu, lam, rho, mask), basis
