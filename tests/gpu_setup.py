"""Test helper: one mesh set up twice -- in libsdme (HIP) and in the oracle --
from the same seeded inputs."""
import numpy as np

from paper_2104_13466_amd import inputs
from paper_2104_13466_amd.sdme import Context
from tests.oracle_setup import make


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


class Pair:
    def __init__(self, n, L, P, kind=4, dirichlet=0, mu=None, lam=None, rho=1.0, E=1.0e3, nu=0.3,
                 Q=None, k=0.5, lambda_h=100.0, ordered=False):
        import torch
        self.torch = torch
        self.pb, self.basis = make(n, L, P, Q=Q, kind=kind, dirichlet=dirichlet, mu=mu, lam=lam,
                                   rho=rho, E=E, nu=nu, k=k, lam_h=lambda_h)
        self.ctx = Context(n, L, P, basis=kind, dirichlet=dirichlet, Q=Q, k=k, lambda_h=lambda_h,
                           ordered=ordered)
        self.n, self.P, self.rho = n, P, rho
        self.mu_t = self.dev(self.pb.mu)
        self.lam_t = self.dev(self.pb.lam)
        self.mat = Context.material(self.mu_t, self.lam_t, rho)
        self.N = 3 * self.ctx.Nn
        self.mask = self.pb.mask

    def dev(self, a, dtype=None):
        t = self.torch
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype or t.float64, device="cuda")

    def zeros(self, dtype=None):
        return self.torch.zeros(self.N, dtype=dtype or self.torch.float64, device="cuda")

    def empty_state(self, dtype=None):
        return self.torch.empty(self.ctx.nqp * 10, dtype=dtype or self.torch.float64, device="cuda")

    def host(self, t):
        self.torch.cuda.synchronize()
        return t.double().cpu().numpy()

    def rand(self, seed, amp, stream=0):
        return inputs.random_coeffs(seed, self.n, self.P, amp, stream=stream)
