"""Parity at full size: the compress_p4 workload (47^3 hexahedra, P = 4,
Q = 6, SDME-H, 20,253,807 DOF, z = 0 clamped and z = 1 prescribed) in the
launch configuration the benchmark times.  The GPU applies the FP32
stored-state tangent with the Dirichlet mask (the PCG operator of the mixed
Newton iteration), the FP64 stored-state tangent and the FP64 internal force
to the whole mesh; the oracle evaluates the same operators on the 3x3x3-element
sub-box around each sampled element (clipped at the mesh boundary), which holds
every element that touches the sampled element's slots, and the outputs are
compared on all slots of the sampled elements.  Tolerances as for the small
meshes: 1e-5 (FP32) and 1e-12 (FP64), relative in the max norm over the
sample; for the internal force of the near-equilibrium state the FP64 bound is
relative to the sum of absolute element contributions.  The PCG operator with
the fused direction update (the kernel the benchmark times) is checked through
two iterations of the mixed-precision PCG against the oracle's FP64 CG on the
whole mesh.  The mass action (a z-marching stencil whose blocks own chunks of
element layers along z) is sampled on the seeded elements and on a whole
column of elements along z, which crosses every chunk boundary whatever the
chunk size the device's occupancy gives."""
import numpy as np
import pytest

from paper_2104_13466_amd import inputs
from paper_2104_13466_amd.sdme import FP32, FP64, MASK_BC, Context
from oracle import solvers as osv
from tests.gpu_setup import relerr
from tests.oracle_setup import make

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
NSAMPLE = 24


class Full:
    def __init__(self, name="compress_p4", nsample=NSAMPLE):
        import torch
        self.torch = torch
        w = inputs.WORKLOADS[name]
        self.w = w
        self.n, self.L, self.P = w["n"], w["L"], w["P"]
        self.ctx = Context(self.n, self.L, self.P, basis=w["kind"], dirichlet=w["dirichlet"])
        lam0, mu0 = inputs.lame(w["E"], w["nu"])
        self.mu0, self.lam0 = mu0, lam0
        dev = "cuda"
        self.mat = Context.material(torch.full((self.ctx.E,), mu0, dtype=torch.float64, device=dev),
                                    torch.full((self.ctx.E,), lam0, dtype=torch.float64, device=dev),
                                    w["rho"])
        # the benchmark's input: 20 % compression plus a seeded perturbation
        G = np.zeros((3, 3))
        G[2, 2] = -0.2
        self.mask = 1.0 - self.ctx.dirichlet_flags().astype(np.float64)
        amp = 1e-3 * min(self.L[i] / self.n[i] for i in range(3))
        self.u = self.ctx.affine_field([0, 0, 0], G) + self.mask * inputs.random_coeffs(
            w["seed"], self.n, self.P, amp)
        self.v = inputs.uniform(w["seed"], self.u.size, -1, 1, stream=3)
        self.N = self.u.size
        self.grid = (self.n[2] * self.P + 1, self.n[1] * self.P + 1, self.n[0] * self.P + 1)
        # sampled elements: seeded, including the clamped and the moved faces
        r = inputs.uniform(w["seed"], 3 * nsample, stream=11).reshape(nsample, 3)
        e = (r * np.array(self.n)).astype(int)
        e[0] = (0, 0, 0)
        e[1] = (self.n[0] - 1, self.n[1] - 1, self.n[2] - 1)
        self.elems = e

    def dev(self, a, dt):
        return self.torch.as_tensor(a, dtype=dt, device="cuda")

    def host(self, t):
        self.torch.cuda.synchronize()
        return t.double().cpu().numpy()

    def field(self, a):
        return a.reshape((3,) + self.grid)

    def sample(self, gpu_out, oracle_fn, abs_sum=False):
        """(gpu values, oracle values, scale) on all slots of the sampled
        elements; oracle_fn(problem, u_sub, v_sub, mask_sub) -> output on the
        sub-box.  With abs_sum, scale holds per slot the sum over the elements
        that touch it of |element contribution| (oracle_fn on one-element
        boxes), the conditioning of the assembly sum; else None."""
        P = self.P
        h = [self.L[i] / self.n[i] for i in range(3)]
        gf, uf, vf, mf = (self.field(a) for a in (gpu_out, self.u, self.v, self.mask))
        got, ref, scale = [], [], []
        for ex, ey, ez in self.elems:
            lo = [max(0, c - 1) for c in (ex, ey, ez)]
            hi = [min(self.n[i], c + 2) for i, c in enumerate((ex, ey, ez))]
            ns = [hi[i] - lo[i] for i in range(3)]
            sl = (slice(None), slice(lo[2] * P, hi[2] * P + 1), slice(lo[1] * P, hi[1] * P + 1),
                  slice(lo[0] * P, hi[0] * P + 1))
            pb, _ = make(ns, [ns[i] * h[i] for i in range(3)], P, kind=self.w["kind"],
                         E=self.w["E"], nu=self.w["nu"])
            y = oracle_fn(pb, uf[sl].ravel().copy(), vf[sl].ravel().copy(), mf[sl].ravel().copy())
            y = y.reshape(uf[sl].shape)
            # slots of the sampled element inside the sub-box
            a0 = [(c - l) * P for c, l in zip((ex, ey, ez), lo)]
            es = (slice(None), slice(a0[2], a0[2] + P + 1), slice(a0[1], a0[1] + P + 1),
                  slice(a0[0], a0[0] + P + 1))
            gs = (slice(None), slice(ez * P, ez * P + P + 1), slice(ey * P, ey * P + P + 1),
                  slice(ex * P, ex * P + P + 1))
            got.append(gf[gs].ravel())
            ref.append(y[es].ravel())
            if abs_sum:
                acc = np.zeros_like(y)
                for kz in range(ns[2]):
                    for ky in range(ns[1]):
                        for kx in range(ns[0]):
                            s1 = (slice(None), slice(kz * P, kz * P + P + 1),
                                  slice(ky * P, ky * P + P + 1), slice(kx * P, kx * P + P + 1))
                            pe, _ = make((1, 1, 1), h, P, kind=self.w["kind"], E=self.w["E"],
                                         nu=self.w["nu"])
                            ue = uf[sl][s1].ravel().copy()
                            ye = oracle_fn(pe, ue, vf[sl][s1].ravel().copy(),
                                           mf[sl][s1].ravel().copy())
                            acc[s1] += np.abs(ye.reshape(acc[s1].shape))
                scale.append(acc[es].ravel())
        return (np.concatenate(got), np.concatenate(ref),
                np.concatenate(scale) if abs_sum else None)


@pytest.fixture(scope="module")
def full():
    return Full()


def test_fullsize_fp32_masked_tangent_state(full):
    t = full.torch
    f32 = t.float32
    u32, v32 = full.u.astype(np.float32), full.v.astype(np.float32)
    st = t.empty(full.ctx.nqp * 10, dtype=f32, device="cuda")
    full.ctx.linearize(full.mat, FP32, full.dev(u32, f32), st)
    y = t.zeros(full.N, dtype=f32, device="cuda")
    full.ctx.tangent_apply(full.mat, FP32, full.dev(v32, f32), y, state=st, flags=MASK_BC)
    full.u = u32.astype(np.float64)
    full.v = v32.astype(np.float64)

    def oracle(pb, u, v, m):
        return m * pb.mesh.tangent_apply(pb.mu, pb.lam, u, m * v)
    got, ref, _ = full.sample(full.host(y), oracle)
    assert relerr(got, ref) < TOL32


def test_fullsize_fp64_force_and_tangent(full):
    t = full.torch
    w = full.w
    G = np.zeros((3, 3))
    G[2, 2] = -0.2
    amp = 1e-3 * min(full.L[i] / full.n[i] for i in range(3))
    full.u = full.ctx.affine_field([0, 0, 0], G) + full.mask * inputs.random_coeffs(
        w["seed"], full.n, full.P, amp)
    full.v = inputs.uniform(w["seed"], full.N, -1, 1, stream=3)
    ud = full.dev(full.u, t.float64)
    st = t.empty(full.ctx.nqp * 10, dtype=t.float64, device="cuda")
    R = t.zeros(full.N, dtype=t.float64, device="cuda")
    full.ctx.internal_force(full.mat, FP64, ud, R, state=st, flags=MASK_BC)
    # Near equilibrium the force entries are sums of element contributions
    # that cancel to about 1e-3 of their size: the bound is taken relative to
    # the sum of the absolute element contributions.
    got, ref, scale = full.sample(full.host(R), lambda pb, u, v, m: m * pb.R(u), abs_sum=True)
    assert np.abs(got - ref).max() < TOL64 * scale.max()
    y = t.zeros(full.N, dtype=t.float64, device="cuda")
    full.ctx.tangent_apply(full.mat, FP64, full.dev(full.v, t.float64), y, state=st)
    got, ref, _ = full.sample(full.host(y),
                              lambda pb, u, v, m: pb.mesh.tangent_apply(pb.mu, pb.lam, u, v))
    assert relerr(got, ref) < TOL64


def test_fullsize_mixed_pcg_fused_operator(full):
    # Two iterations of the mixed-precision PCG from x = 0: both run the FP32
    # operator with the fused direction update, and x2 = a0 z0 + a1 (z1 + b0 z0)
    # with z1 = D^-1 (r0 - a0 A z0) depends on every entry of the first
    # operator output.  The oracle runs the same two FP64 CG iterations on the
    # whole mesh (direct element loops).
    t = full.torch
    w = full.w
    G = np.zeros((3, 3))
    G[2, 2] = -0.2
    amp = 1e-3 * min(full.L[i] / full.n[i] for i in range(3))
    u = full.ctx.affine_field([0, 0, 0], G) + full.mask * inputs.random_coeffs(
        w["seed"], full.n, full.P, amp)
    b = full.mask * inputs.uniform(w["seed"], full.N, -1, 1, stream=5)
    x = t.zeros(full.N, dtype=t.float64, device="cuda")
    st = full.ctx.jacobi_pcg(full.mat, FP32, full.dev(b, t.float64), x,
                             u_lin=full.dev(u, t.float64), rtol=1e-30, maxit=2, inner_rtol=1e-30,
                             check=False)
    assert st["iterations"] == 2
    pb, _ = make(full.n, full.L, full.P, kind=w["kind"], E=w["E"], nu=w["nu"],
                 dirichlet=w["dirichlet"])
    assert np.array_equal(pb.mask, full.mask)
    xr, its, _ = osv.pcg(pb.A(u, 0.0), b, pb.diag(u, 0.0), 1e-30, 2)
    assert its == 2
    assert relerr(full.host(x), xr) < TOL32


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_fullsize_masked_mass(full, prec):
    t = full.torch
    w = full.w
    dt = t.float64 if prec == FP64 else t.float32
    v = inputs.uniform(w["seed"], full.N, -1, 1, stream=7)
    if prec == FP32:
        v = v.astype(np.float32).astype(np.float64)
    y = t.zeros(full.N, dtype=dt, device="cuda")
    full.ctx.mass_apply(1.3, prec, full.dev(v, dt), y, flags=MASK_BC)
    keep_v, keep_e = full.v, full.elems
    full.v = v
    col = np.array([(full.n[0] // 2, full.n[1] - 1, ez) for ez in range(full.n[2])])
    full.elems = np.concatenate([keep_e, col])
    try:
        got, ref, _ = full.sample(full.host(y),
                                  lambda pb, u, vv, m: m * pb.mesh.mass_apply(1.3, m * vv))
    finally:
        full.v, full.elems = keep_v, keep_e
    assert relerr(got, ref) < (TOL64 if prec == FP64 else TOL32)


@pytest.mark.parametrize("name", ["compress_p2", "compress_p6", "compress_p8"])
def test_fullsize_sweep_orders(name):
    # the other members of the polynomial-order sweep at their full sizes
    # (94^3, 31^3, 23^3 elements, about 2e7 DOF each): the FP32 masked
    # stored-state tangent (the PCG operator) and the FP64 masked mass on
    # every slot of 8 sampled elements (two of them the mesh's corners)
    f = Full(name, nsample=8)
    t = f.torch
    f32 = t.float32
    u32, v32 = f.u.astype(np.float32), f.v.astype(np.float32)
    st = t.empty(f.ctx.nqp * 10, dtype=f32, device="cuda")
    f.ctx.linearize(f.mat, FP32, f.dev(u32, f32), st)
    y = t.zeros(f.N, dtype=f32, device="cuda")
    f.ctx.tangent_apply(f.mat, FP32, f.dev(v32, f32), y, state=st, flags=MASK_BC)
    del st
    f.u, f.v = u32.astype(np.float64), v32.astype(np.float64)
    got, ref, _ = f.sample(f.host(y), lambda pb, u, v, m: m * pb.mesh.tangent_apply(
        pb.mu, pb.lam, u, m * v))
    assert relerr(got, ref) < TOL32
    ym = t.zeros(f.N, dtype=t.float64, device="cuda")
    f.ctx.mass_apply(0.7, FP64, f.dev(f.v, t.float64), ym, flags=MASK_BC)
    got, ref, _ = f.sample(f.host(ym), lambda pb, u, v, m: m * pb.mesh.mass_apply(0.7, m * v))
    assert relerr(got, ref) < TOL64
    f.ctx.close()
