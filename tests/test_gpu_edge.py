"""GPU edge cases against the FP64 oracle: single-element meshes (one element
in a block sized for several, so most of the block is idle and every slot lies
on a tile face), a mesh whose every DOF is constrained, a zero right-hand side
and a zero field (the undeformed state).  Tolerances as in the operator
parity tests: 1e-12 (FP64) and 1e-5 (FP32) relative in the max norm."""
import numpy as np
import pytest

from oracle import basis as ob
from paper_2104_13466_amd import inputs
from paper_2104_13466_amd.sdme import FP32, FP64, MASK_BC
from tests.gpu_setup import Pair, relerr

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
ALL_FACES = 0
for _f in range(6):
    ALL_FACES |= inputs.face_bits(_f)


@pytest.mark.parametrize("P,kind", [(1, ob.MODAL), (2, ob.SDME_M), (4, ob.SDME_H),
                                    (6, ob.NODAL), (8, ob.SDME_K)])
def test_single_element(P, kind):
    mu, lam = inputs.lognormal_lame(300 + P, 1, 1.0e3, 0.3)
    p = Pair((1, 1, 1), (0.5, 0.8, 1.1), P, kind=kind, dirichlet=inputs.face_bits(4), mu=mu,
             lam=lam, rho=0.9)
    u = p.rand(11, 0.004)
    v = inputs.uniform(12, p.N, -1, 1, stream=3)
    ud = p.dev(u)
    # internal force with state, FP64 and FP32
    st = p.empty_state()
    R = p.zeros()
    p.ctx.internal_force(p.mat, FP64, ud, R, state=st)
    assert relerr(p.host(R), p.pb.R(u)) < TOL64
    f32 = p.torch.float32
    u32 = u.astype(np.float32)
    R32 = p.zeros(f32)
    p.ctx.internal_force(p.mat, FP32, p.dev(u32, f32), R32)
    assert relerr(p.host(R32), p.pb.R(u32.astype(np.float64))) < TOL32
    # tangent: stored state, recomputed, masked
    ref = p.pb.mesh.tangent_apply(p.pb.mu, p.pb.lam, u, v, 7.0 * p.rho)
    for kw in ({"state": st}, {"u_lin": ud}):
        y = p.zeros()
        p.ctx.tangent_apply(p.mat, FP64, p.dev(v), y, mass_shift=7.0, **kw)
        assert relerr(p.host(y), ref) < TOL64
    y = p.zeros()
    p.ctx.tangent_apply(p.mat, FP64, p.dev(v), y, state=st, mass_shift=7.0, flags=MASK_BC)
    m = p.mask
    refm = m * p.pb.mesh.tangent_apply(p.pb.mu, p.pb.lam, u, m * v, 7.0 * p.rho)
    assert relerr(p.host(y), refm) < TOL64
    # mass and Jacobi diagonal
    y = p.zeros()
    p.ctx.mass_apply(1.3, FP64, p.dev(v), y)
    assert relerr(p.host(y), p.pb.mesh.mass_apply(1.3, v)) < TOL64
    d = p.zeros()
    p.ctx.jacobi_diag(p.mat, FP64, st, 7.0, d)
    assert relerr(p.host(d), p.pb.mesh.tangent_diag(p.pb.mu, p.pb.lam, u, 7.0 * p.rho)) < TOL64
    # strain energy
    e = p.ctx.strain_energy(p.mat, ud)
    eref = p.pb.mesh.strain_energy(p.pb.mu, p.pb.lam, u)
    assert abs(e - eref) < 1e-11 * abs(eref)


def test_zero_field_is_stress_free():
    # undeformed state: zero force, zero energy, tangent = small-strain form
    p = Pair((5, 2, 2), (1.0, 0.4, 0.4), 3, kind=ob.SDME_H, dirichlet=inputs.face_bits(0))
    R = p.zeros()
    st = p.empty_state()
    p.ctx.internal_force(p.mat, FP64, p.zeros(), R, state=st)
    assert np.abs(p.host(R)).max() == 0.0
    assert p.ctx.strain_energy(p.mat, p.zeros()) == 0.0
    v = inputs.uniform(13, p.N, -1, 1)
    y = p.zeros()
    p.ctx.tangent_apply(p.mat, FP64, p.dev(v), y, state=st)
    ref = p.pb.mesh.tangent_apply(p.pb.mu, p.pb.lam, np.zeros(p.N), v)
    assert relerr(p.host(y), ref) < TOL64


def test_every_dof_constrained():
    # P = 1 on a 2x1x1 box: every node lies on the boundary; all faces clamped
    p = Pair((2, 1, 1), (1.0, 0.5, 0.5), 1, kind=ob.MODAL, dirichlet=ALL_FACES)
    assert p.mask.max() == 0.0
    assert np.array_equal(p.ctx.dirichlet_flags(), np.ones(p.N, dtype=np.uint8))
    u = p.rand(14, 0.004)
    ud = p.dev(u)
    R = p.zeros()
    st = p.empty_state()
    p.ctx.internal_force(p.mat, FP64, ud, R, state=st, flags=MASK_BC)
    assert np.abs(p.host(R)).max() == 0.0
    y = p.zeros()
    p.ctx.tangent_apply(p.mat, FP64, p.dev(inputs.uniform(15, p.N, -1, 1)), y, state=st,
                        flags=MASK_BC)
    assert np.abs(p.host(y)).max() == 0.0
    d = p.zeros()
    p.ctx.jacobi_diag(p.mat, FP64, st, 0.0, d, flags=MASK_BC)
    assert np.array_equal(p.host(d), np.ones(p.N))
    # nothing to solve: the masked right-hand side is zero
    for prec in (FP64, FP32):
        x = p.zeros()
        s = p.ctx.jacobi_pcg(p.mat, prec, p.dev(inputs.uniform(16, p.N, -1, 1)), x, u_lin=ud)
        assert s["iterations"] == 0 and s["rel_residual"] == 0.0
        assert np.abs(p.host(x)).max() == 0.0


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_zero_right_hand_side(prec):
    p = Pair((3, 2, 2), (1.0, 1.0, 1.0), 2, kind=ob.SDME_H, dirichlet=inputs.face_bits(0))
    x = p.zeros()
    s = p.ctx.jacobi_pcg(p.mat, prec, p.zeros(), x, u_lin=p.dev(p.mask * p.rand(17, 1e-3)))
    assert s["iterations"] == 0 and s["rel_residual"] == 0.0
    assert np.abs(p.host(x)).max() == 0.0


# Status codes of the C ABI forced from the host: each run ends normally on
# the device and reports its condition as a return value.
def test_status_inverted_element_with_check_jac():
    from paper_2104_13466_amd.sdme import CHECK_JAC, SdmeError
    p = Pair((4, 2, 1), (1.0, 0.5, 0.5), 3, kind=ob.SDME_H, dirichlet=inputs.face_bits(0))
    # F = diag(-0.5, 1, 1): every Gauss point has det F < 0
    u = p.ctx.affine_field([0.0, 0.0, 0.0], np.diag([-1.5, 0.0, 0.0]))
    ud = p.dev(u)
    R = p.zeros()
    with pytest.raises(SdmeError) as e:
        p.ctx.internal_force(p.mat, FP64, ud, R, flags=CHECK_JAC)
    assert e.value.code == -5
    st = p.empty_state()
    with pytest.raises(SdmeError) as e:
        p.ctx.linearize(p.mat, FP64, ud, st, flags=CHECK_JAC)
    assert e.value.code == -5
    y = p.zeros()
    with pytest.raises(SdmeError) as e:
        p.ctx.tangent_apply(p.mat, FP64, p.zeros(), y, u_lin=ud, flags=CHECK_JAC)
    assert e.value.code == -5
    s = p.ctx.jacobi_pcg(p.mat, FP64, p.dev(inputs.uniform(3, p.N, -1, 1)), p.zeros(), u_lin=ud,
                         check=False)
    assert s["status"] == -5
    assert p.ctx.jac_element() == 0  # every element is inverted: the first is named
    # the flag is cleared by the next checked call: a valid state passes
    p.ctx.internal_force(p.mat, FP64, p.dev(p.mask * p.rand(4, 1e-3)), R, flags=CHECK_JAC)
    assert p.ctx.jac_element() is None


@pytest.mark.parametrize("corner", ["first", "last"])
def test_jac_element_names_the_inverted_element(corner):
    # Lagrange-GLL basis at P = 2: the slot at a corner of the box is a node
    # whose shape function lives in the corner element only.  Pushing that
    # node across the element (5 h inwards along every axis) inverts that
    # element and no other; the checked calls report it by index.
    from paper_2104_13466_amd.sdme import CHECK_JAC, SdmeError
    p = Pair((4, 3, 2), (1.0, 0.75, 0.5), 2, kind=ob.NODAL)
    h = np.array([1.0 / 4, 0.75 / 3, 0.5 / 2])
    Nx, Ny, Nz = (4 * 2 + 1, 3 * 2 + 1, 2 * 2 + 1)
    Nn = Nx * Ny * Nz
    u = np.zeros(p.N)
    if corner == "first":
        slot, sign, expect = 0, 1.0, 0
    else:
        slot, sign, expect = Nn - 1, -1.0, 4 * 3 * 2 - 1
    for c in range(3):
        u[c * Nn + slot] = sign * 5.0 * h[c]
    ud = p.dev(u)
    R = p.zeros()
    with pytest.raises(SdmeError) as e:
        p.ctx.internal_force(p.mat, FP64, ud, R, flags=CHECK_JAC)
    assert e.value.code == -5
    assert p.ctx.jac_element() == expect
    with pytest.raises(SdmeError):
        p.ctx.tangent_apply(p.mat, FP32, p.dev(inputs.uniform(5, p.N, -1, 1), p.torch.float32),
                            p.zeros(p.torch.float32), u_lin=p.dev(u, p.torch.float32),
                            flags=CHECK_JAC)
    assert p.ctx.jac_element() == expect


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_status_iteration_limit(prec):
    p = Pair((4, 2, 2), (1.0, 0.5, 0.5), 3, kind=ob.SDME_H, dirichlet=inputs.face_bits(0))
    ud = p.dev(p.mask * p.rand(5, 1e-3))
    b = p.dev(inputs.uniform(6, p.N, -1, 1))
    s = p.ctx.jacobi_pcg(p.mat, prec, b, p.zeros(), u_lin=ud, rtol=1e-10, maxit=1, check=False)
    assert s["status"] == -6 and s["iterations"] == 1
    assert s["rel_residual"] > 1e-10
    # the same solve with room to converge
    s = p.ctx.jacobi_pcg(p.mat, prec, b, p.zeros(), u_lin=ud, rtol=1e-10, check=False)
    assert s["status"] == 0 and s["rel_residual"] <= 1e-10


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_status_breakdown_negative_definite(prec):
    # K_T + s M with a large negative mass shift is negative definite: the
    # first p^T A p is negative and CG reports breakdown
    p = Pair((4, 2, 2), (1.0, 0.5, 0.5), 2, kind=ob.SDME_H, dirichlet=inputs.face_bits(0))
    ud = p.dev(p.mask * p.rand(7, 1e-3))
    b = p.dev(inputs.uniform(8, p.N, -1, 1))
    s = p.ctx.jacobi_pcg(p.mat, prec, b, p.zeros(), u_lin=ud, mass_shift=-1e9, check=False)
    assert s["status"] == -7


def test_binding_refuses_mismatched_device_tensors():
    # device tensors whose dtype, length or layout does not match the call
    # are refused by the binding before any launch; the outputs stay as they
    # were
    p = Pair((3, 2, 1), (1.0, 0.5, 0.5), 2, kind=ob.SDME_H)
    torch = p.torch
    v64 = p.dev(inputs.uniform(9, p.N, -1, 1))
    y = p.zeros()
    with pytest.raises(ValueError, match="dtype"):
        p.ctx.mass_apply(1.0, FP32, v64, y)
    with pytest.raises(ValueError, match="elements"):
        p.ctx.mass_apply(1.0, FP64, v64[:-3], y)
    with pytest.raises(ValueError, match="contiguous"):
        p.ctx.mass_apply(1.0, FP64, torch.zeros(2 * p.N, dtype=torch.float64,
                                                device="cuda")[::2], y)
    with pytest.raises(ValueError, match="elements"):
        p.ctx.linearize(p.mat, FP64, v64, torch.zeros(p.ctx.nqp * 9, dtype=torch.float64,
                                                      device="cuda"))
    short = Pair((3, 2, 1), (1.0, 0.5, 0.5), 2, kind=ob.SDME_H)
    short.mu_t = short.mu_t[:-1].contiguous()
    mat = p.ctx.material(short.mu_t, p.lam_t, 1.0)
    with pytest.raises(ValueError, match="material.mu"):
        p.ctx.internal_force(mat, FP64, v64, y)
    assert np.abs(p.host(y)).max() == 0.0
    # a valid call still runs
    p.ctx.mass_apply(1.0, FP64, v64, y)
    assert relerr(p.host(y), p.pb.mesh.mass_apply(1.0, p.host(v64))) < TOL64
