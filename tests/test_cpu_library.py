"""CPU checks of libsdme: the shared library loads and exports every entry
point declared in include/sdme.h; the host-side basis construction, gather
map, Dirichlet flags and affine-field expansion match the oracle; argument
validation rejects bad input before any device work."""
import os
import re

import numpy as np
import pytest

from oracle import basis as ob
from oracle import solvers as osv
from paper_2104_13466_amd import inputs, sdme
from tests.oracle_setup import make

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "sdme.h")


def test_library_exports_every_declared_symbol():
    import ctypes
    text = open(HEADER).read()
    declared = sorted(set(re.findall(r"\b(sdme_[a-z_0-9]+)\s*\(", text)))
    assert len(declared) >= 25
    L = ctypes.CDLL(sdme.lib_path())
    missing = [d for d in declared if not hasattr(L, d)]
    assert not missing, missing
    # the binding covers every declared symbol
    assert set(declared) <= set(sdme.SIGNATURES), set(declared) - set(sdme.SIGNATURES)


@pytest.mark.parametrize("kind", [ob.NODAL, ob.MODAL, ob.SDME_M, ob.SDME_K, ob.SDME_H])
@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6, 8, 10])
def test_basis_matches_oracle(kind, P):
    Q = P + 2
    t = sdme.basis_build(P, Q, kind, 0.5, 100.0)
    b, x, w, B, D = ob.build(P, Q, kind)
    assert np.abs(t["x"] - x).max() < 1e-15
    assert np.abs(t["w"] - w).max() < 1e-14
    assert np.abs(t["B"] - B).max() < 1e-12
    assert np.abs(t["D"] - D).max() < 1e-11 * max(1.0, np.abs(D).max())
    assert np.abs(t["M1"] - b.M1).max() < 1e-13
    assert np.abs(t["K1"] - b.K1).max() < 1e-11 * max(1.0, np.abs(b.K1).max())
    if kind >= ob.SDME_M and P >= 2:
        assert np.allclose(t["lambda_s"], b.lambda_s, rtol=1e-12)


@pytest.mark.parametrize("kind,k,lam_h", [(ob.SDME_M, 0.0, 100.0), (ob.SDME_M, 1.0, 100.0),
                                           (ob.SDME_K, 0.0, 100.0), (ob.SDME_K, 1.0, 100.0),
                                           (ob.SDME_H, 0.0, 1.0), (ob.SDME_H, 1.0, 400.0),
                                           (ob.SDME_H, 0.5, 1.0), (ob.SDME_H, 0.5, 400.0)])
@pytest.mark.parametrize("P", [2, 4, 6, 8])
def test_basis_parameters_match_oracle(kind, k, lam_h, P):
    # the SD exponent k (Eqs. Y, ParametroK) and the SDME-H weight lambda
    # (Eqs. EffectiveStiffness_lambda, alphaKN) away from the paper's defaults
    Q = P + 2
    t = sdme.basis_build(P, Q, kind, k, lam_h)
    b, x, w, B, D = ob.build(P, Q, kind, k=k, lam=lam_h)
    sc = max(1.0, np.abs(D).max())
    assert np.abs(t["B"] - B).max() < 1e-11 * max(1.0, np.abs(B).max())
    assert np.abs(t["D"] - D).max() < 1e-11 * sc
    assert np.abs(t["M1"] - b.M1).max() < 1e-12 * max(1.0, np.abs(b.M1).max())
    assert np.abs(t["K1"] - b.K1).max() < 1e-11 * max(1.0, np.abs(b.K1).max())
    assert np.allclose(t["lambda_s"], b.lambda_s, rtol=1e-12)
    # the parameter reaches the tables: the internal blocks scale as
    # Lambda^-k (mass) and Lambda^(1-k) (stiffness)
    lm = np.asarray(b.lambda_s)
    assert np.allclose(np.diag(t["M1"])[1:P], lm ** (-k), rtol=1e-10)
    assert np.allclose(np.diag(t["K1"])[1:P], lm ** (1.0 - k), rtol=1e-10)


def test_basis_eval_matches_oracle():
    pts = np.linspace(-1, 1, 23)
    V, dV = sdme.basis_eval(6, ob.SDME_H, pts)
    b = ob.Basis1D(6, ob.SDME_H)
    Vr, dVr = b.eval(pts)
    assert np.abs(V - Vr).max() < 1e-12 and np.abs(dV - dVr).max() < 1e-10


@pytest.mark.parametrize("n,P,bits", [((3, 2, 2), 3, inputs.face_bits(0)),
                                      ((2, 3, 1), 4, inputs.face_bits(4) | inputs.face_bits(5)),
                                      ((1, 1, 2), 2, (1 << 18) - 1)])
def test_host_maps_match_oracle(n, P, bits):
    ctx = sdme.Context(n, (1.0, 2.0, 0.5), P, basis=ob.SDME_H, dirichlet=bits)
    pb, basis = make(n, (1.0, 2.0, 0.5), P, dirichlet=bits)
    assert np.array_equal(ctx.gather_indices(), pb.mesh.gather_map())
    assert np.array_equal(ctx.dirichlet_flags(), (pb.mask == 0).astype(np.uint8))
    G = np.array([[0.1, 0.2, -0.3], [0.05, -0.2, 0.0], [0.3, 0.1, -0.2]])
    a = ctx.affine_field([0.5, -1.0, 2.0], G)
    ref = osv.affine_field(pb.mesh, basis, (0, 0, 0), [0.5, -1.0, 2.0], G)
    assert np.abs(a - ref).max() < 1e-12
    ctx.close()


def test_argument_validation():
    with pytest.raises(sdme.SdmeError) as e:
        sdme.basis_build(0, 2, ob.SDME_H)
    assert e.value.code == -1
    with pytest.raises(sdme.SdmeError):
        sdme.basis_build(4, 4, ob.SDME_H)  # Q < P+1
    with pytest.raises(sdme.SdmeError):
        sdme.Context((2, 2, 2), (1, 1, 1), 9)  # order beyond the compiled kernels
    with pytest.raises(sdme.SdmeError):
        sdme.Context((0, 2, 2), (1, 1, 1), 3)
    with pytest.raises(sdme.SdmeError):
        sdme.Context((2, 2, 2), (1, 1, 1), 3, Q=6)  # only Q = P+2 and P+1 are compiled
    with pytest.raises(sdme.SdmeError):
        sdme.Context((2, 2, 2), (1, 1, 1), 3, Q=3)


@pytest.mark.parametrize("n,P,Q", [((41, 2, 3), 1, None), ((9, 2, 2), 5, 6), ((3, 1, 2), 8, None)])
def test_ordered_assembly_adds_staging_to_the_device_block(n, P, Q):
    # ordered assembly: the device block also holds the staging array, at
    # least one FP64 element vector per element (the diagonal and body load)
    plain = sdme.Context(n, (1.0, 1.0, 1.0), P, Q=Q)
    ordered = sdme.Context(n, (1.0, 1.0, 1.0), P, Q=Q, ordered=True)
    assert ordered.desc.assembly == 1 and plain.desc.assembly == 0
    extra = ordered.context_bytes()[0] - plain.context_bytes()[0]
    assert extra % 256 == 0 and extra >= 8 * 3 * plain.E * (P + 1) ** 3
    assert ordered.context_bytes()[1] == plain.context_bytes()[1]
    # any other assembly mode is refused
    import ctypes
    d = sdme.MeshDesc.from_buffer_copy(plain.desc)
    d.assembly = 2
    h = ctypes.c_void_p()
    assert plain.L.sdme_create(ctypes.byref(d), ctypes.byref(h)) == -1
    plain.close()
    ordered.close()


def test_context_accepts_gll_rule():
    # Q = P+1 selects the Gauss-Lobatto-Legendre volume rule (host-only query)
    c = sdme.Context((2, 1, 1), (1.0, 1.0, 1.0), 3, basis=ob.NODAL, Q=4)
    X = c.quadrature_points()
    # the GLL points include the element end points
    assert abs(X[0, 0, 0]) < 1e-15 and abs(X[0, 0, 3] - 0.5) < 1e-15
    c.close()


def test_lumped_mass_rejects_mass_shifted_operators():
    # the lumped mass is not fused into the mass-shifted tangent: such calls
    # (and Newmark steps) are refused before any device access
    import ctypes
    c = sdme.Context((2, 1, 1), (1.0, 1.0, 1.0), 2, basis=ob.NODAL, lumped_mass=True)
    m = sdme.Material()
    m.mu, m.lam, m.rho = 8, 8, 1.0
    p = ctypes.c_void_p(8)
    rc = c.L.sdme_tangent_apply(c.handle, ctypes.byref(m), 0, None, p, 1.0, p, p, 0, None)
    assert rc == -1
    rc = c.L.sdme_jacobi_diag(c.handle, ctypes.byref(m), 0, p, 1.0, p, 0, None)
    assert rc == -1
    st = sdme.Stats()
    rc = c.L.sdme_newmark_newton_step(c.handle, ctypes.byref(m), 0, p, p, p, None, 1e-3, 0.25,
                                      0.5, 1e-8, 1e-8, 5, 100, ctypes.byref(st), None, 0, None)
    assert rc == -1
    c.close()


def test_size_limits_and_load_argument_checks():
    # 3 Nn must stay below 2^31 (int32 indices in the kernels): a 600^3 mesh
    # at P = 2 (3 x 1201^3 DOF) is refused, 400^3 at P = 2 (3 x 801^3) is not
    with pytest.raises(sdme.SdmeError) as e:
        sdme.Context((600, 600, 600), (1.0, 1.0, 1.0), 2)
    assert e.value.code == -1
    c = sdme.Context((400, 400, 400), (1.0, 1.0, 1.0), 2)
    assert c.Nn == 801 ** 3
    c.close()
    # loads at quadrature points: face index and pointers checked before any
    # device access
    import ctypes
    c = sdme.Context((2, 1, 1), (1.0, 1.0, 1.0), 2)
    p = ctypes.c_void_p(8)
    assert c.L.sdme_face_load(c.handle, 6, p, p, None) == -1
    assert c.L.sdme_face_load(c.handle, -1, p, p, None) == -1
    assert c.L.sdme_body_load(c.handle, None, p, None) == -1
    assert c.L.sdme_l2_error(c.handle, p, None, None, None) == -1
    out = np.zeros(3 * c.E * c.Q ** 3)
    assert c.L.sdme_quadrature_points(c.handle, 7, out.ctypes.data_as(
        ctypes.POINTER(ctypes.c_double))) == -1
    c.close()


def test_bench_refuses_more_than_one_gpu():
    # the benchmark is single-GPU: --gpus N > 1 exits with a message before
    # touching a device
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_context_bytes_and_bind_checks():
    # the caller allocates the context's memory: a size query, then sdme_bind
    # with blocks at least that large (256-byte aligned device block);
    # anything else is refused before the device is touched, and device
    # entry points refuse a context that was never bound
    import ctypes
    c = sdme.Context((5, 2, 2), (1.0, 1.0, 1.0), 3)
    db, hb = c.context_bytes()
    assert db > 0 and db % 256 == 0 and hb >= 2048 + 4
    # tables (volume rule, FP64 + FP32) and per-block partials are inside
    n, Q = 4, 5
    assert db >= 12 * (5 * Q * n + Q + n * n + n)
    big = sdme.Context((40, 60, 60), (1.0, 1.0, 1.0), 3)
    assert big.context_bytes()[0] > db  # partials grow with the block count
    big.close()
    L, h = c.L, c.handle
    p = ctypes.c_void_p(4096)
    assert L.sdme_bind(h, None, db, p, hb, None) == -1
    assert L.sdme_bind(h, p, db, None, hb, None) == -1
    assert L.sdme_bind(h, p, db - 256, p, hb, None) == -1
    assert L.sdme_bind(h, p, db, p, hb - 1, None) == -1
    assert L.sdme_bind(h, ctypes.c_void_p(4096 + 64), db, p, hb, None) == -1
    out_d, out_h = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.sdme_context_bytes(None, ctypes.byref(out_d), ctypes.byref(out_h)) == -1
    assert L.sdme_context_bytes(h, None, ctypes.byref(out_h)) == -1
    # no checked call yet: no element named
    assert c.jac_element() is None
    # unbound: every device entry point returns SDME_EINVAL
    assert L.sdme_mass_apply(h, 1.0, 0, p, p, 0, None) == -1
    m = sdme.Material()
    m.mu, m.lam, m.rho = 8, 8, 1.0
    assert L.sdme_internal_force(h, ctypes.byref(m), 0, p, p, None, 0, None) == -1
    c.close()


def test_binding_validates_device_arguments():
    # dtype against prec, contiguity and length are checked in the binding
    # before any call into the library (then the device: CPU tensors with
    # everything else right are refused as not on the HIP device)
    import torch
    c = sdme.Context((3, 2, 1), (1.0, 1.0, 1.0), 2)
    N = 3 * c.Nn
    d64 = torch.zeros(N, dtype=torch.float64)
    d32 = torch.zeros(N, dtype=torch.float32)
    mu = torch.ones(c.E, dtype=torch.float64)
    with pytest.raises(ValueError, match="HIP device"):
        sdme.Context.material(mu, mu, 1.0)
    with pytest.raises(ValueError, match="dtype"):
        sdme.Context.material(mu.float(), mu, 1.0)
    m = sdme.Material()
    m._keep = (mu, mu)
    with pytest.raises(ValueError, match="dtype"):
        c.mass_apply(1.0, sdme.FP64, d32, d64)
    with pytest.raises(ValueError, match="dtype"):
        c.mass_apply(1.0, sdme.FP32, d64, d32)
    with pytest.raises(ValueError, match="elements"):
        c.mass_apply(1.0, sdme.FP64, d64[:-1], d64)
    with pytest.raises(ValueError, match="contiguous"):
        c.mass_apply(1.0, sdme.FP64, torch.zeros(2 * N, dtype=torch.float64)[::2], d64)
    with pytest.raises(ValueError, match="HIP device"):
        c.mass_apply(1.0, sdme.FP64, d64, d64)
    with pytest.raises(ValueError, match="prec"):
        c.mass_apply(1.0, 7, d64, d64)
    # the per-call length rules: state [E][10][Q^3], per-element arrays [E]
    with pytest.raises(ValueError, match="elements"):
        c._state(torch.zeros(c.nqp * 9, dtype=torch.float64), sdme.FP64)
    with pytest.raises(ValueError, match="dtype"):
        c._state(torch.zeros(c.nqp * 10, dtype=torch.float64), sdme.FP32)
    with pytest.raises(ValueError, match="g_mu"):
        c._e(mu[:-1], "g_mu")
    with pytest.raises(ValueError, match="material"):
        c._mat(sdme.Material())  # not built by Context.material
    bad = sdme.Material()
    bad._keep = (mu[:-1], mu)
    with pytest.raises(ValueError, match="material.mu"):
        c._mat(bad)
    with pytest.raises(ValueError, match="exactly one"):
        c.tangent_apply(m, sdme.FP64, d64, d64)
    # nothing was bound: no device memory was requested by any of these
    assert c._blocks is None
    c.close()
