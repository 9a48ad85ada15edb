"""Pins of the oracle's element operators (Section 3 weak form, Section 4 mass)
against invariants and closed forms: numbering counts printed in the paper,
element mass = tensor product of the 1D mass, zero force under rigid motion,
patch reproduction of homogeneous deformations, consistency of force, tangent
and energy (finite differences), symmetry, the small-strain limit, surface
integrals of constant fields, and brute-force diagonals.  All CPU."""
import os

import numpy as np
import pytest

from oracle import basis as ob
from oracle import fem
from oracle import solvers as osv
from paper_2104_13466_amd import inputs
from tests.oracle_setup import make

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dof_counts.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            kind, P, d = line.split()
            rows.append((kind, int(P), int(d)))
    return rows


@pytest.mark.parametrize("row", _golden())
def test_dof_counts_printed_in_paper(row):
    kind, P, dofs = row
    pb, _ = make((2, 2, 2), (1, 1, 1), P, dirichlet=inputs.face_bits(0))
    mesh = pb.mesh
    free = int(pb.mask.sum())
    if kind == "static":
        assert free == dofs
    else:
        # remove the element-interior modes (all three tensor indices internal)
        interior = 3 * mesh.E * (P - 1) ** 3
        assert free - interior == dofs


@pytest.mark.parametrize("n,P", [((1, 1, 1), 1), ((2, 3, 2), 2), ((3, 2, 2), 4)])
def test_gather_map_structure(n, P):
    pb, _ = make(n, (1, 1, 1), P)
    mesh = pb.mesh
    g = mesh.gather_map()
    nl = (P + 1) ** 3
    assert g.shape == (mesh.E, nl)
    # distinct slots within an element; every slot used; multiplicity = number of
    # elements touching the slot's entity (1 interior, 2 face, 4 edge, 8 vertex)
    for e in range(mesh.E):
        assert len(set(g[e])) == nl
    counts = np.bincount(g.ravel(), minlength=mesh.Nn)
    assert counts.min() >= 1
    ix = np.arange(mesh.Nn) % mesh.Nx
    iy = (np.arange(mesh.Nn) // mesh.Nx) % mesh.Ny
    iz = np.arange(mesh.Nn) // (mesh.Nx * mesh.Ny)
    mult = np.ones(mesh.Nn, dtype=int)
    for idx, N in ((ix, mesh.Nx), (iy, mesh.Ny), (iz, mesh.Nz)):
        shared = (idx % P == 0) & (idx > 0) & (idx < N - 1)
        mult *= np.where(shared, 2, 1)
    assert np.array_equal(counts, mult)
    # anchor coordinates of element mode (a,b,c) = element corner + (a,b,c)
    for e in range(mesh.E):
        ex, ey, ez = e % n[0], (e // n[0]) % n[1], e // (n[0] * n[1])
        for l in range(nl):
            a, b, c = l % (P + 1), (l // (P + 1)) % (P + 1), l // (P + 1) ** 2
            s = g[e, l]
            assert (s % mesh.Nx, (s // mesh.Nx) % mesh.Ny, s // (mesh.Nx * mesh.Ny)) == \
                (ex * P + a, ey * P + b, ez * P + c)


@pytest.mark.parametrize("P,kind", [(2, ob.MODAL), (3, ob.SDME_M), (4, ob.NODAL), (3, ob.SDME_H)])
def test_element_mass_is_tensor_product(P, kind):
    # affine hexahedron: M_e = rho detJ M1 (x) M1 (x) M1 with M1 the 1D mass
    h = (0.5, 0.25, 2.0)
    pb, basis = make((1, 1, 1), h, P, kind=kind)
    mesh = pb.mesh
    rho = 2.5
    n3 = (P + 1) ** 3
    Me = np.zeros((n3, n3))
    for j in range(n3):
        v = np.zeros(3 * mesh.Nn)
        v[j] = 1.0
        Me[:, j] = mesh.mass_apply(rho, v)[:n3]
    ref = rho * np.prod(h) / 8 * np.kron(basis.M1, np.kron(basis.M1, basis.M1))
    assert np.abs(Me - ref).max() < 1e-13 * np.abs(ref).max()
    if kind == ob.SDME_M:  # interior block diagonal and decoupled
        inner = [l for l in range(n3) if all(0 < t < P for t in
                                              (l % (P + 1), (l // (P + 1)) % (P + 1), l // (P + 1) ** 2))]
        for l in inner:
            row = Me[l].copy()
            row[l] = 0.0
            assert np.abs(row).max() < 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("P,kind", [(1, ob.MODAL), (3, ob.SDME_H), (4, ob.SDME_M)])
def test_rigid_motion_zero_force(P, kind):
    pb, basis = make((2, 2, 1), (1.0, 1.0, 0.5), P, kind=kind)
    for th, axis in ((0.3, 2), (1.1, 0), (2.5, 1)):
        c, s = np.cos(th), np.sin(th)
        i, j = [k for k in range(3) if k != axis]
        Rm = np.eye(3)
        Rm[i, i], Rm[i, j], Rm[j, i], Rm[j, j] = c, -s, s, c
        u = osv.affine_field(pb.mesh, basis, (0, 0, 0), (0.3, -0.2, 0.7), Rm - np.eye(3))
        R = pb.R(u)
        # scale: force of a 1% stretch
        ref = pb.R(osv.affine_field(pb.mesh, basis, (0, 0, 0), (0, 0, 0), 0.01 * np.eye(3)))
        assert np.abs(R).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("P,kind", [(2, ob.SDME_H), (3, ob.SDME_M), (4, ob.NODAL)])
def test_patch_homogeneous_deformation(P, kind):
    # constant F solves Div P = 0, so the force at every interior DOF vanishes
    pb, basis = make((2, 2, 2), (1.0, 1.0, 1.0), P, kind=kind, dirichlet=(1 << 18) - 1)
    G = np.array([[0.15, 0.05, 0.0], [-0.02, -0.1, 0.03], [0.04, 0.0, 0.25]])
    u = osv.affine_field(pb.mesh, basis, (0, 0, 0), (0.1, 0, 0), G)
    R = pb.R(u)
    assert np.abs(pb.mask * R).max() < 1e-12 * np.abs(R).max()


def _rand_state(pb, seed, amp):
    return pb.mask * inputs.random_coeffs(seed, (pb.mesh.nx, pb.mesh.ny, pb.mesh.nz), pb.mesh.P, amp)


@pytest.mark.parametrize("P", [2, 3])
def test_force_is_energy_gradient(P):
    pb, _ = make((2, 1, 1), (1.0, 0.5, 0.5), P, dirichlet=inputs.face_bits(0))
    u = _rand_state(pb, 11, 0.02)
    v = inputs.uniform(12, u.size, -1, 1)
    eps = 1e-6
    dE = (pb.mesh.strain_energy(pb.mu, pb.lam, u + eps * v) -
          pb.mesh.strain_energy(pb.mu, pb.lam, u - eps * v)) / (2 * eps)
    assert abs(dE - v @ pb.R(u)) < 1e-7 * abs(dE)


@pytest.mark.parametrize("P,amp", [(2, 0.05), (3, 0.01), (4, 0.001)])
def test_tangent_is_force_derivative(P, amp):
    pb, _ = make((2, 1, 1), (1.0, 0.5, 0.5), P)
    u = inputs.random_coeffs(21, (2, 1, 1), P, amp)
    v = inputs.uniform(22, u.size, -1, 1)
    eps = 1e-6
    fd = (pb.R(u + eps * v) - pb.R(u - eps * v)) / (2 * eps)
    Kv = pb.mesh.tangent_apply(pb.mu, pb.lam, u, v)
    assert np.abs(fd - Kv).max() < 1e-8 * np.abs(Kv).max()


def test_tangent_symmetric_and_mass_shift():
    pb, _ = make((2, 2, 1), (1.0, 1.0, 0.5), 3)
    u = inputs.random_coeffs(31, (2, 2, 1), 3, 0.05)
    v = inputs.uniform(32, u.size, -1, 1)
    w = inputs.uniform(33, u.size, -1, 1)
    Kv = pb.mesh.tangent_apply(pb.mu, pb.lam, u, v)
    Kw = pb.mesh.tangent_apply(pb.mu, pb.lam, u, w)
    assert abs(w @ Kv - v @ Kw) < 1e-13 * abs(w @ Kv) + 1e-13 * np.abs(Kv).max()
    cm = 7.0
    Kv2 = pb.mesh.tangent_apply(pb.mu, pb.lam, u, v, cm)
    assert np.abs(Kv2 - Kv - pb.mesh.mass_apply(cm, v)).max() < 1e-12 * np.abs(Kv2).max()


def test_small_strain_limit_is_linear_elasticity():
    # K_T(0) on affine fields with constant strains G1, G2:
    # w^T K v = Vol (lam tr G1 tr G2 + 2 mu sym(G1):sym(G2))
    L = (1.0, 0.75, 0.5)
    pb, basis = make((2, 2, 2), L, 3)
    lam0, mu0 = pb.lam[0], pb.mu[0]
    G1 = np.array([[0.3, 0.1, -0.2], [0.0, 0.5, 0.4], [0.7, -0.3, 0.2]])
    G2 = np.array([[-0.1, 0.6, 0.2], [0.3, 0.2, 0.0], [0.1, 0.5, -0.4]])
    v = osv.affine_field(pb.mesh, basis, (0, 0, 0), (0, 0, 0), G1)
    w = osv.affine_field(pb.mesh, basis, (0, 0, 0), (0, 0, 0), G2)
    Kv = pb.mesh.tangent_apply(pb.mu, pb.lam, np.zeros_like(v), v)
    e1, e2 = 0.5 * (G1 + G1.T), 0.5 * (G2 + G2.T)
    ref = np.prod(L) * (lam0 * np.trace(G1) * np.trace(G2) + 2 * mu0 * np.sum(e1 * e2))
    assert abs(w @ Kv - ref) < 1e-12 * abs(ref)


def test_mass_of_affine_field_closed_form():
    # v = (1, x, 0): v^T M v = rho int (1 + x^2) dV over [0,Lx]x[0,Ly]x[0,Lz]
    L = (2.0, 1.0, 0.5)
    pb, basis = make((3, 2, 2), L, 4, kind=ob.SDME_M, rho=3.0)
    G = np.zeros((3, 3))
    G[1, 0] = 1.0
    v = osv.affine_field(pb.mesh, basis, (0, 0, 0), (1.0, 0, 0), G)
    ref = 3.0 * (L[0] + L[0] ** 3 / 3) * L[1] * L[2]
    assert abs(v @ pb.mesh.mass_apply(3.0, v) - ref) < 1e-12 * ref


@pytest.mark.parametrize("P,kind", [(2, ob.MODAL), (3, ob.SDME_H)])
def test_diagonal_brute_force(P, kind):
    pb, _ = make((2, 1, 1), (1.0, 0.5, 0.5), P, kind=kind)
    u = inputs.random_coeffs(41, (2, 1, 1), P, 0.05)
    cm = 3.0
    d = pb.mesh.tangent_diag(pb.mu, pb.lam, u, cm)
    N = u.size
    for j in range(0, N, max(1, N // 40)):
        e = np.zeros(N)
        e[j] = 1.0
        assert abs(pb.mesh.tangent_apply(pb.mu, pb.lam, u, e, cm)[j] - d[j]) < 1e-12 * abs(d[j])


def test_face_traction_and_penalty_closed_forms():
    L = (1.0, 2.0, 0.5)
    P = 3
    pb, basis = make((2, 3, 1), L, P, kind=ob.SDME_M)
    xf, wf = ob.gauss_legendre(P + 1)
    Bf, _ = basis.eval(xf)
    ones_z = osv.affine_field(pb.mesh, basis, (0, 0, 0), (0, 0, 1.0), np.zeros((3, 3)))
    ones_x = osv.affine_field(pb.mesh, basis, (0, 0, 0), (1.0, 0, 0), np.zeros((3, 3)))
    # dead traction on face x=max: w^T f = t . w * area
    f = pb.mesh.vec()
    pb.mesh.face_traction(1, [2.0, 0.0, -3.0], Bf, wf, f)
    area = L[1] * L[2]
    assert abs(ones_z @ f + 3.0 * area) < 1e-12 * area
    assert abs(ones_x @ f - 2.0 * area) < 1e-12 * area
    # uniform penetration delta into the plane z=0: energy eps/2 delta^2 A,
    # force eps delta A in +z
    delta, eps = 0.01, 5.0e4
    u = -delta * ones_z
    f = pb.mesh.vec()
    en = pb.mesh.penalty_plane(eps, 0.0, 0.0, Bf, wf, u, f)
    A = L[0] * L[1]
    assert abs(en - 0.5 * eps * delta ** 2 * A) < 1e-12 * en
    assert abs(ones_z @ f - eps * delta * A) < 1e-12 * eps * delta * A
    assert np.abs(ones_x @ f) < 1e-12


def test_material_gradient_is_force_sensitivity():
    pb, _ = make((2, 2, 1), (1.0, 1.0, 0.5), 2)
    u = inputs.random_coeffs(51, (2, 2, 1), 2, 0.05)
    wv = inputs.uniform(52, u.size, -1, 1)
    gm = np.zeros(pb.mesh.E)
    gl = np.zeros(pb.mesh.E)
    pb.mesh.material_grad(u, wv, 1.0, gm, gl)
    for e in range(pb.mesh.E):
        for arr, g in ((pb.mu, gm), (pb.lam, gl)):
            h = 1e-4 * arr[e]
            arr[e] += h
            Rp = pb.R(u)
            arr[e] -= 2 * h
            Rm = pb.R(u)
            arr[e] += h
            fd = wv @ (Rp - Rm) / (2 * h)
            assert abs(fd - g[e]) < 1e-7 * max(abs(fd), 1e-3 * np.abs(gm).max())


@pytest.mark.parametrize("P,kind", [(1, ob.MODAL), (3, ob.SDME_H), (4, ob.NODAL)])
def test_strain_energy_vanishes_at_reference_and_under_rotation(P, kind):
    # Section 3, hyperelastic strain energy: Psi(F = I) = 0 exactly, and the
    # energy is frame-indifferent, so a rigid rotation stores none either
    pb, basis = make((2, 2, 1), (1.0, 1.0, 0.5), P, kind=kind)
    assert pb.mesh.strain_energy(pb.mu, pb.lam, np.zeros(3 * pb.mesh.Nn)) == 0.0
    th = 0.7
    Rm = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0, 0, 1.0]])
    u = osv.affine_field(pb.mesh, basis, (0, 0, 0), (0.2, -0.1, 0.3), Rm - np.eye(3))
    # scale: energy of a 1% stretch (about 1e-4 mu V)
    ref = pb.mesh.strain_energy(pb.mu, pb.lam, osv.affine_field(
        pb.mesh, basis, (0, 0, 0), (0, 0, 0), np.diag([0.01, 0.0, 0.0])))
    assert abs(pb.mesh.strain_energy(pb.mu, pb.lam, u)) < 1e-10 * ref


@pytest.mark.parametrize("s", [0.8, 1.0 + 1e-3, 1.3])
def test_strain_energy_of_uniaxial_stretch_closed_form(s):
    # F = diag(s, 1, 1): tr C - 3 = s^2 - 1 and J = s, so the stored energy of
    # a body of volume V is V [mu/2 (s^2 - 1) - mu ln s + lam/2 (ln s)^2];
    # per-element Lame parameters enter element by element
    L = (1.0, 0.5, 0.25)
    n = (3, 2, 1)
    pb, basis = make(n, L, 3, kind=ob.SDME_M)
    rng = np.random.default_rng(5)
    mu = 300.0 + 200.0 * rng.random(pb.mesh.E)
    lam = 400.0 + 300.0 * rng.random(pb.mesh.E)
    u = osv.affine_field(pb.mesh, basis, (0, 0, 0), (0.05, 0.0, -0.02),
                         np.diag([s - 1.0, 0.0, 0.0]))
    Ve = np.prod(L) / pb.mesh.E
    ls = np.log(s)
    ref = Ve * np.sum(0.5 * mu * (s * s - 1.0) - mu * ls + 0.5 * lam * ls * ls)
    # tr C - 3 cancels near s = 1: rounding of order eps mu V on top of the
    # relative bound
    assert abs(pb.mesh.strain_energy(mu, lam, u) - ref) < 1e-12 * abs(ref) + 1e-13 * Ve * mu.sum()


def test_strain_energy_small_strain_limit():
    # linear-elastic limit of the neo-Hookean energy: for u = t G X,
    # Pi / t^2 -> V (lam/2 (tr G)^2 + mu |sym G|^2) with an O(t) remainder
    L = (1.0, 0.75, 0.5)
    pb, basis = make((2, 1, 1), L, 2)
    lam0, mu0 = pb.lam[0], pb.mu[0]
    G = np.array([[0.3, 0.1, -0.2], [0.0, 0.5, 0.4], [0.7, -0.3, 0.2]])
    eps = 0.5 * (G + G.T)
    ref = np.prod(L) * (0.5 * lam0 * np.trace(G) ** 2 + mu0 * np.sum(eps * eps))
    for t, tol in ((1e-3, 5e-3), (1e-4, 5e-4)):
        u = osv.affine_field(pb.mesh, basis, (0, 0, 0), (0, 0, 0), t * G)
        assert abs(pb.mesh.strain_energy(pb.mu, pb.lam, u) / t ** 2 - ref) < tol * ref
