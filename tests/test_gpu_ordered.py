"""Ordered assembly (element outputs staged, then summed per slot in
ascending element order) against the FP64 oracle and against itself: every
operator within the parity tolerances of the atomic path (1e-12 FP64, 1e-5
FP32, relative in the max norm), every repeated call bit for bit the same,
and whole solves (Jacobi-PCG in both precisions, the static Newton driver,
explicit steps with contact) repeating their iterates exactly.  Meshes whose
x-rows span several element blocks with a ragged last block, and several
element rows in y and z, so that the gather meets slots shared by up to
eight tiles."""
import numpy as np
import pytest

from oracle import basis as ob
from oracle import solvers as osv
from paper_2104_13466_amd import inputs
from paper_2104_13466_amd.sdme import FP32, FP64, MASK_BC
from tests.gpu_setup import Pair, relerr

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5

CASES = [
    ((41, 2, 3), 1, ob.MODAL, None),
    ((37, 3, 2), 2, ob.SDME_H, None),
    ((17, 2, 2), 4, ob.SDME_M, None),
    ((9, 2, 2), 5, ob.NODAL, 6),
    ((5, 2, 2), 7, ob.SDME_K, None),
]
IDS = ["P%d-%s%s" % (c[1], ob.KIND_NAMES[c[2]], "-gll" if c[3] else "") for c in CASES]
BITS = inputs.face_bits(0) | inputs.face_bits(3) | inputs.face_bits(5)


@pytest.fixture(scope="module", params=CASES, ids=IDS)
def pair(request):
    n, P, kind, Q = request.param
    mu, lam = inputs.lognormal_lame(500 + P, n[0] * n[1] * n[2], 1.0e3, 0.3)
    return Pair(n, (2.0, 0.5, 0.75), P, kind=kind, dirichlet=BITS, mu=mu, lam=lam, rho=1.1, Q=Q,
                ordered=True)


def twice(fn):
    """Run fn (which returns a device tensor) twice; both results, on the host."""
    a = fn()
    b = fn()
    return a, b


def same_bits(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_force_and_tangent(pair):
    u = pair.mask * pair.rand(11, 0.004)
    ud = pair.dev(u)
    st = pair.empty_state()

    def force():
        R = pair.zeros()
        pair.ctx.internal_force(pair.mat, FP64, ud, R, state=st)
        return pair.host(R)

    r1, r2 = twice(force)
    assert relerr(r1, pair.pb.R(u)) < TOL64
    assert same_bits(r1, r2)
    u32 = u.astype(np.float32)
    R32 = pair.zeros(pair.torch.float32)
    pair.ctx.internal_force(pair.mat, FP32, pair.dev(u32, pair.torch.float32), R32)
    assert relerr(pair.host(R32), pair.pb.R(u32.astype(np.float64))) < TOL32
    v = inputs.uniform(12, pair.N, -1, 1)
    vd = pair.dev(v)
    m = pair.mask
    ref = m * pair.pb.mesh.tangent_apply(pair.pb.mu, pair.pb.lam, u, m * v, 3.0 * pair.rho)
    for kw in ({"state": st}, {"u_lin": ud}):
        def tan():
            y = pair.zeros()
            pair.ctx.tangent_apply(pair.mat, FP64, vd, y, mass_shift=3.0, flags=MASK_BC, **kw)
            return pair.host(y)
        y1, y2 = twice(tan)
        assert relerr(y1, ref) < TOL64
        assert same_bits(y1, y2)
    st32 = pair.empty_state(pair.torch.float32)
    pair.ctx.linearize(pair.mat, FP32, pair.dev(u32, pair.torch.float32), st32)
    y32 = pair.zeros(pair.torch.float32)
    pair.ctx.tangent_apply(pair.mat, FP32, pair.dev(v, pair.torch.float32), y32, state=st32,
                           mass_shift=3.0, flags=MASK_BC)
    ref32 = m * pair.pb.mesh.tangent_apply(pair.pb.mu, pair.pb.lam, u32.astype(np.float64),
                                           m * v.astype(np.float32).astype(np.float64),
                                           3.0 * pair.rho)
    assert relerr(pair.host(y32), ref32) < TOL32


def test_mass_and_diagonal(pair):
    v = inputs.uniform(13, pair.N, -1, 1)
    vd = pair.dev(v)

    def mass():
        y = pair.zeros()
        pair.ctx.mass_apply(1.3, FP64, vd, y)
        return pair.host(y)

    y1, y2 = twice(mass)
    assert relerr(y1, pair.pb.mesh.mass_apply(1.3, v)) < TOL64
    assert same_bits(y1, y2)
    y32 = pair.zeros(pair.torch.float32)
    pair.ctx.mass_apply(1.3, FP32, pair.dev(v, pair.torch.float32), y32)
    assert relerr(pair.host(y32),
                  pair.pb.mesh.mass_apply(1.3, v.astype(np.float32).astype(np.float64))) < TOL32
    u = pair.mask * pair.rand(14, 0.004)
    st = pair.empty_state()
    pair.ctx.linearize(pair.mat, FP64, pair.dev(u), st)

    def diag():
        d = pair.zeros()
        pair.ctx.jacobi_diag(pair.mat, FP64, st, 2.0, d)
        return pair.host(d)

    d1, d2 = twice(diag)
    assert relerr(d1, pair.pb.mesh.tangent_diag(pair.pb.mu, pair.pb.lam, u, 2.0 * pair.rho)) < TOL64
    assert same_bits(d1, d2)


def test_loads_and_surface_terms(pair):
    from oracle import fabricated as fb
    m = pair.pb.mesh
    shape = (3, m.E, m.Q ** 3)
    b = inputs.uniform(15, int(np.prod(shape)), -1, 1).reshape(shape)
    f = pair.zeros()
    pair.ctx.body_load(pair.dev(b), f)
    assert relerr(pair.host(f), fb.body_load(m, b)) < TOL64
    xf, wf = ob.gauss_legendre(m.P + 1)
    Bf, _ = pair.basis.eval(xf)
    for face in (0, 3, 4):
        fshape = (3, pair.ctx.face_elements(face), (m.P + 1) ** 2)
        t = inputs.uniform(16 + face, int(np.prod(fshape)), -1, 1).reshape(fshape)
        f0 = inputs.uniform(30, pair.N, -1, 1)
        f = pair.dev(f0)
        pair.ctx.face_load(face, pair.dev(t), f)
        assert relerr(pair.host(f), f0 + fb.face_load(m, face, Bf, t)) < TOL64
        f = pair.zeros()
        pair.ctx.face_traction(face, [1.5, -2.0, 0.25], f)
        ref = m.vec()
        m.face_traction(face, [1.5, -2.0, 0.25], Bf, wf, ref)
        assert relerr(pair.host(f), ref) < TOL64
    u = pair.rand(17, 0.02)
    f = pair.zeros()
    pair.ctx.penalty_plane(3.0e4, 0.01, pair.dev(u), f)
    ref = m.vec()
    m.penalty_plane(3.0e4, 0.01, 0.0, Bf, wf, u, ref)
    assert relerr(pair.host(f), ref) < TOL64


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_pcg_repeats_exactly(pair, prec):
    # a state close enough to the reference one that the shifted tangent is
    # positive definite for every case (at 0.003 the P = 5 and P = 7 cases
    # are not, in the oracle too)
    u = pair.mask * pair.rand(18, 0.001)
    ud = pair.dev(u)
    b = pair.dev(pair.mask * inputs.uniform(19, pair.N, -1, 1))

    def solve():
        x = pair.zeros()
        s = pair.ctx.jacobi_pcg(pair.mat, prec, b, x, u_lin=ud, mass_shift=4.0, rtol=1e-10)
        return s, pair.host(x)

    (s1, x1), (s2, x2) = solve(), solve()
    assert s1["iterations"] == s2["iterations"] and s1["outer"] == s2["outer"]
    assert s1["rel_residual"] == s2["rel_residual"] and same_bits(x1, x2)
    A = pair.pb.A(u, 4.0 * pair.rho)  # the oracle's shift multiplies the unit-density mass
    res = pair.mask * (pair.host(b) - A(x1))
    assert np.linalg.norm(res) <= 2e-10 * np.linalg.norm(pair.host(b))


def test_newton_and_explicit_repeat_exactly():
    bits = inputs.face_bits(4) | inputs.face_bits(5)
    p = Pair((19, 3, 3), (3.0, 1.0, 1.0), 2, kind=ob.SDME_H, dirichlet=bits, ordered=True)
    G = np.zeros((3, 3))
    G[2, 2] = -0.1
    u0 = p.ctx.affine_field([0, 0, 0], G) + p.mask * p.rand(8, 1e-3)
    runs = []
    for prec in (FP32, FP32, FP64):
        ud = p.dev(u0)
        s = p.ctx.newton_static(p.mat, prec, ud, newton_rtol=1e-8, pcg_rtol=1e-8)
        runs.append((s, p.host(ud)))
    (s1, x1), (s2, x2), (s3, x3) = runs
    assert s1["iterations"] == s2["iterations"] and s1["newton"] == s2["newton"]
    assert same_bits(x1, x2)
    assert s1["newton_rel"] <= 1e-8 and s3["newton_rel"] <= 1e-8
    assert relerr(x1, x3) < 1e-7
    # explicit steps with penalty contact, twice from the same start
    q = Pair((9, 3, 2), (1.5, 1.0, 0.5), 2, kind=ob.SDME_M, ordered=True)
    v0 = q.ctx.affine_field([0, 0, -1.0], np.zeros((3, 3)))
    ends = []
    for _ in range(2):
        u1 = q.zeros()
        q.ctx.explicit_step(q.mat, FP64, None, q.zeros(), u1, 2e-4, v0=q.dev(v0),
                            contact=(3.0e4, 0.0), mass_rtol=1e-13)
        prev, cur = q.zeros(), u1
        for _ in range(6):
            nxt = q.zeros()
            q.ctx.explicit_step(q.mat, FP64, prev, cur, nxt, 2e-4, contact=(3.0e4, 0.0),
                                mass_rtol=1e-13)
            prev, cur = cur, nxt
        ends.append(q.host(cur))
    assert same_bits(ends[0], ends[1])
    xf, wf = ob.gauss_legendre(3)
    Bf, _ = q.basis.eval(xf)
    cont = osv.Contact(3.0e4, 0.0, 0.0, Bf, wf)
    up = osv.explicit_start(q.pb, np.zeros(q.N), v0, np.zeros(q.N), 2e-4, 1e-13, cont)
    cur_r = osv.explicit_step(q.pb, up, np.zeros(q.N), np.zeros(q.N), 2e-4, 1e-13, cont)
    prev_r = np.zeros(q.N)
    for _ in range(6):
        prev_r, cur_r = cur_r, osv.explicit_step(q.pb, prev_r, cur_r, np.zeros(q.N), 2e-4, 1e-13,
                                                 cont)
    assert relerr(ends[0], cur_r) < 1e-9


def test_resumed_explicit_run_is_bitwise_the_uninterrupted_one():
    # checkpoint/resume of the central-difference recursion: the state is
    # (u_prev, u_cur); storing it to the host after 3 steps and continuing
    # from the stored copy gives the same bits as 6 uninterrupted steps
    q = Pair((9, 3, 2), (1.5, 1.0, 0.5), 2, kind=ob.SDME_M, ordered=True)
    v0 = q.dev(q.ctx.affine_field([0, 0, -1.0], np.zeros((3, 3))))

    def run(n, prev, cur):
        for _ in range(n):
            nxt = q.zeros()
            q.ctx.explicit_step(q.mat, FP64, prev, cur, nxt, 2e-4, contact=(3.0e4, 0.0),
                                mass_rtol=1e-13)
            prev, cur = cur, nxt
        return prev, cur

    u1 = q.zeros()
    q.ctx.explicit_step(q.mat, FP64, None, q.zeros(), u1, 2e-4, v0=v0, contact=(3.0e4, 0.0),
                        mass_rtol=1e-13)
    _, full = run(6, q.zeros(), u1.clone())
    prev, cur = run(3, q.zeros(), u1.clone())
    saved = (q.host(prev), q.host(cur))
    _, resumed = run(3, q.dev(saved[0]), q.dev(saved[1]))
    assert same_bits(q.host(full), q.host(resumed))


def test_condensed_solve_repeats_exactly():
    # the condensed solve (two operator actions and the interior solves per
    # iteration) on an ordered context: twice the same bits, and the full
    # Jacobi-PCG solution to the solve tolerance
    p = Pair((9, 3, 2), (1.5, 0.75, 0.5), 3, kind=ob.SDME_H, dirichlet=inputs.face_bits(0),
             ordered=True)
    u = p.mask * p.rand(21, 0.001)
    b = p.dev(p.mask * inputs.uniform(22, p.N, -1, 1))
    runs = []
    for _ in range(2):
        x = p.zeros()
        s = p.ctx.condensed_pcg(p.mat, b, x, u_lin=p.dev(u), mass_shift=50.0, rtol=1e-11)
        runs.append((s, p.host(x)))
    assert runs[0][0]["iterations"] == runs[1][0]["iterations"]
    assert same_bits(runs[0][1], runs[1][1])
    xf = p.zeros()
    p.ctx.jacobi_pcg(p.mat, FP64, b, xf, u_lin=p.dev(u), mass_shift=50.0, rtol=1e-11)
    assert relerr(runs[0][1], p.host(xf)) < 1e-8
