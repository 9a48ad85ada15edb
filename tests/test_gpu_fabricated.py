"""GPU parity of the loads given at quadrature points and of the L2 error
(Section 5 fabricated-solution problems) against the oracle, and the static
large-strain example of Section 5.1 solved on the GPU: its L2 errors against
the values the paper prints (Table Tab:Static_error), its Newton iteration
count, its independence of the basis, and its agreement with the oracle's
solution.  Load and error parity: 1e-12 relative in the max norm, on meshes
whose rows span several element blocks, every order P = 1..8."""
import numpy as np
import pytest

from oracle import basis as ob
from oracle import fabricated as fb
from paper_2104_13466_amd import fabricated as pf
from paper_2104_13466_amd import inputs
from paper_2104_13466_amd.sdme import FP32, FP64, Context
from tests.gpu_setup import Pair, relerr
from tests.test_oracle_fabricated import paper_l2, within_factor

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

CASES = [
    ((5, 2, 3), 1, ob.MODAL),
    ((4, 3, 2), 2, ob.SDME_H),
    ((3, 2, 2), 3, ob.SDME_M),
    ((3, 2, 1), 4, ob.SDME_H),
    ((2, 2, 1), 5, ob.NODAL),
    ((2, 1, 2), 6, ob.SDME_K),
    ((2, 1, 1), 7, ob.MODAL),
    ((1, 2, 1), 8, ob.SDME_H),
]
IDS = ["P%d-%s" % (c[1], ob.KIND_NAMES[c[2]]) for c in CASES]


@pytest.fixture(scope="module", params=CASES, ids=IDS)
def pair(request):
    n, P, kind = request.param
    return Pair(n, (1.0, 0.75, 1.25), P, kind=kind)


def test_quadrature_points(pair):
    m = pair.pb.mesh
    assert np.abs(pair.ctx.quadrature_points() - fb.volume_points(m)).max() <= 1e-15
    for face in range(6):
        assert np.abs(pair.ctx.quadrature_points(face) - fb.face_points(m, face)).max() <= 1e-15


def test_body_load(pair):
    m = pair.pb.mesh
    shape = (3, m.E, m.Q ** 3)
    b = inputs.uniform(11, int(np.prod(shape)), -1, 1).reshape(shape)
    f = pair.zeros()
    pair.ctx.body_load(pair.dev(b), f)
    assert relerr(pair.host(f), fb.body_load(m, b)) < TOL64


@pytest.mark.parametrize("face", range(6))
def test_face_load(pair, face):
    m = pair.pb.mesh
    xf, _ = ob.gauss_legendre(m.P + 1)
    Bf, _ = pair.basis.eval(xf)
    shape = (3, pair.ctx.face_elements(face), (m.P + 1) ** 2)
    t = inputs.uniform(20 + face, int(np.prod(shape)), -1, 1).reshape(shape)
    f = pair.zeros()
    f0 = inputs.uniform(30, pair.N, -1, 1)
    f.copy_(pair.dev(f0))  # accumulates into the existing vector
    pair.ctx.face_load(face, pair.dev(t), f)
    assert relerr(pair.host(f), f0 + fb.face_load(m, face, Bf, t)) < TOL64


def test_l2_error(pair):
    m = pair.pb.mesh
    u = pair.rand(12, 1.0)
    shape = (3, m.E, m.Q ** 3)
    g = inputs.uniform(13, int(np.prod(shape)), -1, 1).reshape(shape)
    err = pair.ctx.l2_error(pair.dev(u), pair.dev(g))
    assert relerr(err, fb.l2_error(m, u, g)) < TOL64


# ------------------------------------------------ static example, Section 5.1
def static_solve(P, kind, prec, pcg_rtol=1e-8, newton_rtol=1e-8):
    import torch
    ctx = Context((2, 2, 2), (1.0, 1.0, 1.0), P, basis=kind, dirichlet=pf.DIRICHLET_X0)
    lam, mu = pf.lame()
    mu_t = torch.full((ctx.E,), mu, dtype=torch.float64, device="cuda")
    lam_t = torch.full((ctx.E,), lam, dtype=torch.float64, device="cuda")
    mat = Context.material(mu_t, lam_t, 1.0)
    f = torch.zeros(3 * ctx.Nn, dtype=torch.float64, device="cuda")
    pf.static_loads(ctx, f)
    u = torch.zeros_like(f)
    st = ctx.newton_static(mat, prec, u, f_ext=f, newton_rtol=newton_rtol, pcg_rtol=pcg_rtol,
                           max_newton=20, max_pcg=20000)
    err = ctx.l2_error(u, pf.static_exact_at_gauss_points(ctx))
    return u.cpu().numpy(), st, err, f.cpu().numpy()


def test_static_loads_match_oracle():
    mesh, Bf = fb.static_mesh(3, ob.SDME_H)
    _, _, _, f = static_solve(3, ob.SDME_H, FP64)
    assert relerr(f, fb.static_loads(mesh, Bf)) < 1e-9  # oracle: numeric differentiation


@pytest.mark.parametrize("P", [2, 4, 6, 8])
@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "mixed"])
def test_static_example_matches_paper(P, prec):
    ref = paper_l2()[P]
    u, st, err, _ = static_solve(P, ob.SDME_H, prec)
    print("P=%d %s L2 errors %s paper %s newton %d pcg %d" % (
        P, "fp64" if prec == FP64 else "mixed", err, ref[1:], st["newton"], st["iterations"]))
    assert st["newton"] == 5
    if P <= 4:
        assert within_factor(err, ref[1:], 1.5), (err, ref)
    else:
        # the printed errors decay more slowly from P = 4 on than the
        # discretisation error does (a floor of the paper's solver tolerances
        # or quadrature): the solution here is at least as accurate
        assert np.all(err <= 1.5 * np.asarray(ref[1:])), (err, ref)


def test_static_example_matches_oracle_p2():
    u, st, err, _ = static_solve(2, ob.SDME_H, FP64)
    uo, hist, erro = fb.static_solve(2, ob.SDME_H, pcg_rtol=1e-8, max_pcg=2000)
    assert relerr(err, erro) < 1e-6
    assert relerr(u, uo) < 1e-8


def test_static_example_basis_independent_p4():
    errs = [static_solve(4, kind, FP64)[2] for kind in (ob.SDME_H, ob.SDME_M, ob.MODAL, ob.NODAL)]
    for e in errs[1:]:
        assert relerr(e, errs[0]) < 1e-5


def _pcg_per_newton(P, kind):
    _, st, _, _ = static_solve(P, kind, FP64)
    return st["iterations"] / st["newton"]


def test_static_example_iteration_trend_matches_paper():
    # Table Tab:NH_average_IT_CGD: the standard modal basis needs 3.7x (P=4) and
    # 7.9x (P=8) the CGD iterations of SDME-M, and SDME-H needs fewer than
    # SDME-M at P = 4
    r = {P: {k: _pcg_per_newton(P, k) for k in (ob.MODAL, ob.SDME_M, ob.SDME_H)} for P in (4, 8)}
    for P in (4, 8):
        assert r[P][ob.MODAL] >= 3.0 * r[P][ob.SDME_M]
    assert r[8][ob.MODAL] / r[8][ob.SDME_M] > r[4][ob.MODAL] / r[4][ob.SDME_M]
    assert r[4][ob.SDME_H] < r[4][ob.SDME_M]


# ----------------------------------------- transient example, Section 5.2
from tests.test_oracle_fabricated import (WAVE_DT_EXPLICIT, WAVE_DT_NEWMARK,  # noqa: E402
                                          WAVE_STEPS_EXPLICIT, WAVE_STEPS_NEWMARK, paper_wave_l2)


def wave_ctx(P, kind):
    import torch
    ctx = Context((2, 2, 2), (1.0, 1.0, 1.0), P, basis=kind, dirichlet=pf.DIRICHLET_X0)
    lam, mu = pf.lame()
    mat = Context.material(torch.full((ctx.E,), mu, dtype=torch.float64, device="cuda"),
                           torch.full((ctx.E,), lam, dtype=torch.float64, device="cuda"), pf.RHO)
    return ctx, mat


def check_paper(P, err, ref):
    # u_x within 1.5x; the lateral components within 2x (the paper's u_y and
    # u_z differ by up to 10 % from each other although the problem is
    # symmetric in y and z, so its lateral errors carry some asymmetry of its
    # set-up); from P = 6 on, the printed errors are a floor the solution
    # here stays below
    if P <= 4:
        assert within_factor(err[0], ref[0], 1.5), (err, ref)
        assert within_factor(err[1:], ref[1:], 2.0), (err, ref)
    else:
        assert np.all(err <= 1.5 * np.asarray(ref)), (err, ref)


# the modal basis needs ~1300 mass-PCG iterations per explicit step at P = 4:
# it is run at P = 2 only
@pytest.mark.parametrize("P,kind", [(2, ob.MODAL), (2, ob.SDME_M), (4, ob.SDME_M), (6, ob.SDME_M)],
                         ids=["P2-modal", "P2-sdme_m", "P4-sdme_m", "P6-sdme_m"])
def test_wave_explicit_matches_paper(P, kind):
    ctx, mat = wave_ctx(P, kind)
    u, mass_its = pf.wave_explicit(ctx, mat, WAVE_DT_EXPLICIT, WAVE_STEPS_EXPLICIT, FP64)
    err = ctx.l2_error(u, pf.exact_at_gauss_points(ctx, "wave", 0.25))
    ref = paper_wave_l2()[("explicit", ob.KIND_NAMES[kind].replace("-", "_"), P)]
    print("explicit P=%d %s L2 %s paper %s mass its/step %.1f" % (
        P, ob.KIND_NAMES[kind], err, ref, mass_its / WAVE_STEPS_EXPLICIT))
    check_paper(P, err, ref)


@pytest.mark.parametrize("P", [2, 4, 6])
@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "mixed"])
def test_wave_newmark_matches_paper(P, prec):
    ctx, mat = wave_ctx(P, ob.SDME_H)
    u, newton, pcg = pf.wave_newmark(ctx, mat, WAVE_DT_NEWMARK, WAVE_STEPS_NEWMARK, prec)
    err = ctx.l2_error(u, pf.exact_at_gauss_points(ctx, "wave", 0.25))
    ref = paper_wave_l2()[("newmark", "sdme_h", P)]
    print("newmark P=%d L2 %s paper %s newton %d pcg/solve %.1f" % (P, err, ref, newton,
                                                                   pcg / newton))
    check_paper(P, err, ref)


def test_wave_explicit_matches_oracle_p2():
    ctx, mat = wave_ctx(2, ob.SDME_M)
    u, _ = pf.wave_explicit(ctx, mat, WAVE_DT_EXPLICIT, WAVE_STEPS_EXPLICIT, FP64)
    uo, erro = fb.wave_explicit(2, ob.SDME_M, WAVE_DT_EXPLICIT, WAVE_STEPS_EXPLICIT)
    assert relerr(u.cpu().numpy(), uo) < 1e-7


def test_wave_newmark_matches_oracle_p2():
    ctx, mat = wave_ctx(2, ob.SDME_H)
    u, newton, _ = pf.wave_newmark(ctx, mat, WAVE_DT_NEWMARK, WAVE_STEPS_NEWMARK, FP64)
    uo, erro, newton_o, _ = fb.wave_newmark(2, ob.SDME_H, WAVE_DT_NEWMARK, WAVE_STEPS_NEWMARK)
    assert relerr(u.cpu().numpy(), uo) < 1e-7
    assert abs(newton - newton_o) <= max(1, 0.02 * newton_o)


def test_wave_newmark_iteration_trend_matches_paper():
    # Table Tab:TransientNmk_NH_NIT_Hexa: ST needs 18x the CGD iterations of
    # SDME-M and SDME-H at P = 4
    its = {}
    for kind in (ob.MODAL, ob.SDME_M, ob.SDME_H):
        ctx, mat = wave_ctx(4, kind)
        _, newton, pcg = pf.wave_newmark(ctx, mat, WAVE_DT_NEWMARK, 25, FP64)
        its[kind] = pcg / newton
    assert its[ob.MODAL] >= 5.0 * its[ob.SDME_M]
    assert its[ob.MODAL] >= 5.0 * its[ob.SDME_H]


# ------------------------------- Lagrange basis with a diagonal (lumped) mass
def lumped_ctx(P):
    import torch
    ctx = Context((2, 2, 2), (1.0, 1.0, 1.0), P, basis=ob.NODAL, dirichlet=pf.DIRICHLET_X0,
                  lumped_mass=True)
    lam, mu = pf.lame()
    mat = Context.material(torch.full((ctx.E,), mu, dtype=torch.float64, device="cuda"),
                           torch.full((ctx.E,), lam, dtype=torch.float64, device="cuda"), pf.RHO)
    return ctx, mat


@pytest.mark.parametrize("P", [2, 5])
def test_lumped_mass_matches_oracle_and_is_diagonal(P):
    ctx, mat = lumped_ctx(P)
    mm, _ = fb.static_mesh(P, ob.NODAL, Q=P + 1)
    v = inputs.uniform(4, 3 * ctx.Nn, -1, 1)
    import torch
    y = torch.zeros(3 * ctx.Nn, dtype=torch.float64, device="cuda")
    ctx.mass_apply(1.5, FP64, torch.as_tensor(v, device="cuda"), y)
    ref = mm.mass_apply(1.5, v)
    assert relerr(y.cpu().numpy(), ref) < TOL64
    dg = mm.tangent_diag(np.zeros(mm.E), np.zeros(mm.E), np.zeros_like(v), 1.5)
    assert relerr(ref, dg * v) < TOL64


@pytest.mark.parametrize("P", [2, 4, 6])
def test_wave_explicit_lagrange_diagonal_mass_matches_paper(P):
    ctx, mat = lumped_ctx(P)
    u, mass_its = pf.wave_explicit(ctx, mat, WAVE_DT_EXPLICIT, WAVE_STEPS_EXPLICIT, FP64)
    eg, _ = wave_ctx(P, ob.NODAL)  # error by the Gauss rule of P+2 points
    err = eg.l2_error(u, pf.exact_at_gauss_points(eg, "wave", 0.25))
    ref = paper_wave_l2()[("explicit", "lagrange_diag", P)]
    print("explicit lumped P=%d L2 %s paper %s mass its/step %.2f" % (
        P, err, ref, mass_its / WAVE_STEPS_EXPLICIT))
    check_paper(P, err, ref)
    assert mass_its <= WAVE_STEPS_EXPLICIT  # a diagonal mass: one PCG iteration per solve


def test_wave_explicit_lagrange_diagonal_mass_matches_oracle_p2():
    ctx, mat = lumped_ctx(2)
    u, _ = pf.wave_explicit(ctx, mat, WAVE_DT_EXPLICIT, WAVE_STEPS_EXPLICIT, FP64)
    uo, _ = fb.wave_explicit(2, ob.NODAL, WAVE_DT_EXPLICIT, WAVE_STEPS_EXPLICIT, lumped=True)
    assert relerr(u.cpu().numpy(), uo) < 1e-7


# ------------------- quartic field x^4 sin(2 pi t), Newmark (Section 5.2)
QUARTIC_T = 0.025


def test_quartic_newmark_time_convergence_is_quadratic():
    # the paper: time convergence at P = 5 is quadratic for the Newmark
    # method; x^4 lies in the P = 5 space, so the error is the time error
    errs = []
    for nsteps in (8, 16, 32):
        ctx, mat = wave_ctx(5, ob.SDME_H)
        u, _, _ = pf.wave_newmark(ctx, mat, QUARTIC_T / nsteps, nsteps, FP64, newton_rtol=1e-10,
                                  pcg_rtol=1e-10, name="quartic")
        errs.append(ctx.l2_error(u, pf.exact_at_gauss_points(ctx, "quartic", QUARTIC_T))[0])
    print("quartic P=5 errors", errs)
    for a, b in zip(errs, errs[1:]):
        assert 3.8 < a / b < 4.2


def test_quartic_newmark_spatial_convergence_to_the_time_floor():
    # dt = 3.9e-4 (the paper's), P = 2, 3, 4: the error falls by more than
    # 1e4 from P = 2 to P = 4, where the spatial error is below the time error
    errs = []
    for P in (2, 3, 4, 5):
        ctx, mat = wave_ctx(P, ob.SDME_H)
        u, _, _ = pf.wave_newmark(ctx, mat, QUARTIC_T / 64, 64, FP64, name="quartic")
        errs.append(ctx.l2_error(u, pf.exact_at_gauss_points(ctx, "quartic", QUARTIC_T))[0])
    print("quartic dt=3.9e-4 errors P=2..5", errs)
    assert errs[0] / errs[1] > 5 and errs[1] / errs[2] > 100
    assert abs(errs[3] - errs[2]) < 0.05 * errs[2]  # the time floor


def test_quartic_newmark_matches_oracle_p2():
    ctx, mat = wave_ctx(2, ob.SDME_H)
    u, newton, _ = pf.wave_newmark(ctx, mat, QUARTIC_T / 16, 16, FP64, name="quartic")
    uo, _, newton_o, _ = fb.wave_newmark(2, ob.SDME_H, QUARTIC_T / 16, 16, field=fb.quartic_field)
    assert relerr(u.cpu().numpy(), uo) < 1e-7
    assert abs(newton - newton_o) <= max(1, 0.02 * newton_o)
