"""GPU parity of the condensed solve (static condensation of the element-
interior modes, Section 4) against the oracle's dense condensation of the
same system: the solution to the solve tolerance, the condensed CG's
iteration count within max(1, 2 %) of the oracle's CG with the same
diagonal preconditioner, and equality with the library's full Jacobi-PCG
solution.  Cases: the mass-shifted tangent (implicit step), the tangent
alone (static), the mass alone (explicit step), P = 2, 3, 4, ragged runs."""
import numpy as np
import pytest

from oracle import basis as ob
from oracle import condense as oc
from paper_2104_13466_amd import inputs
from paper_2104_13466_amd.sdme import FP64
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu

CASES = [((3, 2, 1), 2, ob.SDME_H, 400.0, False),
         ((5, 1, 1), 2, ob.SDME_M, 0.0, True),
         ((2, 2, 1), 3, ob.SDME_M, 0.0, False),
         ((2, 1, 1), 4, ob.SDME_H, 250.0, False),
         ((3, 1, 1), 3, ob.NODAL, 50.0, False)]


@pytest.mark.parametrize("n,P,kind,shift,mass_only", CASES,
                         ids=["P%d-%s-%s" % (c[1], ob.KIND_NAMES[c[2]],
                                             "mass" if c[4] else "s%g" % c[3]) for c in CASES])
def test_condensed_pcg_matches_oracle(n, P, kind, shift, mass_only):
    p = Pair(n, (1.0, 0.5, 0.5), P, kind=kind, dirichlet=inputs.face_bits(0), rho=1.3)
    u = p.mask * p.rand(81, 2e-3)
    b = p.mask * inputs.uniform(82, p.N, -1, 1)
    if mass_only:
        op = p.pb.M
    else:
        op = p.pb.A(u, shift * p.rho)
    A = oc.dense_operator(op, p.N)
    B, I = oc.partition(p.pb, A)
    rtol = 1e-12
    x_ref, its_ref = oc.condensed_pcg(A, b, B, I, rtol)
    x = p.zeros()
    st = p.ctx.condensed_pcg(p.mat, p.dev(b), x, u_lin=p.dev(u), mass_shift=shift,
                             mass_only=mass_only, rtol=rtol)
    xh = p.host(x)
    assert st["status"] == 0 and st["rel_residual"] <= rtol
    assert abs(st["iterations"] - its_ref) <= max(1, 0.02 * its_ref), (st["iterations"], its_ref)
    assert np.abs(xh - x_ref).max() <= 1e-8 * np.abs(x_ref).max()
    # the same system by the full Jacobi-PCG
    xf = p.zeros()
    p.ctx.jacobi_pcg(p.mat, FP64, p.dev(b), xf, u_lin=p.dev(u), mass_shift=shift,
                     mass_only=mass_only, rtol=rtol)
    assert np.abs(xh - p.host(xf)).max() <= 1e-8 * np.abs(x_ref).max()
    # the condensed system is smaller: its CG needs no more iterations here
    assert p.ctx.condensed_sizes()[0] == len(B)
