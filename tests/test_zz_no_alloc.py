"""The allocation-free PCG entry point (sdme_jacobi_pcg_noalloc, workspace in
the library's device-resident scratch array) against sdme_jacobi_pcg with a
caller workspace, through the C ABI: two calls in a row, the second on a
smaller mesh, in FP64 and mixed precision; requests beyond the array's size
are refused.  Iterative results are compared as the parity tests compare
solves: iteration counts within max(1, 2 %), both at the tolerance, and the
solutions within a bound set by the tolerance."""
import numpy as np
import pytest

from oracle import basis as ob
from paper_2104_13466_amd import inputs
from paper_2104_13466_amd.sdme import FP32, FP64, SdmeError
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _solve_both(p, prec, seed, shift):
    ud = p.dev(p.mask * p.rand(seed, 1e-3))
    b = p.dev(inputs.uniform(seed + 1, p.N, -1, 1))
    x_ref, x_na = p.zeros(), p.zeros()
    s_ref = p.ctx.jacobi_pcg(p.mat, prec, b, x_ref, u_lin=ud, mass_shift=shift, rtol=RTOL)
    rc, s_na = p.ctx.jacobi_pcg_noalloc(p.mat, prec, b, x_na, u_lin=ud, mass_shift=shift,
                                        rtol=RTOL)
    assert rc == 0 and s_na["status"] == 0
    it_r, it_n = s_ref["iterations"], s_na["iterations"]
    # FP64: the parity bar for iteration counts.  Mixed: the order of the FP32
    # atomic additions in the operator changes the rounding of the FP32
    # recursion from run to run, and with it the count by a few percent
    # (also between two calls of the same entry point)
    tol = max(1, 0.02 * it_r) if prec == FP64 else max(2, 0.05 * it_r)
    assert abs(it_r - it_n) <= tol, (it_r, it_n)
    assert s_ref["rel_residual"] <= RTOL and s_na["rel_residual"] <= RTOL
    xr, xn = p.host(x_ref), p.host(x_na)
    assert np.abs(xn - xr).max() <= 1e-6 * np.abs(xr).max()
    return it_n


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_noalloc_pcg_matches_workspace_pcg_two_calls(prec):
    big = Pair((6, 3, 3), (1.0, 0.5, 0.5), 3, kind=ob.SDME_H, dirichlet=inputs.face_bits(0))
    small = Pair((3, 2, 2), (0.5, 0.5, 0.5), 2, kind=ob.SDME_M, dirichlet=inputs.face_bits(4))
    assert small.N < big.N
    assert _solve_both(big, prec, 31, 0.0) > 10
    # second call: smaller input, the scratch array still holds the first
    # call's contents
    assert _solve_both(small, prec, 41, 50.0) > 5


def test_noalloc_pcg_refuses_oversized_workspace():
    # a mesh whose solve needs more than the scratch array is refused before
    # any launch (SDME_ENOMEM); x is untouched
    p = Pair((24, 8, 8), (1.0, 0.5, 0.5), 4, kind=ob.SDME_H, dirichlet=inputs.face_bits(0))
    assert p.ctx.workspace_bytes(0, FP64) > 32 * 2 ** 20
    x = p.zeros()
    with pytest.raises(SdmeError) as e:
        p.ctx.jacobi_pcg_noalloc(p.mat, FP64, p.dev(inputs.uniform(5, p.N, -1, 1)), x,
                                 u_lin=p.zeros())
    assert e.value.code == -2
    assert np.abs(p.host(x)).max() == 0.0
