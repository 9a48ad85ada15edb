"""Pins of the oracle's static condensation (Section 4, Schur complement of
the element-interior modes) on the CPU: the condensed solve equals the full
solve of the same system; the condensed operator is the energy minimum over
the interior modes (x_B^T S x_B = min over x_I of x^T A x); the interior
modes of the printed meshes give the condensed DOF counts of Section 5.2
(276, 1296 for the printed 1246, 3084), also from the library's host query."""
import os

import numpy as np
import pytest

from oracle import basis as ob
from oracle import condense as oc
from paper_2104_13466_amd import inputs
from tests.oracle_setup import make


def _system(n, P, kind, cm, seed):
    pb, _ = make(n, (1.0, 0.5, 0.5), P, kind=kind, dirichlet=inputs.face_bits(0))
    u = pb.mask * inputs.random_coeffs(seed, n, P, 2e-3)
    A = oc.dense_operator(pb.A(u, cm * pb.rho), 3 * pb.mesh.Nn)
    b = pb.mask * inputs.uniform(seed + 1, 3 * pb.mesh.Nn, -1, 1)
    return pb, A, b


@pytest.mark.parametrize("n,P,kind,cm", [((2, 1, 1), 2, ob.SDME_H, 0.0),
                                         ((2, 2, 1), 2, ob.SDME_M, 400.0),
                                         ((1, 1, 1), 3, ob.MODAL, 50.0)])
def test_condensed_solve_equals_full_solve(n, P, kind, cm):
    pb, A, b = _system(n, P, kind, cm, 61)
    B, I = oc.partition(pb, A)
    assert len(I) == 3 * pb.mesh.E * (P - 1) ** 3
    free = np.flatnonzero(pb.mask > 0)
    x_full = np.zeros_like(b)
    x_full[free] = np.linalg.solve(A[np.ix_(free, free)], b[free])
    x_c = oc.condensed_solve(A, b, B, I)
    assert np.abs(x_c - x_full).max() < 1e-11 * np.abs(x_full).max()
    # the condensed CG reaches the same solution
    x_cg, its = oc.condensed_pcg(A, b, B, I, 1e-13)
    assert its > 0 and np.abs(x_cg - x_full).max() < 1e-9 * np.abs(x_full).max()


def test_condensed_operator_is_interior_energy_minimum():
    # for SPD A: min over x_I of [x_B; x_I]^T A [x_B; x_I] = x_B^T S x_B,
    # attained at x_I = -A_II^-1 A_IB x_B
    pb, A, b = _system((2, 1, 1), 3, ob.SDME_K, 10.0, 71)
    B, I = oc.partition(pb, A)
    S, _ = oc.condensed_system(A, b, B, I)
    xB = inputs.uniform(72, len(B), -1, 1)
    xI = -np.linalg.solve(A[np.ix_(I, I)], A[np.ix_(I, B)] @ xB)

    def energy(xi):
        x = np.zeros_like(b)
        x[B], x[I] = xB, xi
        return x @ A @ x
    e0 = energy(xI)
    assert abs(e0 - xB @ S @ xB) < 1e-11 * abs(e0)
    for s in (73, 74):
        assert energy(xI + 1e-3 * inputs.uniform(s, len(I), -1, 1)) > e0
    assert np.allclose(S, S.T, atol=1e-12 * np.abs(S).max())


def test_condensed_sizes_match_printed_counts():
    from paper_2104_13466_amd import sdme
    golden = os.path.join(os.path.dirname(__file__), "golden", "dof_counts.txt")
    rows = [line.split() for line in open(golden)
            if line.strip() and not line.startswith("#")]
    for kind, P, dofs in rows:
        if kind != "condensed":
            continue
        c = sdme.Context((2, 2, 2), (1.0, 1.0, 1.0), int(P), dirichlet=inputs.face_bits(0))
        free_b, inner, nI = c.condensed_sizes()
        assert free_b == int(dofs) and inner == 8 * 3 * (int(P) - 1) ** 3
        assert nI == 3 * (int(P) - 1) ** 3
        c.close()
