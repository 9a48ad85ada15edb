"""Pins of the oracle's 1D bases (Section 2) against what the paper and the
mathematics fix: closed-form quadrature, closed-form 1D matrices, closed-form
generalised eigenvalues of the internal block, the diagonal/decoupled blocks the
SD and ME steps are defined to produce, and basis independence of the SDME
construction.  All CPU."""
import numpy as np
import pytest
import scipy.special

from oracle import basis as ob


@pytest.mark.parametrize("q", [1, 2, 3, 4, 6, 10, 12])
def test_gauss_legendre_exactness(q):
    x, w = ob.gauss_legendre(q)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * q):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * x ** k).sum() - exact) < 1e-13


def test_gauss_legendre_closed_forms():
    x, w = ob.gauss_legendre(2)
    assert np.allclose(np.sort(x), [-1 / np.sqrt(3), 1 / np.sqrt(3)], atol=1e-15)
    assert np.allclose(w, 1.0, atol=1e-15)
    x, w = ob.gauss_legendre(3)
    o = np.argsort(x)
    assert np.allclose(x[o], [-np.sqrt(0.6), 0.0, np.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w[o], [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("n", range(0, 9))
@pytest.mark.parametrize("ab", [(1.0, 1.0), (0.0, 0.0), (2.0, 0.5)])
def test_jacobi_matches_library(n, ab):
    a, b = ab
    x = np.linspace(-1, 1, 17)
    v, d = ob.jacobi(n, a, b, x)
    assert np.allclose(v, scipy.special.eval_jacobi(n, a, b, x), rtol=1e-13, atol=1e-13)
    if n > 0:
        ref = 0.5 * (n + a + b + 1) * scipy.special.eval_jacobi(n - 1, a + 1, b + 1, x)
        assert np.allclose(d, ref, rtol=1e-13, atol=1e-13)


def test_modal_p2_matrices_closed_form():
    # psi0=(1-x)/2, psi1=(1+x)/2, psi2=(1-x)(1+x)/4: exact integrals
    M, K, vi, ii = ob.mass_stiffness(2, "modal")
    Mref = np.array([[2 / 3, 1 / 3, 1 / 6], [1 / 3, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 1 / 15]])
    Kref = np.array([[0.5, -0.5, 0.0], [-0.5, 0.5, 0.0], [0.0, 0.0, 1 / 6]])
    assert np.abs(M - Mref).max() < 1e-15
    assert np.abs(K - Kref).max() < 1e-15


@pytest.mark.parametrize("P", range(2, 11))
def test_modal_stiffness_vertex_internal_decoupled(P):
    # linear vertex modes have constant derivative; bubble derivatives integrate to 0
    M, K, vi, ii = ob.mass_stiffness(P, "modal")
    assert np.abs(K[np.ix_(vi, ii)]).max() < 1e-14
    # K annihilates constants: psi0 + psi1 = 1
    one = np.zeros(P + 1)
    one[vi] = 1.0
    assert np.abs(K @ one).max() < 1e-14


CLOSED_LAMBDA_S = {
    2: [2.5],
    3: [2.5, 10.5],
    4: [14 - np.sqrt(133), 10.5, 14 + np.sqrt(133)],
    5: [14 - np.sqrt(133), 30 - np.sqrt(405), 14 + np.sqrt(133), 30 + np.sqrt(405)],
}


@pytest.mark.parametrize("P", [2, 3, 4, 5])
@pytest.mark.parametrize("kind", [ob.SDME_M, ob.SDME_K, ob.SDME_H])
@pytest.mark.parametrize("start", ["modal", "nodal"])
def test_lambda_s_closed_forms(P, kind, start):
    # generalised eigenvalues of (K_ii, M_ii) on the bubble space (Eq. diagL)
    b = ob.Basis1D(P, kind, start=start)
    assert np.allclose(b.lambda_s, sorted(CLOSED_LAMBDA_S[P]), rtol=1e-12)


@pytest.mark.parametrize("P", range(2, 11))
@pytest.mark.parametrize("k", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("kind", [ob.SDME_M, ob.SDME_K, ob.SDME_H])
def test_sd_internal_blocks_diagonal(P, k, kind):
    # Eq. ParametroK: M'_ii = Lambda_S^-k, K'_ii = Lambda_S^(1-k)
    b = ob.Basis1D(P, kind, k=k)
    Mii, Kii = b.M1[1:P, 1:P], b.K1[1:P, 1:P]
    ls = b.lambda_s
    assert np.allclose(Mii, np.diag(ls ** -k), atol=1e-12 * ls.max() ** abs(k), rtol=0)
    assert np.allclose(Kii, np.diag(ls ** (1 - k)), atol=1e-11 * ls.max(), rtol=0)
    if k == 1.0:  # condition number 1 for the internal stiffness block
        assert np.allclose(np.diag(Kii), 1.0, atol=1e-12)
    if k == 0.0:
        assert np.allclose(np.diag(Mii), 1.0, atol=1e-12)


@pytest.mark.parametrize("P", range(2, 11))
@pytest.mark.parametrize("kind", [ob.SDME_M, ob.SDME_K, ob.SDME_H])
def test_me_coupling_zero(P, kind):
    # ME step zeroes the vertex-internal coupling block of the chosen norm
    lam = 100.0
    b = ob.Basis1D(P, kind, lam=lam)
    A = {ob.SDME_M: b.M1, ob.SDME_K: b.K1, ob.SDME_H: b.K1 + lam * b.M1}[kind]
    scale = np.abs(A).max()
    vert = [0, P]
    assert np.abs(A[np.ix_(vert, list(range(1, P)))]).max() < 1e-13 * scale


def test_sdme_m_p2_vertex_mode_closed_form():
    # alpha^M = M_vi M_ii^-1 = [2.5, 2.5] for the modal start, so
    # phi_0 = (1-x)/2 - 2.5 (1-x)(1+x)/4 (Eq. alphaMassa)
    b = ob.Basis1D(2, ob.SDME_M)
    x = np.linspace(-1, 1, 11)
    V, Dv = b.eval(x)
    assert np.allclose(V[:, 0], 0.5 * (1 - x) - 0.625 * (1 - x * x), atol=1e-14)
    assert np.allclose(V[:, 2], 0.5 * (1 + x) - 0.625 * (1 - x * x), atol=1e-14)
    assert np.allclose(Dv[:, 0], -0.5 + 1.25 * x, atol=1e-14)


@pytest.mark.parametrize("P", [2, 3, 5, 8])
def test_sdme_k_vertex_modes_linear(P):
    # modal start already has K_vi = 0, so the energy-norm extension is linear
    b = ob.Basis1D(P, ob.SDME_K)
    x = np.linspace(-1, 1, 9)
    V, _ = b.eval(x)
    assert np.allclose(V[:, 0], 0.5 * (1 - x), atol=1e-13)
    assert np.allclose(V[:, P], 0.5 * (1 + x), atol=1e-13)


@pytest.mark.parametrize("P", range(1, 11))
@pytest.mark.parametrize("kind", [ob.NODAL, ob.MODAL, ob.SDME_M, ob.SDME_K, ob.SDME_H])
def test_vertex_and_bubble_values(P, kind):
    b = ob.Basis1D(P, kind)
    V, _ = b.eval(np.array([-1.0, 1.0]))
    ref = np.zeros((2, P + 1))
    ref[0, 0] = 1.0
    ref[1, P] = 1.0
    assert np.abs(V - ref).max() < 1e-12


@pytest.mark.parametrize("P", [2, 4, 6, 8, 10])
@pytest.mark.parametrize("kind", [ob.SDME_M, ob.SDME_K, ob.SDME_H])
def test_sdme_basis_independent_of_start(P, kind):
    # SD and ME depend only on the spaces; with the fixed order/sign reading the
    # tables from the modal and from the nodal start coincide
    b1 = ob.Basis1D(P, kind, start="modal")
    b2 = ob.Basis1D(P, kind, start="nodal")
    _, _, B1, D1 = b1.tables(P + 2)
    _, _, B2, D2 = b2.tables(P + 2)
    assert np.abs(B1 - B2).max() < 1e-11
    assert np.abs(D1 - D2).max() < 1e-10


@pytest.mark.parametrize("P", [1, 2, 5, 8])
def test_nodal_collocation(P):
    b = ob.Basis1D(P, ob.NODAL)
    V, _ = b.eval(ob.gll_points(P))
    assert np.abs(V - np.eye(P + 1)).max() < 1e-13


@pytest.mark.parametrize("P", [2, 4, 8])
@pytest.mark.parametrize("kind", [ob.NODAL, ob.MODAL, ob.SDME_H])
def test_derivative_table_matches_difference_quotient(P, kind):
    b = ob.Basis1D(P, kind)
    x, _ = ob.gauss_legendre(P + 2)
    _, Dv = b.eval(x)
    eps = 1e-6
    Vp, _ = b.eval(x + eps)
    Vm, _ = b.eval(x - eps)
    assert np.abs((Vp - Vm) / (2 * eps) - Dv).max() < 1e-6 * max(1.0, np.abs(Dv).max())


@pytest.mark.parametrize("P", [1, 2, 4, 8])
@pytest.mark.parametrize("kind", [ob.NODAL, ob.MODAL, ob.SDME_M, ob.SDME_H])
def test_affine_coefficients(P, kind):
    b = ob.Basis1D(P, kind)
    g1, gx = b.affine_coeffs()
    x = np.linspace(-1, 1, 13)
    V, _ = b.eval(x)
    assert np.abs(V @ g1 - 1.0).max() < 1e-12
    assert np.abs(V @ gx - x).max() < 1e-12
    # vertex coefficients are the vertex values
    assert abs(g1[0] - 1) < 1e-12 and abs(g1[P] - 1) < 1e-12
    assert abs(gx[0] + 1) < 1e-12 and abs(gx[P] - 1) < 1e-12


def test_gll_rule_closed_forms_and_exactness():
    # Q = 2: the trapezoidal rule; Q = 3: Simpson's rule; exact to degree 2Q - 3
    x, w = ob.gll_rule(2)
    assert np.allclose(x, [-1, 1], atol=1e-15) and np.allclose(w, [1, 1], atol=1e-15)
    x, w = ob.gll_rule(3)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    for Q in range(2, 11):
        x, w = ob.gll_rule(Q)
        for d in range(2 * Q - 2):
            exact = 0.0 if d % 2 else 2.0 / (d + 1)
            assert abs(w @ x ** d - exact) < 1e-13
        # degree 2Q - 2 is not integrated exactly
        d = 2 * Q - 2
        assert abs(w @ x ** d - 2.0 / (d + 1)) > 1e-6


@pytest.mark.parametrize("P", [1, 2, 4, 7])
def test_nodal_basis_with_gll_rule_has_diagonal_mass(P):
    # Lagrange basis on the GLL points, integrated with the same points: the
    # 1D mass B^T W B is diagonal (collocation), and so is the element mass
    # M1 x M1 x M1
    b, x, w, B, D = ob.build(P, P + 1, ob.NODAL)
    M = B.T @ np.diag(w) @ B
    assert np.abs(M - np.diag(np.diag(M))).max() < 1e-14 * np.abs(M).max()
    # and the mass weights are the GLL weights (vertex slots first/last)
    assert np.allclose(np.sort(np.diag(M)), np.sort(w), atol=1e-14)


def test_condition_numbers_follow_the_paper_figure():
    # Fig. ConditionNumbers1D and its discussion (Section 2): the SDME-M mass
    # (k = 1/2) is better conditioned than the ST mass and grows slowly with
    # P; with k = 1 the SDME-M internal stiffness block has condition number 1;
    # the SDME-H (lambda = 1, k = 1) equivalent stiffness K + M is almost
    # constant in P while the ST one grows
    c_st, c_m, c_h, c_hst = [], [], [], []
    for P in range(2, 11):
        st = ob.Basis1D(P, ob.MODAL)
        sm = ob.Basis1D(P, ob.SDME_M, k=0.5)
        sm1 = ob.Basis1D(P, ob.SDME_M, k=1.0)
        sh = ob.Basis1D(P, ob.SDME_H, k=1.0, lam=1.0)
        c_st.append(np.linalg.cond(st.M1))
        c_m.append(np.linalg.cond(sm.M1))
        assert abs(np.linalg.cond(sm1.K1[1:P, 1:P]) - 1.0) < 1e-10
        c_h.append(np.linalg.cond(sh.K1 + sh.M1))
        c_hst.append(np.linalg.cond(st.K1 + st.M1))
    assert all(a < b / 10 for a, b in zip(c_m, c_st))
    assert c_m[-1] / c_m[0] < c_st[-1] / c_st[0]
    assert max(c_h) / min(c_h) < 1.05
    assert c_hst[-1] / c_hst[0] > 1.5
