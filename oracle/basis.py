"""ORACLE -- test infrastructure only.

Plain FP64 construction of the one-dimensional bases of Section 2 (construction
of high-order bases).  Only ``tests/``, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product library never does.

What is built, in the paper's order:

* Gauss-Legendre rule (library routine ``numpy.polynomial.legendre.leggauss``).
* Starting bases: Lagrange nodal on Gauss-Lobatto-Legendre points (Eq.
  lagrangian / shape_functions_lag) and the Jacobi modal "ST" basis with
  alpha = beta = 1 (Eq. BasePadrao1D).
* 1D mass and stiffness matrices (Eqs. Matrizesmassa, Matrizesrigidez) with the
  vertex / internal partition (Eq. BlocosMassa).
* Simultaneous diagonalisation of the internal block (Eqs. Diagonalizacao1 ..
  ParametroK): eig(M_ii) -> X, Lambda_M;  L = (X Lambda_M^-1/2)^T K_ii (..);
  eig(L) -> Z, Lambda_S;  Y = (X Lambda_M^-1/2 Z Lambda_S^-k/2)^T.
* Minimum-energy vertex modes (Eqs. ExtensaoMEmassa, alphaMassa,
  alphaRigidez, alphaKN): phi_k = psi_k - sum_j alpha_kj phi_j with
  alpha = A_vi A_ii^-1 for A = M (SDME-M), K (SDME-K), K + lambda M (SDME-H).

Readings where the paper is silent (each is listed in the design notes):
* internal modes are ordered by ascending Lambda_S and each is signed so that
  its derivative at xi = -1 is positive;
* slot order for the tensor product: slot 0 = left vertex mode, slots
  1..P-1 = internal modes, slot P = right vertex mode;
* the SD/ME step is applied to the internal modes produced by SD (the paper
  writes the ME sum over psi_j^i; the span is the same, so the vertex modes are
  the same function).

A basis is held as a coefficient matrix T (slot x starting-basis index) over
its starting basis: phi_s(x) = sum_m T[s, m] psi_m(x).
"""
import numpy as np
from numpy.polynomial import legendre as _npleg

NODAL, MODAL, SDME_M, SDME_K, SDME_H = 0, 1, 2, 3, 4
KIND_NAMES = {NODAL: "nodal", MODAL: "modal", SDME_M: "sdme-m",
              SDME_K: "sdme-k", SDME_H: "sdme-h"}


def gauss_legendre(q):
    """Gauss-Legendre points and weights on [-1, 1] (library routine)."""
    x, w = _npleg.leggauss(q)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def gll_points(P):
    """Gauss-Lobatto-Legendre points: -1, the roots of L_P', +1 (Section 2,
    nodal basis on GLL collocation points)."""
    if P == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(P + 1)
    c[P] = 1.0
    r = np.sort(np.real(_npleg.legroots(_npleg.legder(c))))
    return np.concatenate([[-1.0], r, [1.0]])


def gll_rule(q):
    """Gauss-Lobatto-Legendre rule of q points on [-1, 1]: the points of
    gll_points(q - 1), weights 2 / (q (q - 1) L_{q-1}(x)^2); exact for
    polynomials of degree 2q - 3."""
    x = gll_points(q - 1)
    c = np.zeros(q)
    c[q - 1] = 1.0
    L = _npleg.legval(x, c)
    return x, 2.0 / (q * (q - 1) * L * L)


def volume_rule(P, Q):
    """The volume rule of the meshes: Gauss-Legendre for Q = P + 2 (Q points),
    Gauss-Lobatto-Legendre for Q = P + 1 (collocated with the nodal basis)."""
    return gll_rule(Q) if Q == P + 1 else gauss_legendre(Q)


def jacobi(n, a, b, x):
    """Jacobi polynomial P_n^{a,b}(x) and its derivative, by the three-term
    recurrence and d/dx P_n^{a,b} = (n+a+b+1)/2 P_{n-1}^{a+1,b+1}."""
    x = np.asarray(x, dtype=np.float64)

    def val(n, a, b):
        p0 = np.ones_like(x)
        if n == 0:
            return p0
        p1 = 0.5 * ((a - b) + (a + b + 2.0) * x)
        for m in range(1, n):
            c = 2.0 * m + a + b
            a1 = 2.0 * (m + 1) * (m + a + b + 1) * c
            a2 = (c + 1.0) * (a * a - b * b)
            a3 = c * (c + 1.0) * (c + 2.0)
            a4 = 2.0 * (m + a) * (m + b) * (c + 2.0)
            p0, p1 = p1, ((a2 + a3 * x) * p1 - a4 * p0) / a1
        return p1

    v = val(n, a, b)
    d = np.zeros_like(x) if n == 0 else 0.5 * (n + a + b + 1.0) * val(n - 1, a + 1.0, b + 1.0)
    return v, d


def modal_start(P, x, alpha=1.0, beta=1.0):
    """Standard modal basis (Eq. BasePadrao1D): psi_0 = (1-x)/2,
    psi_1 = (1+x)/2, psi_p = (1-x)(1+x)/4 P_{p-2}^{alpha,beta}(x).
    Returns (values, derivatives) with shape [P+1, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    V = np.zeros((P + 1, x.size))
    Dv = np.zeros((P + 1, x.size))
    V[0], Dv[0] = 0.5 * (1.0 - x), -0.5
    V[1], Dv[1] = 0.5 * (1.0 + x), 0.5
    for p in range(2, P + 1):
        j, dj = jacobi(p - 2, alpha, beta, x)
        bub = 0.25 * (1.0 - x) * (1.0 + x)
        V[p] = bub * j
        Dv[p] = -0.5 * x * j + bub * dj
    return V, Dv


def nodal_start(P, x):
    """Lagrange polynomials on the GLL points (Eq. lagrangian), values and
    derivatives, shape [P+1, len(x)]; index a follows the points left to right."""
    x = np.asarray(x, dtype=np.float64)
    z = gll_points(P)
    n = P + 1
    V = np.ones((n, x.size))
    Dv = np.zeros((n, x.size))
    for a in range(n):
        for b in range(n):
            if b != a:
                V[a] *= (x - z[b]) / (z[a] - z[b])
        for m in range(n):
            if m == a:
                continue
            t = np.full(x.size, 1.0 / (z[a] - z[m]))
            for b in range(n):
                if b != a and b != m:
                    t *= (x - z[b]) / (z[a] - z[b])
            Dv[a] += t
    return V, Dv


def _start(P, start, x):
    if start == "modal":
        V, Dv = modal_start(P, x)
        return V, Dv, [0, 1], list(range(2, P + 1))
    if start == "nodal":
        V, Dv = nodal_start(P, x)
        return V, Dv, [0, P], list(range(1, P))
    raise ValueError(start)


def mass_stiffness(P, start):
    """1D element mass and stiffness of the starting basis (Eqs. Matrizesmassa,
    Matrizesrigidez), integrated exactly with P+2 Gauss points (degree 2P)."""
    xg, wg = gauss_legendre(P + 2)
    V, Dv, vi, ii = _start(P, start, xg)
    M = (V * wg) @ V.T
    K = (Dv * wg) @ Dv.T
    return M, K, vi, ii


class Basis1D:
    """A 1D basis: coefficient matrix T (slots x starting index) and the data
    needed to evaluate and report it."""

    def __init__(self, P, kind, k=0.5, lam=100.0, start="modal"):
        self.P, self.kind, self.k, self.lam = P, kind, k, lam
        if kind == NODAL:
            start = "nodal"
        elif kind == MODAL:
            start = "modal"
        self.start = start
        n = P + 1
        M, K, vi, ii = mass_stiffness(P, start)
        self.lambda_s = np.zeros(max(P - 1, 0))
        T = np.zeros((n, n))
        if kind in (NODAL, MODAL) or P < 2:
            # slot 0 = left vertex, P = right vertex, internal in natural order
            T[0, vi[0]] = 1.0
            T[P, vi[1]] = 1.0
            for s, m in enumerate(ii, start=1):
                T[s, m] = 1.0
            if kind not in (NODAL, MODAL) and P == 1:
                pass  # no internal modes: SDME of order 1 is the linear basis
        else:
            Mii = M[np.ix_(ii, ii)]
            Kii = K[np.ix_(ii, ii)]
            # simultaneous diagonalisation (Eqs. diagMassa, L, diagL, Y)
            lam_m, X = np.linalg.eigh(Mii)
            Xs = X @ np.diag(lam_m ** -0.5)
            L = Xs.T @ Kii @ Xs
            lam_s, Z = np.linalg.eigh(0.5 * (L + L.T))
            Y = (Xs @ Z @ np.diag(lam_s ** (-0.5 * k))).T
            self.lambda_s = lam_s
            Tint = np.zeros((P - 1, n))
            Tint[:, ii] = Y
            # sign: derivative at xi = -1 positive
            _, d0 = _start(P, start, np.array([-1.0]))[:2]
            dm1 = Tint @ d0[:, 0]
            Tint *= np.where(dm1 < 0.0, -1.0, 1.0)[:, None]
            # minimum-energy vertex modes (Eqs. ExtensaoMEmassa .. alphaKN)
            if kind == SDME_M:
                A = M
            elif kind == SDME_K:
                A = K
            elif kind == SDME_H:
                A = K + lam * M
            else:
                raise ValueError(kind)
            Avi = np.array([[Tint[j] @ A[vv] for j in range(P - 1)] for vv in vi])
            Aii = Tint @ A @ Tint.T
            alpha = Avi @ np.linalg.inv(Aii)
            self.alpha = alpha
            for slot, vv, row in ((0, vi[0], 0), (P, vi[1], 1)):
                T[slot, vv] = 1.0
                T[slot] -= alpha[row] @ Tint
            T[1:P] = Tint
        self.T = T
        self.M1 = T @ M @ T.T
        self.K1 = T @ K @ T.T

    def eval(self, x):
        """Values and derivatives of the slots at points x: arrays [len(x), P+1]."""
        V, Dv, _, _ = _start(self.P, self.start, np.atleast_1d(x))
        return (self.T @ V).T, (self.T @ Dv).T

    def tables(self, Q):
        """Points/weights of the volume rule with Q points (volume_rule) and
        B[q][s], D[q][s] there."""
        x, w = volume_rule(self.P, Q)
        B, D = self.eval(x)
        return x, w, B, D

    def affine_coeffs(self):
        """Coefficients gamma1, gammax with 1 = sum gamma1[s] phi_s(xi) and
        xi = sum gammax[s] phi_s(xi): the 1D expansion of the functions 1 and xi,
        obtained by L2 projection onto the span (exact: both lie in it)."""
        x, w = gauss_legendre(self.P + 2)
        B, _ = self.eval(x)
        G = (B.T * w) @ B
        g1 = np.linalg.solve(G, B.T @ w)
        gx = np.linalg.solve(G, B.T @ (w * x))
        return g1, gx


def build(P, Q, kind, k=0.5, lam=100.0, start="modal"):
    """Convenience: (basis, x, w, B, D) for the element tables at Q points."""
    b = Basis1D(P, kind, k=k, lam=lam, start=start)
    x, w, B, D = b.tables(Q)
    return b, x, w, B, D
