"""ORACLE -- test infrastructure only.

Static condensation of the element-interior modes (Section 4: the Schur
complement of the interior block, Eqs. Eq:Matrix_form_schur1, Schur_split1,
Schur_split2, Eq:Newmark_Matrix_form_schur1), done densely on small meshes:
the global matrix of the operator is formed column by column from the
oracle's direct operator actions, restricted to the free DOFs, and the
interior unknowns are eliminated by their definition,

    S = A_BB - A_BI A_II^-1 A_IB,   g = b_B - A_BI A_II^-1 b_I,
    x_B = S^-1 g,                  x_I = A_II^-1 (b_I - A_IB x_B).

An interior mode has all three tensor indices internal, i.e. its slot
(ix, iy, iz) has every index off the element boundaries (index mod P != 0).
The CG of the condensed system uses the diagonal of A_BB as preconditioner
(the preconditioner of the library's condensed solve).
"""
import numpy as np

from oracle import solvers as osv


def interior_slots(mesh):
    """Boolean [3 Nn]: DOFs on element-interior slots."""
    P = mesh.P
    g = np.arange(mesh.Nn)
    ix, iy, iz = g % mesh.Nx, (g // mesh.Nx) % mesh.Ny, g // (mesh.Nx * mesh.Ny)
    inner = (ix % P != 0) & (iy % P != 0) & (iz % P != 0)
    return np.tile(inner, 3)


def dense_operator(apply, N):
    """The matrix of a linear operator on R^N, column by column."""
    A = np.zeros((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        A[:, j] = apply(e)
        e[j] = 0.0
    return A


def partition(pb, A):
    """Free DOFs split into boundary (B) and interior (I) index sets."""
    free = pb.mask > 0
    inner = interior_slots(pb.mesh)
    B = np.flatnonzero(free & ~inner)
    I = np.flatnonzero(free & inner)
    return B, I


def condensed_system(A, b, B, I):
    """S and g of the condensed system (dense)."""
    AII = A[np.ix_(I, I)]
    AIB = A[np.ix_(I, B)]
    ABI = A[np.ix_(B, I)]
    X = np.linalg.solve(AII, np.column_stack([AIB, b[I]]))
    S = A[np.ix_(B, B)] - ABI @ X[:, :-1]
    g = b[B] - ABI @ X[:, -1]
    return S, g


def condensed_solve(A, b, B, I):
    """x on the free DOFs by condensation (zeros elsewhere)."""
    S, g = condensed_system(A, b, B, I)
    x = np.zeros_like(b)
    x[B] = np.linalg.solve(S, g)
    x[I] = np.linalg.solve(A[np.ix_(I, I)], b[I] - A[np.ix_(I, B)] @ x[B])
    return x


def condensed_pcg(A, b, B, I, rtol, maxit=100000):
    """Jacobi-preconditioned CG on the condensed system (diagonal of A_BB);
    returns (x on all DOFs, iterations)."""
    S, g = condensed_system(A, b, B, I)
    xB, its, _ = osv.pcg(lambda v: S @ v, g, np.diag(A)[B], rtol, maxit)
    x = np.zeros_like(b)
    x[B] = xB
    x[I] = np.linalg.solve(A[np.ix_(I, I)], b[I] - A[np.ix_(I, B)] @ xB)
    return x, its
