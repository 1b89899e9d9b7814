"""Dense-matrix helpers for pinning the oracle on tiny grids.

These build explicit sparse-pattern matrices from the stencil arrays with
numpy, so that the tests can check the oracle against linear algebra that
shares none of its code: the definition M = L U = A + N of Stone's method,
a textbook ILU(0), and dense triangular / full solves.
"""
import numpy as np

P, W, E, S, N, B, T = range(7)
LB, LW, LS, LP, UN, UE, UT = range(7)

# grid offsets (di, dj, dk) of the stencil directions
OFF = {P: (0, 0, 0), W: (-1, 0, 0), E: (1, 0, 0), S: (0, -1, 0), N: (0, 1, 0), B: (0, 0, -1), T: (0, 0, 1)}


def cells(ni, nj, nk):
    for k in range(nk):
        for j in range(nj):
            for i in range(ni):
                yield i, j, k


def lin(i, j, k, ni, nj):
    return i + ni * (j + nj * k)


def inside(i, j, k, ni, nj, nk):
    return 0 <= i < ni and 0 <= j < nj and 0 <= k < nk


def dense_A(A):
    """Dense matrix of a (7, nk, nj, ni) stencil; out-of-block couplings dropped."""
    _, nk, nj, ni = A.shape
    n = ni * nj * nk
    M = np.zeros((n, n))
    for i, j, k in cells(ni, nj, nk):
        p = lin(i, j, k, ni, nj)
        for d, (di, dj, dk) in OFF.items():
            if inside(i + di, j + dj, k + dk, ni, nj, nk):
                M[p, lin(i + di, j + dj, k + dk, ni, nj)] += A[d, k, j, i]
    return M


def dense_LU(LU):
    """Dense L (B, W, S, P diagonals) and unit-upper U (N, E, T) from factor arrays."""
    _, nk, nj, ni = LU.shape
    n = ni * nj * nk
    L = np.zeros((n, n))
    U = np.eye(n)
    for i, j, k in cells(ni, nj, nk):
        p = lin(i, j, k, ni, nj)
        L[p, p] = LU[LP, k, j, i]
        for f, d in ((LB, B), (LW, W), (LS, S)):
            di, dj, dk = OFF[d]
            if inside(i + di, j + dj, k + dk, ni, nj, nk):
                L[p, lin(i + di, j + dj, k + dk, ni, nj)] = LU[f, k, j, i]
        for f, d in ((UN, N), (UE, E), (UT, T)):
            di, dj, dk = OFF[d]
            if inside(i + di, j + dj, k + dk, ni, nj, nk):
                U[p, lin(i + di, j + dj, k + dk, ni, nj)] = LU[f, k, j, i]
    return L, U


# The six positions that L U adds to the 7-point pattern, each with the two
# stencil neighbours that span it (Q = Q1 + Q2 - P in grid offsets).
EXTRA = {
    "BN": (B, N), "BE": (B, E), "WN": (W, N), "WT": (W, T), "SE": (S, E), "ST": (S, T),
}


def stone_N(M, ni, nj, nk, alpha):
    """N expected by Stone's partial cancellation, built from the extra-diagonal
    entries e of M: N[P,Q] = e, N[P,Q1] = N[P,Q2] = -alpha e, N[P,P] = +alpha e
    (phi_Q ~ alpha (phi_Q1 + phi_Q2 - phi_P))."""
    n = M.shape[0]
    Nx = np.zeros((n, n))
    for i, j, k in cells(ni, nj, nk):
        p = lin(i, j, k, ni, nj)
        for d1, d2 in EXTRA.values():
            o1, o2 = OFF[d1], OFF[d2]
            qi, qj, qk = i + o1[0] + o2[0], j + o1[1] + o2[1], k + o1[2] + o2[2]
            if not inside(qi, qj, qk, ni, nj, nk):
                continue
            q = lin(qi, qj, qk, ni, nj)
            e = M[p, q]
            q1 = lin(i + o1[0], j + o1[1], k + o1[2], ni, nj)
            q2 = lin(i + o2[0], j + o2[1], k + o2[2], ni, nj)
            Nx[p, q] += e
            Nx[p, q1] -= alpha * e
            Nx[p, q2] -= alpha * e
            Nx[p, p] += alpha * e
    return Nx


def ilu0(Ad):
    """Textbook ILU(0) (IKJ Gaussian elimination with fill dropped outside the
    pattern of A).  Returns (Lunit, Uupper) with A ~ Lunit @ Uupper."""
    a = Ad.copy()
    n = a.shape[0]
    pat = Ad != 0.0
    for i in range(1, n):
        for k in range(i):
            if not pat[i, k]:
                continue
            a[i, k] /= a[k, k]
            for j in range(k + 1, n):
                if pat[i, j]:
                    a[i, j] -= a[i, k] * a[k, j]
    Lu = np.tril(a, -1) + np.eye(n)
    Uu = np.triu(a)
    return Lu, Uu


def random_mmatrix(ni, nj, nk, rng, symmetric=False):
    """Random diagonally dominant M-matrix stencil (negative couplings)."""
    A = np.empty((7, nk, nj, ni))
    A[1:] = -rng.uniform(0.2, 2.0, size=(6, nk, nj, ni))
    if symmetric:
        A[W, :, :, 1:] = A[E, :, :, :-1]
        A[S, :, 1:, :] = A[N, :, :-1, :]
        A[B, 1:, :, :] = A[T, :-1, :, :]
    A[W, :, :, 0] = 0
    A[E, :, :, -1] = 0
    A[S, :, 0, :] = 0
    A[N, :, -1, :] = 0
    A[B, 0, :, :] = 0
    A[T, -1, :, :] = 0
    A[P] = -A[1:].sum(axis=0) + rng.uniform(0.05, 1.0, size=(nk, nj, ni))
    return A
