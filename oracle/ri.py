"""RI assembly for the oracle (TEST INFRASTRUCTURE ONLY).

The paper's resolution-of-the-identity form of the electron-repulsion integrals (eq. 14) combines the
three-centre integrals (ab|P) with the inverse of the two-centre metric (P|Q).  Writing the metric
as its Cholesky factorisation (P|Q) = L L^T, the inverse splits into L^-T L^-1, so

    B[R, ab]  = sum_P (L^-1)[R, P] (ab|P)        (B solves L B = A, A[P, ab] = (ab|P))
    (ab|cd)  ~= sum_R B[R, ab] B[R, cd].

Pairs are the canonical pairs a >= b, index ab = a (a + 1) / 2 + b.  Everything here is plain FP64
numpy: the triangular solve is forward substitution written out row by row, the final sum is one
matrix product.
"""
import numpy as np


def pair_index(a, b):
    """Canonical pair index of basis functions a, b (order-free)."""
    a, b = max(a, b), min(a, b)
    return a * (a + 1) // 2 + b


def pairs_matrix(abP):
    """A[P, ab] = (ab|P) over canonical pairs, from abP laid out [P][a][b]."""
    na, nb, _ = abP.shape
    A = np.empty((na, nb * (nb + 1) // 2))
    for a in range(nb):
        for b in range(a + 1):
            A[:, pair_index(a, b)] = abP[:, a, b]
    return A


def forward_substitution(L, A):
    """Solve L X = A for lower-triangular L, one row of X at a time in increasing order."""
    n = L.shape[0]
    X = np.zeros_like(A)
    for r in range(n):
        X[r] = (A[r] - L[r, :r] @ X[:r]) / L[r, r]
    return X


def ri_assemble(abP, L):
    """(B, eri): B[R, ab] and the RI electron-repulsion matrix eri[ab, cd] (eq. 14)."""
    B = forward_substitution(np.asarray(L, dtype=np.float64), pairs_matrix(np.asarray(abP, dtype=np.float64)))
    return B, B.T @ B
