"""Dense NumPy brute force for small systems (test-side checker).

Builds the full matrices of Sec. 4.1 with Kronecker products so that the
oracle's loop-based operators and factorizations can be compared with the
definitions written as plain linear algebra.
"""
import numpy as np


def dense_J(sys, k=0):
    T, m = sys.T, sys.m
    D = np.zeros((T * m, T * m))
    for i in range(T):
        for a in range(sys.row_ptr[i], sys.row_ptr[i + 1]):
            j = sys.col_idx[a]
            D[i * m:(i + 1) * m, j * m:(j + 1) * m] = sys.J[k if sys.nJ > 1 else 0, a]
    return D


def dense_M(sys):
    T, m = sys.T, sys.m
    D = np.zeros((T * m, T * m))
    for i in range(T):
        D[i * m:(i + 1) * m, i * m:(i + 1) * m] = sys.M[i]
    return D


def blockdiag(mats):
    n = sum(a.shape[0] for a in mats)
    D = np.zeros((n, n))
    o = 0
    for a in mats:
        D[o:o + a.shape[0], o:o + a.shape[0]] = a
        o += a.shape[0]
    return D


def dense_B(sys, Ainv, dt=None, s=None):
    """A^{-1} (x) M - dt diag(J_1..J_s)  (Eq. big-irk)."""
    s = sys.s if s is None else s
    dt = sys.dt if dt is None else dt
    Js = [dense_J(sys, k) for k in range(s)]
    return np.kron(Ainv, dense_M(sys)) - dt * blockdiag(Js)


def dense_B_untransformed(sys, A, dt=None, s=None):
    """I (x) M - dt [a_kl J_k]  (Eq. newton-system-2)."""
    s = sys.s if s is None else s
    dt = sys.dt if dt is None else dt
    n = sys.T * sys.m
    D = np.kron(np.eye(s), dense_M(sys))
    for k in range(s):
        Jk = dense_J(sys, k)
        for l in range(s):
            D[k * n:(k + 1) * n, l * n:(l + 1) * n] -= dt * A[k, l] * Jk
    return D


def factors_dense(bm):
    """(L~, U~) of a factored oracle.BlockMatrix as dense matrices."""
    m = bm.m
    N = bm.nb * m
    L = np.eye(N)
    U = np.zeros((N, N))
    for i in range(bm.nb):
        for a in range(bm.ptr[i], bm.ptr[i + 1]):
            j = bm.col[a]
            blk = bm.val[a]
            if j < i:
                L[i * m:(i + 1) * m, j * m:(j + 1) * m] = blk
            else:
                U[i * m:(i + 1) * m, j * m:(j + 1) * m] = blk
    return L, U
