"""Independent numpy/scipy checks for the oracle (tiny blocks only).

Nothing here shares code with ``oracle/``: the operator is built from 1D
path-graph Laplacians by Kronecker products, Eq. (1) of Sec. 2.1 is solved
as one dense N x N system, G is taken from ``numpy.linalg.pinv`` (Sec. 2.2:
the Green's functions form the pseudo-inverse of A) and the DCT form of
Eq. (4) uses ``scipy.fft.dctn``/``idctn`` with orthonormal scaling.
"""
from __future__ import annotations

import numpy as np
import scipy.fft


def path_laplacian(n: int) -> np.ndarray:
    """Graph Laplacian of the path on n nodes (-d^2/dx^2 with mirrored ends)."""
    T = np.zeros((n, n))
    for i in range(n - 1):
        T[i, i] += 1
        T[i + 1, i + 1] += 1
        T[i, i + 1] -= 1
        T[i + 1, i] -= 1
    return T


def neg_laplacian(w: int, h: int) -> np.ndarray:
    """-L on a w x h block, pixels row-major (index y*w + x)."""
    return np.kron(np.eye(h), path_laplacian(w)) + np.kron(path_laplacian(h), np.eye(w))


def operator(w: int, h: int, s: int = 1) -> np.ndarray:
    return np.linalg.matrix_power(neg_laplacian(w, h), s)


def solve_eq1(w: int, h: int, pos, r, A: np.ndarray) -> np.ndarray:
    """Eq. (1): M (u - f) - (I - M) A u = 0, dense solve; returns (h, w)."""
    N = w * h
    m = np.zeros(N)
    f = np.zeros(N)
    m[np.asarray(pos, dtype=np.int64)] = 1.0
    f[np.asarray(pos, dtype=np.int64)] = r
    M = np.diag(m)
    S = M - (np.eye(N) - M) @ A
    return np.linalg.solve(S, M @ f).reshape(h, w)


def dct_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix C (C @ x == scipy dct(x, norm='ortho'))."""
    return scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0)


def eq4_evaluate(w: int, h: int, pos, c, a: float, lam: np.ndarray) -> np.ndarray:
    """Eq. (4): u = C^-1 diag(lambda) C (M c) + a with scipy's 2D DCT-II."""
    Mc = np.zeros(w * h)
    Mc[np.asarray(pos, dtype=np.int64)] = c
    spec = scipy.fft.dctn(Mc.reshape(h, w), type=2, norm="ortho")
    return scipy.fft.idctn(lam * spec, type=2, norm="ortho") + a
