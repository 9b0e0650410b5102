"""Closed-form inverse of a scalar tridiagonal matrix (block size b = 1).

Independent pin for the oracle at b = 1: the entries of T^{-1} follow from
the continuants theta_k (leading k x k minors) and phi_k (trailing minors),
    theta_0 = 1, theta_1 = a_0, theta_k = a_{k-1} theta_{k-1} - c_{k-2} d_{k-2} theta_{k-2}
    phi_n = 1,  phi_{n-1} = a_{n-1}, phi_k = a_k phi_{k+1} - c_k d_k phi_{k+2}
    (T^{-1})_{ij} = (-1)^{i+j} c_i...c_{j-1} theta_i phi_{j+1} / theta_n   (i <= j)
    (T^{-1})_{ij} = (-1)^{i+j} d_j...d_{i-1} theta_j phi_{i+1} / theta_n   (i >  j)
(a = diagonal, c_i = T_{i,i+1}, d_i = T_{i+1,i}; 0-based).  The lesser
function X B X^dagger is then summed entry by entry.
"""

import numpy as np


def _full_inverse(a, c, d):
    n = a.shape[0]
    theta = np.zeros(n + 1, dtype=np.complex128)
    phi = np.zeros(n + 2, dtype=np.complex128)
    theta[0] = 1.0
    if n >= 1:
        theta[1] = a[0]
    for k in range(2, n + 1):
        theta[k] = a[k - 1] * theta[k - 1] - c[k - 2] * d[k - 2] * theta[k - 2]
    phi[n] = 1.0
    phi[n + 1] = 0.0
    if n >= 1:
        phi[n - 1] = a[n - 1]
    for k in range(n - 2, -1, -1):
        phi[k] = a[k] * phi[k + 1] - c[k] * d[k] * phi[k + 2]
    X = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            if i <= j:
                prod = np.prod(c[i:j]) if j > i else 1.0
                X[i, j] = (-1) ** (i + j) * prod * theta[i] * phi[j + 1] / theta[n]
            else:
                prod = np.prod(d[j:i])
                X[i, j] = (-1) ** (i + j) * prod * theta[j] * phi[i + 1] / theta[n]
    return X


def tridiag_inverse_selected(T, Bs=()):
    """Same result layout as ``oracle.rgf.rgf_selected`` for b = 1 blocks.

    T and each B are (diag[n,1,1], upper[n-1,1,1], lower[n-1,1,1]) triples.
    """
    a = T[0][:, 0, 0]
    c = T[1][:, 0, 0]
    d = T[2][:, 0, 0]
    n = a.shape[0]
    X = _full_inverse(a, c, d)

    def sel(M):
        dd = np.array([M[i, i] for i in range(n)]).reshape(n, 1, 1)
        uu = np.array([M[i, i + 1] for i in range(n - 1)]).reshape(n - 1, 1, 1)
        ll = np.array([M[i + 1, i] for i in range(n - 1)]).reshape(n - 1, 1, 1)
        return dd, uu, ll

    out = []
    for B in Bs:
        Bm = np.zeros((n, n), dtype=np.complex128)
        for i in range(n):
            Bm[i, i] = B[0][i, 0, 0]
        for i in range(n - 1):
            Bm[i, i + 1] = B[1][i, 0, 0]
            Bm[i + 1, i] = B[2][i, 0, 0]
        S = np.zeros((n, n), dtype=np.complex128)
        for i in range(n):
            for j in range(n):
                acc = 0.0j
                for k in range(n):
                    for m in range(n):
                        if Bm[k, m] != 0:
                            acc += X[i, k] * Bm[k, m] * np.conj(X[j, m])
                S[i, j] = acc
        out.append(sel(S))
    return sel(X), out
