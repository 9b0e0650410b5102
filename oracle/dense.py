"""The plain definition of the selected solution (Eq. system-solve).

X^R = Mt^{-1} and X^s = Mt^{-1} B^s Mt^{-dagger}, formed densely and then
cut back to the diagonal and first off-diagonal blocks ("selected" elements,
Sec. 3.2 "Selected System Solver").  O((n b)^3): only for small systems.
"""

import numpy as np


def dense_from_bt(diag, upper, lower):
    """Assemble a dense (n b) x (n b) matrix from block-tridiagonal blocks."""
    diag = np.asarray(diag)
    n, b = diag.shape[0], diag.shape[1]
    A = np.zeros((n * b, n * b), dtype=np.complex128)
    for i in range(n):
        A[i * b:(i + 1) * b, i * b:(i + 1) * b] = diag[i]
    for i in range(n - 1):
        A[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = upper[i]
        A[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = lower[i]
    return A


def _select(X, n, b):
    d = np.stack([X[i * b:(i + 1) * b, i * b:(i + 1) * b] for i in range(n)])
    if n > 1:
        u = np.stack([X[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b]
                      for i in range(n - 1)])
        l = np.stack([X[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b]
                      for i in range(n - 1)])
    else:
        u = np.zeros((0, b, b), dtype=np.complex128)
        l = np.zeros((0, b, b), dtype=np.complex128)
    return d, u, l


def dense_selected(Mt, Bs=()):
    """Same interface and result layout as ``oracle.rgf.rgf_selected``."""
    n, b = Mt[0].shape[0], Mt[0].shape[1]
    A = dense_from_bt(*Mt)
    X = np.linalg.inv(A)
    XR = _select(X, n, b)
    XS = []
    for B in Bs:
        Bd = dense_from_bt(*B)
        XS.append(_select(X @ Bd @ X.conj().T, n, b))
    return XR, XS
