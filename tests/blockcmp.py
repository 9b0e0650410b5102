"""Per-block relative Frobenius error used by every parity test.

err(X_i) = ||X_i - R_i||_F / ||R_i||_F for each block i of one output
(diag, upper or lower) at one energy; when ||R_i||_F is below 1e-13 times the
largest block norm of that output at that energy, the largest block norm is
the denominator instead (tiny blocks carry no relative information).
"""

import numpy as np


def block_rel_err(X, R, floor=1e-13):
    X = np.asarray(X)
    R = np.asarray(R)
    if R.size == 0:
        return np.zeros(R.shape[:-2])
    num = np.linalg.norm(X - R, axis=(-2, -1))
    den = np.linalg.norm(R, axis=(-2, -1))
    # max over the block axis (axis -1 of den) per leading index
    big = np.max(den, axis=-1, keepdims=True) if den.ndim >= 1 else den
    den = np.where(den < floor * big, big, den)
    den = np.where(den == 0, 1.0, den)
    return num / den


def max_rel_err(X, R):
    e = block_rel_err(X, R)
    return float(np.max(e)) if e.size else 0.0


def triple_err(XT, RT):
    return max(max_rel_err(x, r) for x, r in zip(XT, RT))
