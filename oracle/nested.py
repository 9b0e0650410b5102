"""Nested-dissection selected inversion (the partitioned solver of Sec. 4.4).

TEST INFRASTRUCTURE ONLY (see the package header).

The block rows 0..n-1 of a block-tridiagonal matrix A are split into P_S
contiguous partitions: one top, P_S - 2 middle, one bottom.  The blocks that
touch a neighbouring partition are the separators: the last block of the
top partition, the first and last blocks of each middle partition, the first
block of the bottom partition.  Every other block is interior.  Interior
blocks of different partitions never couple, so after the permutation that
puts all interior blocks first (partition by partition) and the separators
last,

    P A P^T = [[A_II, A_IS], [A_SI, A_SS]],   A_II block diagonal by partition,

and the steps are the scheme's three phases:

1. per partition (independent, "forward"): A_II^{-1} of its interior and its
   contribution A_SI A_II^{-1} A_IS to the reduced system;
2. the reduced system S = A_SS - A_SI A_II^{-1} A_IS on the separators (block
   tridiagonal in separator order, with the fill-in coupling the two
   separators of each middle partition) and X_SS = S^{-1};
3. per partition (independent, "backward"):
       X_IS = -A_II^{-1} A_IS X_SS,   X_SI = -X_SS A_SI A_II^{-1},
       X_II = A_II^{-1} + A_II^{-1} A_IS X_SS A_SI A_II^{-1}.

The selected blocks of X^R = A^{-1} (diagonal, first off-diagonals) are read
from the un-permuted result.  Plain dense arithmetic per step (complex128),
meant to be checked by eye; pins in tests/test_oracle_nested.py.
"""

import numpy as np


def partitions(n, P):
    """Contiguous block ranges [lo, hi) of the P partitions (as equal as
    possible; middle partitions need at least two blocks)."""
    if P < 2:
        raise ValueError("at least two partitions")
    sizes = [n // P + (1 if p < n % P else 0) for p in range(P)]
    if sizes[0] < 1 or sizes[-1] < 1 or any(s < 2 for s in sizes[1:-1]):
        raise ValueError("too few blocks for %d partitions" % P)
    out, lo = [], 0
    for s in sizes:
        out.append((lo, lo + s))
        lo += s
    return out


def separators(n, P):
    """Sorted separator block indices."""
    parts = partitions(n, P)
    sep = {parts[0][1] - 1, parts[-1][0]}
    for lo, hi in parts[1:-1]:
        sep.update((lo, hi - 1))
    return sorted(sep)


def _dense(d, u, l):
    n, b = d.shape[0], d.shape[1]
    A = np.zeros((n * b, n * b), np.complex128)
    for i in range(n):
        A[i * b:(i + 1) * b, i * b:(i + 1) * b] = d[i]
        if i + 1 < n:
            A[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = u[i]
            A[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = l[i]
    return A


def nested_dissection_selected(Mt, P):
    """Selected blocks of X^R = Mt^{-1} by the partitioned scheme.

    Mt: (diag[n,b,b], upper[n-1,b,b], lower[n-1,b,b]); P: partitions.
    Returns ((diag, upper, lower) of X^R, reduced system S (dense, separator
    order), separator block indices)."""
    d, u, l = (np.asarray(t, dtype=np.complex128) for t in Mt)
    n, b = d.shape[0], d.shape[1]
    A = _dense(d, u, l)
    sep = separators(n, P)
    parts = partitions(n, P)
    interior = [[i for i in range(lo, hi) if i not in sep] for lo, hi in parts]
    inter = [i for blk in interior for i in blk]

    def rows(blocks):
        return np.concatenate([np.arange(i * b, (i + 1) * b) for i in blocks]) \
            if blocks else np.zeros(0, int)

    rI, rS = rows(inter), rows(sep)
    A_II = A[np.ix_(rI, rI)]
    A_IS = A[np.ix_(rI, rS)]
    A_SI = A[np.ix_(rS, rI)]
    A_SS = A[np.ix_(rS, rS)]
    # phase 1: interiors independently (A_II is block diagonal by partition)
    iA_II = np.zeros_like(A_II)
    off = 0
    for blk in interior:
        k = len(blk) * b
        if k:
            iA_II[off:off + k, off:off + k] = np.linalg.inv(A_II[off:off + k, off:off + k])
        off += k
    # phase 2: the reduced system on the separators
    S = A_SS - A_SI @ iA_II @ A_IS
    X_SS = np.linalg.inv(S)
    # phase 3: interiors independently
    X_IS = -iA_II @ A_IS @ X_SS
    X_SI = -X_SS @ A_SI @ iA_II
    X_II = iA_II + iA_II @ A_IS @ X_SS @ A_SI @ iA_II
    X = np.zeros_like(A)
    X[np.ix_(rI, rI)] = X_II
    X[np.ix_(rI, rS)] = X_IS
    X[np.ix_(rS, rI)] = X_SI
    X[np.ix_(rS, rS)] = X_SS
    blk = lambda i, j: X[i * b:(i + 1) * b, j * b:(j + 1) * b]
    XR = (np.stack([blk(i, i) for i in range(n)]),
          np.stack([blk(i, i + 1) for i in range(n - 1)]),
          np.stack([blk(i + 1, i) for i in range(n - 1)]))
    return XR, S, sep
