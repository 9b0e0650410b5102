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

The lesser/greater solutions X^s = A^{-1} B^s A^{-dagger} follow the same
three phases: the right-hand side is permuted like A and carried through
the block factorisation A = L diag(A_II, S) U, which gives the reduced
right-hand side of the separators in phase 1, X^s_SS = X_SS B~ X_SS^dagger
in phase 2 and the interior blocks in phase 3 (formulas in the code).

The selected blocks (diagonal, first off-diagonals) are read from the
un-permuted results.  Plain dense arithmetic per step (complex128),
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


def nested_dissection_selected(Mt, P, Bs=()):
    """Selected blocks of X^R = Mt^{-1} and X^s = X^R B^s X^R^dagger by the
    partitioned scheme.

    Mt: (diag[n,b,b], upper[n-1,b,b], lower[n-1,b,b]); P: partitions; Bs:
    right-hand sides B^s as triples of the same shape (general blocks, no
    symmetry assumed).  Returns a dict with
      XR   (diag, upper, lower) of X^R,
      XS   [(diag, upper, lower) of X^s per right-hand side],
      S    reduced system (dense, separator order),
      BS   [reduced right-hand side per B^s (dense, separator order)],
      sep  separator block indices.
    """
    d, u, l = (np.asarray(t, dtype=np.complex128) for t in Mt)
    n, b = d.shape[0], d.shape[1]
    A = _dense(d, u, l)
    Bd = [_dense(*(np.asarray(t, dtype=np.complex128) for t in B)) for B in Bs]
    sep = separators(n, P)
    parts = partitions(n, P)
    interior = [[i for i in range(lo, hi) if i not in sep] for lo, hi in parts]
    inter = [i for blk in interior for i in blk]

    def rows(blocks):
        return np.concatenate([np.arange(i * b, (i + 1) * b) for i in blocks]) \
            if blocks else np.zeros(0, int)

    rI, rS = rows(inter), rows(sep)
    cut = lambda M, r, c: M[np.ix_(r, c)]
    A_II, A_IS, A_SI, A_SS = cut(A, rI, rI), cut(A, rI, rS), cut(A, rS, rI), cut(A, rS, rS)
    h = lambda M: M.conj().T
    # phase 1: interiors independently (A_II is block diagonal by partition)
    a = np.zeros_like(A_II)
    off = 0
    for blk in interior:
        k = len(blk) * b
        if k:
            a[off:off + k, off:off + k] = np.linalg.inv(A_II[off:off + k, off:off + k])
        off += k
    # phase 2: the reduced system on the separators
    S = A_SS - A_SI @ a @ A_IS
    X_SS = np.linalg.inv(S)
    # phase 3: interiors independently
    X_IS = -a @ A_IS @ X_SS
    X_SI = -X_SS @ A_SI @ a
    X_II = a + a @ A_IS @ X_SS @ A_SI @ a
    X = np.zeros_like(A)
    X[np.ix_(rI, rI)] = X_II
    X[np.ix_(rI, rS)] = X_IS
    X[np.ix_(rS, rI)] = X_SI
    X[np.ix_(rS, rS)] = X_SS

    # Lesser/greater: with A = L diag(A_II, S) U (L, U unit block
    # triangular), X^s = U^{-1} diag(a, X_SS) [L^{-1} B L^{-dagger}]
    # diag(a, X_SS)^dagger U^{-dagger}; every factor is applied in turn.
    XSs, BSs = [], []
    for B in Bd:
        B_II, B_IS, B_SI, B_SS = cut(B, rI, rI), cut(B, rI, rS), cut(B, rS, rI), cut(B, rS, rS)
        # phase 1: the reduced right-hand side (L^{-1} B L^{-dagger})_SS
        BS = B_SS - A_SI @ a @ B_IS - B_SI @ h(a) @ h(A_SI) + A_SI @ a @ B_II @ h(a) @ h(A_SI)
        # phase 2: the separators' block of the solution
        XS_SS = X_SS @ BS @ h(X_SS)
        # phase 3: the interiors
        C_IS = a @ (B_IS - B_II @ h(a) @ h(A_SI)) @ h(X_SS)
        C_SI = X_SS @ (B_SI - A_SI @ a @ B_II) @ h(a)
        XS_IS = C_IS - a @ A_IS @ XS_SS
        XS_SI = C_SI - XS_SS @ h(A_IS) @ h(a)
        XS_II = (a @ B_II @ h(a) - a @ A_IS @ C_SI - C_IS @ h(A_IS) @ h(a)
                 + a @ A_IS @ XS_SS @ h(A_IS) @ h(a))
        Y = np.zeros_like(A)
        Y[np.ix_(rI, rI)] = XS_II
        Y[np.ix_(rI, rS)] = XS_IS
        Y[np.ix_(rS, rI)] = XS_SI
        Y[np.ix_(rS, rS)] = XS_SS
        XSs.append(_selected(Y, n, b))
        BSs.append(BS)
    return {"XR": _selected(X, n, b), "XS": XSs, "S": S, "BS": BSs, "sep": sep}


def _selected(X, n, b):
    blk = lambda i, j: X[i * b:(i + 1) * b, j * b:(j + 1) * b]
    z = np.zeros((0, b, b), np.complex128)
    return (np.stack([blk(i, i) for i in range(n)]),
            np.stack([blk(i, i + 1) for i in range(n - 1)]) if n > 1 else z,
            np.stack([blk(i + 1, i) for i in range(n - 1)]) if n > 1 else z)
