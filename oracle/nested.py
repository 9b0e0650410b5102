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


# ---------------------------------------------------------------------------
# The same scheme in block form, as each partition would run it on its own
# device: a block-tridiagonal elimination along the partition with the
# fill-in of Fig. nested-dissection, then the reduced system, then the
# partition's backward recursion.
#
# Elimination order.  The top partition eliminates its interior top-down
# towards its separator (its last block), the bottom partition bottom-up
# towards its separator (its first block); both are the plain forward
# recursion of Sec. 3.2.3 stopped before the separator.  A middle partition
# eliminates its interior top-down while its first block T (the top
# separator) stays; every elimination then couples the next block to T
# (the fill-in column M_{k,T} and row M_{T,k}), updates T's own block, and
# leaves T coupled to the bottom separator when the interior is done.
#
# One elimination step.  Let k be the block eliminated and N the blocks it
# is still coupled to (the next block of the chain, and T in a middle
# partition).  With x_k = (current diagonal block)^{-1}, the Schur
# complement updates every pair (i, j) of N by
#     M_ij -= M_ik x_k M_kj,
#     R_ij -= l_i R_kj + R_ik l_j^dagger - l_i R_kk l_j^dagger,   l_i = M_ik x_k,
# (R is the right-hand side, carried as L^{-1} B L^{-dagger}), and once the
# blocks of N are known the backward step recovers k from them:
#     X_kN  = -x_k M_kN X_NN,          X_Nk = -X_NN M_Nk x_k,
#     X_kk  =  x_k + x_k M_kN X_NN M_Nk x_k,
#     X^s_kN = -x_k M_kN X^s_NN - x^s_k (X_NN M_Nk)^dagger + x_k R_kN X_NN^dagger,
#     X^s_Nk = -X^s_NN (x_k M_kN)^dagger - X_NN M_Nk x^s_k + X_NN R_Nk x_k^dagger,
#     X^s_kk =  x^s_k + P X^s_NN P^dagger + Z x^s_k + x^s_k Z^dagger
#               - x_k R_kN X_NN^dagger P^dagger - P X_NN R_Nk x_k^dagger,
# with x^s_k = x_k R_kk x_k^dagger, P = x_k M_kN, Z = P X_NN M_Nk; these are
# the forward-pass / backward-pass relations of Sec. 3.2.3 with the single
# neighbour replaced by the set N (general B: no symmetry is assumed).
# ---------------------------------------------------------------------------


def nested_dissection_blocks(Mt, P, Bs=()):
    """Selected blocks of X^R and X^s by the partitioned scheme in block form.

    Same arguments as nested_dissection_selected; returns a dict with XR, XS
    (selected triples) and the reduced system S and right-hand sides BS
    (dense, separator order), as that function does.
    """
    d, u, l = (np.asarray(t, dtype=np.complex128) for t in Mt)
    n, b = d.shape[0], d.shape[1]
    Bt = [tuple(np.asarray(t, dtype=np.complex128) for t in B) for B in Bs]
    h = lambda M: M.conj().T
    inv = np.linalg.inv

    def blk(T, i, j):
        """Block (i, j) of a block-tridiagonal triple (zero off the band)."""
        if i == j:
            return T[0][i]
        if j == i + 1:
            return T[1][i]
        if i == j + 1:
            return T[2][j]
        return np.zeros((b, b), np.complex128)

    A = lambda i, j: blk((d, u, l), i, j)
    parts = partitions(n, P)
    sep = separators(n, P)
    jx = {s: q for q, s in enumerate(sep)}
    ns = len(sep)
    S = np.zeros((ns * b, ns * b), np.complex128)
    BS = [np.zeros_like(S) for _ in Bt]

    def put(M, i, j, v):
        M[jx[i] * b:(jx[i] + 1) * b, jx[j] * b:(jx[j] + 1) * b] = v

    def get(M, i, j):
        return M[jx[i] * b:(jx[i] + 1) * b, jx[j] * b:(jx[j] + 1) * b]

    # couplings between the separators of neighbouring partitions: original
    for p in range(P - 1):
        i, j = parts[p][1] - 1, parts[p + 1][0]
        put(S, i, j, A(i, j))
        put(S, j, i, A(j, i))
        for s, B in enumerate(Bt):
            put(BS[s], i, j, blk(B, i, j))
            put(BS[s], j, i, blk(B, j, i))

    # ---- phase 1: every partition's forward elimination ----------------
    saved = []
    for p, (lo, hi) in enumerate(parts):
        if p == 0:
            chain, N, T = list(range(lo, hi - 1)), hi - 1, None
        elif p == P - 1:
            chain, N, T = list(range(hi - 1, lo, -1)), lo, None
        else:
            chain, N, T = list(range(lo + 1, hi - 1)), hi - 1, lo
        m = len(chain)
        st = {"chain": chain, "N": N, "T": T, "x": [], "xs": [], "q": [], "r": [],
              "RkT": [], "RTk": []}
        if m == 0:
            SNN = A(N, N)
            RNN = [blk(B, N, N) for B in Bt]
            if T is not None:
                STT, STN, SNT = A(T, T), A(T, N), A(N, T)
                RTT = [blk(B, T, T) for B in Bt]
                RTN = [blk(B, T, N) for B in Bt]
                RNT = [blk(B, N, T) for B in Bt]
        else:
            c0 = chain[0]
            D = A(c0, c0)
            Rkk = [blk(B, c0, c0) for B in Bt]
            if T is not None:
                q, r, STT = A(c0, T), A(T, c0), A(T, T)
                RkT = [blk(B, c0, T) for B in Bt]
                RTk = [blk(B, T, c0) for B in Bt]
                RTT = [blk(B, T, T) for B in Bt]
            for k, c in enumerate(chain):
                x = inv(D)
                st["x"].append(x)
                st["xs"].append([x @ R @ h(x) for R in Rkk])
                nx = chain[k + 1] if k + 1 < m else N
                ln = A(nx, c) @ x
                Dn = A(nx, nx) - ln @ A(c, nx)
                Rn = [blk(B, nx, nx) - ln @ blk(B, c, nx) - blk(B, nx, c) @ h(ln)
                      + ln @ Rkk[s] @ h(ln) for s, B in enumerate(Bt)]
                if T is not None:
                    st["q"].append(q)
                    st["r"].append(r)
                    st["RkT"].append(list(RkT))
                    st["RTk"].append(list(RTk))
                    lT = r @ x
                    qn = -ln @ q
                    rn = -lT @ A(c, nx)
                    STT = STT - lT @ q
                    RnT = [-ln @ RkT[s] - blk(B, nx, c) @ h(lT) + ln @ Rkk[s] @ h(lT)
                           for s, B in enumerate(Bt)]
                    RTn = [-lT @ blk(B, c, nx) - RTk[s] @ h(ln) + lT @ Rkk[s] @ h(ln)
                           for s, B in enumerate(Bt)]
                    RTT = [RTT[s] - lT @ RkT[s] - RTk[s] @ h(lT) + lT @ Rkk[s] @ h(lT)
                           for s in range(len(Bt))]
                    q, r, RkT, RTk = qn, rn, RnT, RTn
                D, Rkk = Dn, Rn
            SNN, RNN = D, Rkk
            if T is not None:
                STN, SNT, RTN, RNT = r, q, RTk, RkT
        put(S, N, N, SNN)
        for s in range(len(Bt)):
            put(BS[s], N, N, RNN[s])
        if T is not None:
            put(S, T, T, STT)
            put(S, T, N, STN)
            put(S, N, T, SNT)
            for s in range(len(Bt)):
                put(BS[s], T, T, RTT[s])
                put(BS[s], T, N, RTN[s])
                put(BS[s], N, T, RNT[s])
        saved.append(st)

    # ---- phase 2: the reduced system ------------------------------------
    XS_ = inv(S)
    XSs_ = [XS_ @ R @ h(XS_) for R in BS]

    # ---- phase 3: every partition's backward recursion --------------------
    X, Xs = {}, [dict() for _ in Bt]
    for i in sep:
        for j in sep:
            if abs(i - j) <= 1:
                X[(i, j)] = get(XS_, i, j)
                for s in range(len(Bt)):
                    Xs[s][(i, j)] = get(XSs_[s], i, j)
    for st in saved:
        chain, N, T = st["chain"], st["N"], st["T"]
        idx = [N] if T is None else [N, T]
        XNN = np.block([[get(XS_, i, j) for j in idx] for i in idx])
        XsNN = [np.block([[get(R, i, j) for j in idx] for i in idx]) for R in XSs_]
        for k in range(len(chain) - 1, -1, -1):
            c = chain[k]
            nx = chain[k + 1] if k + 1 < len(chain) else N
            x, xs = st["x"][k], st["xs"][k]
            if T is None:
                MkN, MNk = A(c, nx), A(nx, c)
                RkN = [blk(B, c, nx) for B in Bt]
                RNk = [blk(B, nx, c) for B in Bt]
            else:
                MkN = np.hstack([A(c, nx), st["q"][k]])
                MNk = np.vstack([A(nx, c), st["r"][k]])
                RkN = [np.hstack([blk(B, c, nx), st["RkT"][k][s]]) for s, B in enumerate(Bt)]
                RNk = [np.vstack([blk(B, nx, c), st["RTk"][k][s]]) for s, B in enumerate(Bt)]
            Pk = x @ MkN
            Zk = Pk @ XNN @ MNk
            XkN = -Pk @ XNN
            XNk = -XNN @ MNk @ x
            Xkk = x + Zk @ x
            XskN, XsNk, Xskk = [], [], []
            for s in range(len(Bt)):
                XskN.append(-Pk @ XsNN[s] - xs[s] @ h(XNN @ MNk) + x @ RkN[s] @ h(XNN))
                XsNk.append(-XsNN[s] @ h(Pk) - XNN @ MNk @ xs[s] + XNN @ RNk[s] @ h(x))
                Xskk.append(xs[s] + Pk @ XsNN[s] @ h(Pk) + Zk @ xs[s] + xs[s] @ h(Zk)
                            - x @ RkN[s] @ h(XNN) @ h(Pk) - Pk @ XNN @ RNk[s] @ h(x))
            X[(c, c)] = Xkk
            X[(c, nx)] = XkN[:, :b]
            X[(nx, c)] = XNk[:b]
            for s in range(len(Bt)):
                Xs[s][(c, c)] = Xskk[s]
                Xs[s][(c, nx)] = XskN[s][:, :b]
                Xs[s][(nx, c)] = XsNk[s][:b]
            if T is not None and k == 0:
                # the first interior block neighbours T
                X[(c, T)] = XkN[:, b:]
                X[(T, c)] = XNk[b:]
                for s in range(len(Bt)):
                    Xs[s][(c, T)] = XskN[s][:, b:]
                    Xs[s][(T, c)] = XsNk[s][b:]
            if T is None:
                XNN = Xkk
                XsNN = Xskk
            else:
                XNN = np.block([[Xkk, XkN[:, b:]], [XNk[b:], XNN[b:, b:]]])
                XsNN = [np.block([[Xskk[s], XskN[s][:, b:]], [XsNk[s][b:], XsNN[s][b:, b:]]])
                        for s in range(len(Bt))]

    def sel(Y):
        z = np.zeros((0, b, b), np.complex128)
        return (np.stack([Y[(i, i)] for i in range(n)]),
                np.stack([Y[(i, i + 1)] for i in range(n - 1)]) if n > 1 else z,
                np.stack([Y[(i + 1, i)] for i in range(n - 1)]) if n > 1 else z)

    return {"XR": sel(X), "XS": [sel(Y) for Y in Xs], "S": S, "BS": BS, "sep": sep}
