"""Assembly of the block-tridiagonal system (paper Sec. 3.2.2 and Table
"quantities").

Electrons (G-type):
    Mt(E)  = E S - H - Sigma^R(E)            (Sigma^R includes the OBC blocks)
    B^s(E) = Sigma^s(E)
Screened Coulomb (W-type):
    Mt(E)  = I - V P^R(E)
    B^s(E) = V P^s(E) V^dagger
For W the products are formed in the block-tridiagonal (BT) representation:
V and P are BT, V P^R has block bandwidth five and V P^s V^dagger seven; the
system is kept block-tridiagonal by dropping every block with |i-j| > 1, the
cut-off that the BT grouping of the device imposes.

Blocks are plain loops over block indices; a dense version of the same
products is used by the tests to check these loops.
"""

import numpy as np


def _bt_get(T, i, j, n):
    """Block (i, j) of a BT triple (diag, upper, lower), None when zero."""
    d, u, l = T
    if i == j:
        return d[i]
    if j == i + 1 and u is not None:
        return u[i]
    if i == j + 1 and l is not None:
        return l[j]
    return None


def _banded_product(Tl, Tr, n, bw_l, bw_r):
    """Blocks of Tl @ Tr for block-banded operands, as a dict {(i,j): blk}.

    Tl, Tr are callables (i, j) -> block or None with block bandwidths bw_l
    and bw_r; the product has bandwidth bw_l + bw_r.
    """
    out = {}
    bw = bw_l + bw_r
    for i in range(n):
        for j in range(max(0, i - bw), min(n, i + bw + 1)):
            acc = None
            for k in range(max(0, i - bw_l), min(n, i + bw_l + 1)):
                if abs(k - j) > bw_r:
                    continue
                a = Tl(i, k)
                bblk = Tr(k, j)
                if a is None or bblk is None:
                    continue
                term = a @ bblk
                acc = term if acc is None else acc + term
            if acc is not None:
                out[(i, j)] = acc
    return out


def _truncate_bt(blocks, n, b):
    d = np.zeros((n, b, b), dtype=np.complex128)
    u = np.zeros((max(n - 1, 0), b, b), dtype=np.complex128)
    l = np.zeros((max(n - 1, 0), b, b), dtype=np.complex128)
    for (i, j), blk in blocks.items():
        if i == j:
            d[i] = blk
        elif j == i + 1:
            u[i] = blk
        elif i == j + 1:
            l[j] = blk
    return d, u, l


def assemble_g(E, H, sigma_r, S=None):
    """Mt = E S - H - Sigma^R for one energy.

    H, sigma_r, S : BT triples (diag, upper, lower); sigma_r upper/lower and
    S may be None (zero off-diagonal self-energy; S = identity).
    """
    Hd, Hu, Hl = H
    n, b = Hd.shape[0], Hd.shape[1]
    eye = np.eye(b, dtype=np.complex128)
    Sd = S[0] if S is not None else np.broadcast_to(eye, (n, b, b))
    Su = S[1] if S is not None and S[1] is not None else None
    Sl = S[2] if S is not None and S[2] is not None else None
    Rd, Ru, Rl = sigma_r
    d = E * Sd - Hd - Rd
    u = -Hu.copy()
    l = -Hl.copy()
    if Su is not None:
        u = u + E * Su
    if Sl is not None:
        l = l + E * Sl
    if Ru is not None:
        u = u - Ru
    if Rl is not None:
        l = l - Rl
    return d, u, l


def assemble_w(V, P_r, P_s_list):
    """W-type system for one energy.

    V       : BT triple of the bare Coulomb matrix (energy independent)
    P_r     : BT triple of the retarded polarization P^R(E)
    P_s_list: BT triples of P^<(E), P^>(E)
    Returns Mt = I - trunc(V P^R) and [trunc(V P^s V^dagger), ...].
    """
    n, b = V[0].shape[0], V[0].shape[1]
    Vf = lambda i, j: _bt_get(V, i, j, n)
    Vh = lambda i, j: (None if _bt_get(V, j, i, n) is None
                       else _bt_get(V, j, i, n).conj().T)    # (V^dag)_{ij}
    Pr = lambda i, j: _bt_get(P_r, i, j, n)
    VP = _banded_product(Vf, Pr, n, 1, 1)
    md, mu, ml = _truncate_bt(VP, n, b)
    eye = np.eye(b, dtype=np.complex128)
    Mt = (eye[None] - md, -mu, -ml)
    Bs = []
    for P_s in P_s_list:
        Ps = lambda i, j, P_s=P_s: _bt_get(P_s, i, j, n)
        VPs = _banded_product(Vf, Ps, n, 1, 1)
        VPsf = lambda i, j: VPs.get((i, j))
        VPsVh = _banded_product(VPsf, Vh, n, 2, 1)
        Bs.append(_truncate_bt(VPsVh, n, b))
    return Mt, Bs


def w_retarded_diag(XR, V):
    """Diagonal blocks of W^R = X^R V (Table "quantities": W = (I-VP)^{-1} V).

    (X^R V)_ii = X_{i,i-1} V_{i-1,i} + X_ii V_ii + X_{i,i+1} V_{i+1,i};
    only the diagonal is exact from the selected blocks of X^R.
    """
    Xd, Xu, Xl = XR
    Vd, Vu, Vl = V
    n = Xd.shape[0]
    out = np.empty_like(Xd)
    for i in range(n):
        acc = Xd[i] @ Vd[i]
        if i > 0:
            acc = acc + Xl[i - 1] @ Vu[i - 1]
        if i < n - 1:
            acc = acc + Xu[i] @ Vl[i]
        out[i] = acc
    return out
