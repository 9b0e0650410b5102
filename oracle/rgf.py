"""RGF selected inversion, written out in the paper's order and notation.

Paper: arXiv 2508.19138, Sec. 3.2.3 "Recursive Green's Function (RGF)
Solver", Eq. (forward-pass) and Eq. (backward-pass), applied to the system of
Eq. (system-solve):  Mt X^R = I  and  Mt X^s Mt^dagger = B^s,  s in {<, >}.

Block notation (0-based here, 1-based in the paper):
  Mt_ii        diagonal block i                        ``Mt[0][i]``
  Mt_{i,i+1}   upper block (row i, column i+1)          ``Mt[1][i]``
  Mt_{i+1,i}   lower block (row i+1, column i)          ``Mt[2][i]``
The same (diag, upper, lower) triple is used for every right-hand side B^s.

Readings of the paper used here (each was confirmed against the dense
definition in ``oracle.dense`` by the tests):
  * In the forward lesser/greater step the cross term is
    y_i = Mt_{i,i-1} x^R_{i-1} B^s_{i-1,i}; as printed it carries x^s_{i-1},
    which is not linear in B and does not reproduce A^{-1} B A^{-dagger}.
  * Mt^dagger_{j,k} denotes the (j,k) block of the adjoint matrix, i.e.
    (Mt_{k,j})^dagger.
  * The paper writes the lesser/greater terms with y - y^dagger, Y - Y^dagger
    and Z - Z^dagger, which assumes anti-Hermitian B^s.  This oracle writes
    each of those terms out separately (general B^s), so the anti-Hermitian
    symmetry of the output is a property the tests check, not an input.
  * The first off-diagonal blocks of X (which the paper says RGF also
    provides, without printing them) follow from the same block elimination:
      X_{i,i+1}   = -x_i Mt_{i,i+1} X_{i+1}
      X_{i+1,i}   = -X_{i+1} Mt_{i+1,i} x_i
      X^s_{i,i+1} = -x_i Mt_{i,i+1} X^s_{i+1} - x^s_i (X_{i+1} Mt_{i+1,i})^dagger
                    + x_i B^s_{i,i+1} X_{i+1}^dagger
      X^s_{i+1,i} = -X_{i+1} Mt_{i+1,i} x^s_i + X_{i+1} B^s_{i+1,i} x_i^dagger
                    - X^s_{i+1} (x_i Mt_{i,i+1})^dagger
"""

import numpy as np


def _inv(a):
    """Plain inverse of one complex block (LAPACK getrf/getri via NumPy)."""
    return np.linalg.inv(a)


def _h(a):
    """Adjoint (conjugate transpose) of one block."""
    return a.conj().T


def rgf_selected(Mt, Bs=()):
    """Selected blocks of X^R = Mt^{-1} and X^s = Mt^{-1} B^s Mt^{-dagger}.

    Mt : (diag[n,b,b], upper[n-1,b,b], lower[n-1,b,b]) complex128
    Bs : sequence of (diag, upper, lower) triples, one per right-hand side
    Returns (XR, [XS ...]) where each result is a (diag, upper, lower) triple
    of the diagonal and first off-diagonal blocks.
    """
    Md, Mu, Ml = (np.asarray(t, dtype=np.complex128) for t in Mt)
    n = Md.shape[0]
    Bs = [tuple(np.asarray(t, dtype=np.complex128) for t in B) for B in Bs]

    # ---- forward pass (Eq. forward-pass): left-connected x^R_i, x^s_i ----
    xR = [None] * n
    xS = [[None] * n for _ in Bs]
    xR[0] = _inv(Md[0])                                   # x^R_1 = Mt_11^{-1}
    for s, (Bd, Bu, Bl) in enumerate(Bs):
        xS[s][0] = xR[0] @ Bd[0] @ _h(xR[0])              # x^s_1 = x^R_1 B_11 x^R_1^dag
    for i in range(1, n):
        Mil = Ml[i - 1]                                   # Mt_{i,i-1}
        Mli = Mu[i - 1]                                   # Mt_{i-1,i}
        xR[i] = _inv(Md[i] - Mil @ xR[i - 1] @ Mli)
        for s, (Bd, Bu, Bl) in enumerate(Bs):
            y = Mil @ xR[i - 1] @ Bu[i - 1]               # y_i (x^R, see header)
            y_adj_general = Bl[i - 1] @ _h(xR[i - 1]) @ _h(Mil)
            inner = (Bd[i]
                     + Mil @ xS[s][i - 1] @ _h(Mil)        # Mt_{i,i-1} x^s Mt^dag_{i-1,i}
                     - y - y_adj_general)
            xS[s][i] = xR[i] @ inner @ _h(xR[i])

    # ---- backward pass (Eq. backward-pass): full X^R_i, X^s_i -----------
    XRd = np.empty_like(Md)
    XRu = np.empty_like(Mu)
    XRl = np.empty_like(Ml)
    XSd = [np.empty_like(Md) for _ in Bs]
    XSu = [np.empty_like(Mu) for _ in Bs]
    XSl = [np.empty_like(Ml) for _ in Bs]
    XRd[n - 1] = xR[n - 1]
    for s in range(len(Bs)):
        XSd[s][n - 1] = xS[s][n - 1]
    for i in range(n - 2, -1, -1):
        Mup = Mu[i]                                       # Mt_{i,i+1}
        Mlo = Ml[i]                                       # Mt_{i+1,i}
        Xn = XRd[i + 1]                                   # X^R_{i+1}
        # X^R_i = x_i + x_i Mt_{i,i+1} X_{i+1} Mt_{i+1,i} x_i
        XRd[i] = xR[i] + xR[i] @ Mup @ Xn @ Mlo @ xR[i]
        XRu[i] = -xR[i] @ Mup @ Xn
        XRl[i] = -Xn @ Mlo @ xR[i]
        for s, (Bd, Bu, Bl) in enumerate(Bs):
            XSn = XSd[s][i + 1]
            # Y_i = x_i B_{i,i+1} (x_i Mt_{i,i+1} X_{i+1})^dag, and its general
            # counterpart for a B that is not anti-Hermitian.
            Y = xR[i] @ Bu[i] @ _h(xR[i] @ Mup @ Xn)
            Y_general_adj = (xR[i] @ Mup @ Xn) @ Bl[i] @ _h(xR[i])
            # Z_i = x_i Mt_{i,i+1} X_{i+1} Mt_{i+1,i} x^s_i
            Z = xR[i] @ Mup @ Xn @ Mlo @ xS[s][i]
            Z_general_adj = xS[s][i] @ _h(xR[i] @ Mup @ Xn @ Mlo)
            XSd[s][i] = (xS[s][i]
                         + xR[i] @ Mup @ XSn @ _h(Mup) @ _h(xR[i])
                         - Y - Y_general_adj
                         + Z + Z_general_adj)
            XSu[s][i] = (-xR[i] @ Mup @ XSn
                         - xS[s][i] @ _h(Xn @ Mlo)
                         + xR[i] @ Bu[i] @ _h(Xn))
            XSl[s][i] = (-Xn @ Mlo @ xS[s][i]
                         + Xn @ Bl[i] @ _h(xR[i])
                         - XSn @ _h(xR[i] @ Mup))
    XR = (XRd, XRu, XRl)
    XS = [(XSd[s], XSu[s], XSl[s]) for s in range(len(Bs))]
    return XR, XS
