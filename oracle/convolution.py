"""Energy convolution of two energy-resolved quantities (Sec. "Energy
Convolutions", Eq. interaction).

TEST INFRASTRUCTURE ONLY (see the package header).

The scattering term of Eq. (B) is the energy convolution of two particle
descriptors, entry by entry of the selected blocks:
B_scatt(E) is proportional to the integral over E' of X1(E - E') X2(E'),
with X1, X2 taken as G or W and the products element-wise (Sec. "Energy
Convolutions").  The paper gives neither the prefactor nor the grids, so the
operation is stated on uniform energy grids of one spacing dE, with the
prefactor (the sign, i / 2 pi, dE) folded into one complex scale s:

    B[k][i] = s * sum_{k'=0}^{n2-1} X1'[k + shift - k'][i] * X2[k'][i]

for 0 <= k < n_out, where X1' = X1, or X1 with its energy order reversed
(X1'[j] = X1[n1 - 1 - j]), terms whose X1' index lies outside [0, n1) are
left out, and `shift` places the difference grid of X1 against the output
grid (X1'[j] samples energy difference (j - shift) dE when X2[k'] and B[k]
sample the same grid).  Reversing X1 gives the correlation
sum_{k'} X1[k' - k + ...] X2[k'] that the polarization's form
G(E') G(E' - E) takes.  Data are energy-major, [energy][element], which is
the layout of the solver's outputs ([energy][block][b][b]).

Written as the definition: one explicit loop over k and k', each term added
in the order of k' (the element index is vectorised).
"""

import numpy as np


def energy_convolution(X1, X2, n_out, shift=0, scale=1.0, reverse1=False):
    """X1: [n1, ...], X2: [n2, ...] complex arrays on uniform energy grids
    (energy first, any element shape after it).  Returns B: [n_out, ...]."""
    X1 = np.asarray(X1, dtype=np.complex128)
    X2 = np.asarray(X2, dtype=np.complex128)
    n1, n2 = X1.shape[0], X2.shape[0]
    if X1.shape[1:] != X2.shape[1:]:
        raise ValueError("element shapes differ")
    X1p = X1[::-1] if reverse1 else X1
    B = np.zeros((n_out,) + X1.shape[1:], dtype=np.complex128)
    for k in range(n_out):
        acc = np.zeros(X1.shape[1:], dtype=np.complex128)
        for kp in range(n2):
            j = k + shift - kp
            if 0 <= j < n1:
                acc = acc + X1p[j] * X2[kp]
        B[k] = scale * acc
    return B
