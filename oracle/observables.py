"""Observables from the selected blocks (Sec. "Observables").

TEST INFRASTRUCTURE ONLY (see the package header).

The paper names the local density of states, the charge density and the
current as functions of the diagonal and first off-diagonal blocks of the
lesser and greater Green's functions, without printing formulas.  The
standard energy-resolved forms (units e = hbar = 1, one spin, per unit
energy) are used, for block i at one energy:

    dos_i     = Tr(A_ii) / (2 pi),          A_ii = i (G^>_ii - G^<_ii)
    density_i = Tr(-i G^<_ii) / (2 pi)
    current_i = 2 Re Tr(H_{i,i+1} G^<_{i+1,i}) / (2 pi)   (interface i|i+1,
                                                            positive from i to i+1)

H_{i,i+1} is the Hamiltonian coupling (S = I off the diagonal).  Integrating
over energy is left to the caller.
"""

import numpy as np

_INV_2PI = 1.0 / (2.0 * np.pi)


def observables(GL, GG, H_upper):
    """GL, GG: (diag[n,b,b], upper[n-1,b,b], lower[n-1,b,b]) of G^<, G^> at one
    energy; H_upper: [n-1, b, b].  Returns (dos[n], density[n], current[n-1])."""
    gl_d, _, gl_l = (np.asarray(t) for t in GL)
    gg_d = np.asarray(GG[0])
    n = gl_d.shape[0]
    dos = np.array([np.real(np.trace(1j * (gg_d[i] - gl_d[i]))) for i in range(n)]) * _INV_2PI
    dens = np.array([np.real(np.trace(-1j * gl_d[i])) for i in range(n)]) * _INV_2PI
    cur = np.array([2.0 * np.real(np.trace(H_upper[i] @ gl_l[i])) for i in range(n - 1)]) \
        * _INV_2PI
    return dos, dens, cur
