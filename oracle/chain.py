"""Closed-form Green's function of a uniform 1-D tight-binding chain.

Independent pin for the RGF oracle (not derived from the recursion).  The
device is n identical transport cells with on-site block h0 (Hermitian,
b x b) and nearest-neighbour coupling t*I, S = I.  Exact semi-infinite
leads of the same chain are attached to blocks 0 and n-1 as retarded
open-boundary self-energies (the B^R_OBC blocks of Sec. 3.1 "Open Boundary
Conditions"), so the finite device reproduces the infinite chain.

In the eigenbasis h0 = U diag(eps_k) U^dagger the chain splits into b
scalar chains.  For each, the surface recursion of Eq. (retarded-recursion)
has the exact solution Sigma_k = t lambda_k with
    lambda_k + 1/lambda_k = (E - eps_k) / t,
choosing |lambda_k| < 1 outside the band and Im(Sigma_k) < 0 (retarded)
inside it.  The infinite-chain Green's function is
    G_{jl} = lambda^{|j-l|} / (t (1/lambda - lambda)).
Lesser function with lead injection only (Sigma^<_L/R = i f_{L/R} Gamma,
fluctuation-dissipation form of Sec. 3.1.2):
    G^<_{jl} = G_{j0} Sigma^<_L G_{l0}^dagger + G_{j,n-1} Sigma^<_R G_{l,n-1}^dagger.
"""

import numpy as np


def _lambda(E, eps, t):
    z = (E - eps) / t
    root = np.sqrt(z.astype(np.complex128) ** 2 - 4.0)
    l1 = (z + root) / 2.0
    l2 = (z - root) / 2.0
    in_band = np.abs(z) < 2.0
    # retarded choice inside the band: Im(t * lambda) < 0
    pick_in = np.where(np.imag(t * l1) < 0, l1, l2)
    pick_out = np.where(np.abs(l1) < 1.0, l1, l2)
    return np.where(in_band, pick_in, pick_out)


def chain_lead_self_energy(E, h0, t):
    """Retarded lead self-energy block U diag(t lambda_k) U^dagger."""
    eps, U = np.linalg.eigh(h0)
    lam = _lambda(E, eps, t)
    return (U * (t * lam)) @ U.conj().T


def chain_closed_form(E, h0, t, n, f_left=None, f_right=None):
    """Selected blocks of G^R (and of G^< if both occupations are given).

    Returns (diag[n], upper[n-1], lower[n-1]) for G^R, and, when f_left and
    f_right are given, the same triple for G^<.
    """
    eps, U = np.linalg.eigh(h0)
    lam = _lambda(E, eps, t)
    g00 = 1.0 / (t * (1.0 / lam - lam))

    def g(j, l):                     # eigenbasis diagonal of G_{jl}
        return lam ** abs(j - l) * g00

    def to_block(v):
        return (U * v) @ U.conj().T

    b = h0.shape[0]
    d = np.stack([to_block(g(i, i)) for i in range(n)])
    u = np.stack([to_block(g(i, i + 1)) for i in range(n - 1)]) if n > 1 \
        else np.zeros((0, b, b), np.complex128)
    l = np.stack([to_block(g(i + 1, i)) for i in range(n - 1)]) if n > 1 \
        else np.zeros((0, b, b), np.complex128)
    if f_left is None:
        return (d, u, l)
    sig = t * lam
    gamma = -2.0 * np.imag(sig)              # i (Sigma - Sigma^dagger)
    sl = 1j * f_left * gamma
    sr = 1j * f_right * gamma

    def gl(j, k):
        return (g(j, 0) * sl * np.conj(g(k, 0))
                + g(j, n - 1) * sr * np.conj(g(k, n - 1)))

    ld = np.stack([to_block(gl(i, i)) for i in range(n)])
    lu = np.stack([to_block(gl(i, i + 1)) for i in range(n - 1)]) if n > 1 \
        else np.zeros((0, b, b), np.complex128)
    ll = np.stack([to_block(gl(i + 1, i)) for i in range(n - 1)]) if n > 1 \
        else np.zeros((0, b, b), np.complex128)
    return (d, u, l), (ld, lu, ll)
