"""Seeded synthetic inputs for block-tridiagonal RGF solves.

This module only draws and lays out input data; it holds none of the
solver's arithmetic.  Both the HIP path (through its callers) and the CPU
oracle consume exactly the arrays produced here.

Conventions
-----------
* Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
* "complex N(0, s2)" is circular: real and imaginary parts are independent
  N(0, s2/2), so E|z|^2 = s2.
* Draw order for a Hermitian block-tridiagonal matrix: all n diagonal
  generators X (real parts of the whole stack, then imaginary parts), then
  all n-1 upper blocks (same order).  H_ii = (X + X^dagger)/2,
  H_{i+1,i} = H_{i,i+1}^dagger.
* Blocks are row-major b x b complex128; a block-tridiagonal operand is a
  (diag[n,b,b], upper[n-1,b,b], lower[n-1,b,b]) triple, with
  upper[i] = block (i, i+1) and lower[i] = block (i+1, i).
* Energies: a uniform grid including both ends, linspace(-2, 2, N_E).
* Occupations: Fermi f(E) = 1/(1+exp((E-mu)/kT)); 1-f is evaluated directly as
  1/(1+exp(-(E-mu)/kT)) so that it never rounds to an exact zero.
* Self-energies of the G-type workloads (electrons):
    Sigma^R_ii = -i*eta*I on every block, plus -i*eta_obc*I on blocks 0 and n-1
    (the two contact blocks of the open boundary), Gamma = i(Sigma^R - Sigma^A),
    Sigma^< = i f Gamma,  Sigma^> = -i (1-f) Gamma.
  All of these are multiples of the identity; they are described by one
  complex scalar per (energy, block) and expanded to full blocks on request.
"""

import numpy as np


# ----------------------------------------------------------------- basics --

def cn(rng, shape, var):
    """Circular complex normal with E|z|^2 = var."""
    s = np.sqrt(var / 2.0)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * s


def hermitian_bt(rng, n, b, diag_var=1.0, off_var=0.25, scale=1.0):
    """Random Hermitian block-tridiagonal matrix (diag, upper, lower).

    H_ii = (X + X^dagger)/2 with X ~ CN(0, diag_var/b);
    H_{i,i+1} ~ CN(0, off_var/b); H_{i+1,i} = H_{i,i+1}^dagger.
    """
    X = cn(rng, (n, b, b), diag_var / b)
    d = 0.5 * (X + np.conj(np.swapaxes(X, 1, 2)))
    u = cn(rng, (max(n - 1, 0), b, b), off_var / b)
    l = np.conj(np.swapaxes(u, 1, 2)).copy()
    if scale != 1.0:
        d, u, l = d * scale, u * scale, l * scale
    return d, u, l


def energy_grid(n_e, lo=-2.0, hi=2.0):
    return np.linspace(lo, hi, n_e)


def fermi(E, mu=0.0, kT=0.025):
    return 1.0 / (1.0 + np.exp((np.asarray(E) - mu) / kT))


def one_minus_fermi(E, mu=0.0, kT=0.025):
    return 1.0 / (1.0 + np.exp(-(np.asarray(E) - mu) / kT))


def eye_blocks(scalars, b):
    """Expand an array of complex scalars [..., n] to [..., n, b, b] = s * I."""
    scalars = np.asarray(scalars, dtype=np.complex128)
    out = np.zeros(scalars.shape + (b, b), dtype=np.complex128)
    idx = np.arange(b)
    out[..., idx, idx] = scalars[..., None]
    return out


# ------------------------------------------------------- G-type workloads --

def g_sigma_scalars(energies, n, eta=0.01, eta_obc=0.1, mu=0.0, kT=0.025):
    """Per-(energy, block) scalars of Sigma^R, Sigma^<, Sigma^> (times I)."""
    E = np.asarray(energies, dtype=np.float64)
    gam = np.full(n, 2.0 * eta)
    gam[0] += 2.0 * eta_obc
    gam[-1] += 2.0 * eta_obc
    sr = np.broadcast_to(-0.5j * gam, (E.shape[0], n)).astype(np.complex128)
    f = fermi(E, mu, kT)
    fb = one_minus_fermi(E, mu, kT)
    sl = 1j * f[:, None] * gam[None, :]
    sg = -1j * fb[:, None] * gam[None, :]
    return sr.copy(), sl.astype(np.complex128), sg.astype(np.complex128)


def g_problem(seed, n, b, n_e=None, energies=None, eta=0.01, eta_obc=0.1,
              mu=0.0, kT=0.025, bt_sigma=False, expand=True):
    """Electron (G-type) workload.

    Returns a dict with H (BT triple), energies [N_E], and the self-energies
    either expanded (sigma_r/l/g diag [N_E,n,b,b], plus upper [N_E,n-1,b,b]
    when ``bt_sigma``) or as scalars (``expand=False``; block-diagonal only).

    ``bt_sigma`` adds an energy-independent Hermitian BT part K (drawn after
    H, CN variance 0.005/b per entry) to Gamma: Gamma -> Gamma + K, so that
    Sigma^< = i f Gamma, Sigma^> = -i (1-f) Gamma and Sigma^R = -i Gamma/2
    all have off-diagonal blocks while Sigma^> - Sigma^< = Sigma^R - Sigma^A
    still holds.
    """
    rng = np.random.default_rng(seed)
    H = hermitian_bt(rng, n, b, 1.0, 0.25)
    if energies is None:
        energies = energy_grid(n_e)
    energies = np.asarray(energies, dtype=np.float64)
    sr, sl, sg = g_sigma_scalars(energies, n, eta, eta_obc, mu, kT)
    out = {"kind": "G", "n": n, "b": b, "energies": energies, "H": H,
           "seed": seed}
    if not expand:
        assert not bt_sigma
        out["sigma_scalars"] = (sr, sl, sg)
        return out
    Rd, Ld, Gd = eye_blocks(sr, b), eye_blocks(sl, b), eye_blocks(sg, b)
    if bt_sigma:
        Kd, Ku, Kl = hermitian_bt(rng, n, b, 0.005, 0.005)
        f = fermi(energies, mu, kT)[:, None, None, None]
        fb = one_minus_fermi(energies, mu, kT)[:, None, None, None]
        Rd = Rd + (-0.5j) * Kd[None]
        Ld = Ld + 1j * f * Kd[None]
        Gd = Gd - 1j * fb * Kd[None]
        Ru = np.broadcast_to(-0.5j * Ku[None], (len(energies),) + Ku.shape).copy()
        Rl = np.broadcast_to(-0.5j * Kl[None], (len(energies),) + Kl.shape).copy()
        Lu = 1j * f * Ku[None]
        Ll = 1j * f * Kl[None]
        Gu = -1j * fb * Ku[None]
        Gl = -1j * fb * Kl[None]
        out["sigma_r"] = (Rd, Ru, Rl)
        out["sigma_l"] = (Ld, Lu, Ll)
        out["sigma_g"] = (Gd, Gu, Gl)
    else:
        z = np.zeros((len(energies), max(n - 1, 0), b, b), np.complex128)
        out["sigma_r"] = (Rd, None, None)
        out["sigma_l"] = (Ld, z, z.copy())
        out["sigma_g"] = (Gd, z.copy(), z.copy())
    return out


# ------------------------------------------------------- W-type workloads --

def w_problem(seed, n, b, energies, mu=0.0, kT=0.025):
    """Screened-Coulomb (W-type) workload.

    V = 0.5 G_V and P_h = 0.5 G_P with G_V, G_P drawn by ``hermitian_bt``
    (V first);  P^R(E) = 0.5 (P_h + 0.1 E I) - 0.01 i I  (block-tridiagonal);
    Gamma_P = i(P^R - P^A) = 0.02 I;  P^< = i f Gamma_P,  P^> = -i (1-f) Gamma_P
    (diagonal blocks only).
    Returns a dict with V (BT triple) and P_r, P_l, P_g (BT triples with a
    leading energy axis).
    """
    rng = np.random.default_rng(seed)
    V = hermitian_bt(rng, n, b, 1.0, 0.25, scale=0.5)
    Ph = hermitian_bt(rng, n, b, 1.0, 0.25, scale=0.5)
    E = np.asarray(energies, dtype=np.float64)
    ne = E.shape[0]
    eye = np.eye(b, dtype=np.complex128)
    Prd = 0.5 * (Ph[0][None] + 0.1 * E[:, None, None, None] * eye) - 0.01j * eye
    Pru = np.broadcast_to(0.5 * Ph[1][None], (ne,) + Ph[1].shape).copy()
    Prl = np.broadcast_to(0.5 * Ph[2][None], (ne,) + Ph[2].shape).copy()
    gam = 0.02
    f = fermi(E, mu, kT)
    fb = one_minus_fermi(E, mu, kT)
    Pld = eye_blocks(np.broadcast_to((1j * f * gam)[:, None], (ne, n)), b)
    Pgd = eye_blocks(np.broadcast_to((-1j * fb * gam)[:, None], (ne, n)), b)
    z = np.zeros((ne, max(n - 1, 0), b, b), np.complex128)
    return {"kind": "W", "n": n, "b": b, "energies": E, "V": V,
            "P_r": (Prd, Pru, Prl), "P_l": (Pld, z, z.copy()),
            "P_g": (Pgd, z.copy(), z.copy()), "seed": seed}


# ---------------------------------------------------- general test inputs --

def random_bt(rng, n, b, diag_shift=0.0, scale=1.0):
    """General (non-symmetric) complex BT triple, entries CN(0, scale^2/b);
    ``diag_shift`` is added to every diagonal element of the diagonal blocks."""
    d = cn(rng, (n, b, b), scale ** 2 / b)
    d = d + diag_shift * np.eye(b)[None]
    u = cn(rng, (max(n - 1, 0), b, b), scale ** 2 / b)
    l = cn(rng, (max(n - 1, 0), b, b), scale ** 2 / b)
    return d, u, l


def random_antihermitian_bt(rng, n, b, scale=1.0):
    """Random anti-Hermitian BT triple: B = i K with K Hermitian BT."""
    d, u, l = hermitian_bt(rng, n, b, scale ** 2, scale ** 2)
    return 1j * d, 1j * u, 1j * l


# ------------------------------------------------ batched uneven workload --

UNEVEN_BLOCK_SIZES = (64, 128, 256, 384, 512, 768)


def uneven_specs(seed, count=512, block_sizes=UNEVEN_BLOCK_SIZES,
                 n_range=(8, 128)):
    """Descriptors of independent single-energy solves of mixed shape.

    Half are G-type, half W-type, shuffled; b uniform over ``block_sizes``,
    n uniform over n_range (inclusive), E uniform in [-2, 2].  Each entry
    carries its own seed for the input draw.
    """
    rng = np.random.default_rng(seed)
    kinds = np.array(["G"] * (count // 2) + ["W"] * (count - count // 2))
    rng.shuffle(kinds)
    bs = rng.choice(np.asarray(block_sizes), size=count)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    es = rng.uniform(-2.0, 2.0, size=count)
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    return [{"kind": str(k), "b": int(b), "n": int(n), "E": float(e),
             "seed": int(s)} for k, b, n, e, s in zip(kinds, bs, ns, es, seeds)]


def lead_blocks(seed, b, energies, eta=0.05):
    """Contact blocks of a semi-infinite lead, one set per energy.

    The lead repeats one layer: on-site H00 = (X + X^dagger)/2, X complex
    N(0, 1/b), and coupling H01 complex N(0, 0.25/b) to the next layer (same
    draw order as a Hermitian block-tridiagonal matrix with n = 1 plus one
    upper block).  With S = I and a retarded broadening eta:
        m(E) = (E + i eta) I - H00,   n = -H01,   n' = -H01^dagger.
    Returns m [N_E, b, b], n [b, b], n' [b, b] (n, n' shared by all energies).
    """
    rng = np.random.default_rng(seed)
    X = cn(rng, (b, b), 1.0 / b)
    h00 = 0.5 * (X + X.conj().T)
    h01 = cn(rng, (b, b), 0.25 / b)
    E = np.asarray(energies, dtype=np.float64)
    eye = np.eye(b, dtype=np.complex128)
    m = (E[:, None, None] + 1j * eta) * eye[None] - h00[None]
    return np.ascontiguousarray(m), np.ascontiguousarray(-h01), \
        np.ascontiguousarray(-h01.conj().T)


def lyapunov_blocks(seed, b, n_e, rho=0.8):
    """Operands of w = q - a w a^dagger for n_e energies: a complex
    N(0, rho^2/b) (spectral radius about rho by the circular law), q
    anti-Hermitian, (Y - Y^dagger)/2 with Y complex N(0, 1/b), as a lesser or
    greater quantity is.  Draw order: all a, then all Y."""
    rng = np.random.default_rng(seed)
    a = cn(rng, (n_e, b, b), rho * rho / b)
    Y = cn(rng, (n_e, b, b), 1.0 / b)
    q = 0.5 * (Y - np.conj(np.swapaxes(Y, 1, 2)))
    return np.ascontiguousarray(a), np.ascontiguousarray(q)
