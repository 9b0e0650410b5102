"""Pins of the lead surface-function oracle (Sec. "Retarded OBC").

The oracle's two solvers of Eq. (retarded-recursion) are checked against
results fixed independently of either iteration:

* the uniform chain with coupling t*I: in the eigenbasis of the on-site
  block the lead splits into scalar chains whose surface function is
  lambda_k / t, lambda_k the root of lambda + 1/lambda = (z - eps_k)/t with
  |lambda_k| < 1 (z = E + i eta); at real E outside the band the boundary
  block t^2 x must equal the chain module's lead self-energy;
* brute force: the surface block of the dense inverse of a long finite
  lead (L identical layers), which differs from x by O(|lambda|^(2L));
* the defining equation itself, retardation (Im x <= 0 for a Hermitian
  lead) and the fixed point's invariance when started at the solution.
"""

import numpy as np
import pytest

from oracle import chain_lead_self_energy, obc_fixed_point, obc_sancho_rubio
from paper_2508_19138_amd import synth


def _chain_surface(z, h0, t):
    """U diag(lambda_k / t) U^dagger with |lambda_k| < 1 (decaying root)."""
    eps, U = np.linalg.eigh(h0)
    w = (z - eps) / t
    r = np.sqrt(w.astype(np.complex128) ** 2 - 4.0)
    l1, l2 = (w + r) / 2.0, (w - r) / 2.0
    lam = np.where(np.abs(l1) < 1.0, l1, l2)
    return (U * (lam / t)) @ U.conj().T


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _finite_lead_surface(m, n, np_, L):
    """Block (0, 0) of the inverse of the L-layer lead (dense, brute force)."""
    b = m.shape[0]
    A = np.zeros((L * b, L * b), np.complex128)
    for j in range(L):
        A[j * b:(j + 1) * b, j * b:(j + 1) * b] = m
        if j + 1 < L:
            A[j * b:(j + 1) * b, (j + 1) * b:(j + 2) * b] = n
            A[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = np_
    return np.linalg.inv(A)[:b, :b]


@pytest.mark.parametrize("b,t,E,eta", [(1, 1.0, 0.3, 0.05), (4, 0.7, -0.5, 0.1),
                                       (6, 1.3, 1.1, 0.02)])
def test_chain_surface_function_closed_form(b, t, E, eta):
    rng = np.random.default_rng(7 + b)
    X = synth.cn(rng, (b, b), 1.0 / b)
    h0 = 0.5 * (X + X.conj().T)
    z = E + 1j * eta
    m = z * np.eye(b) - h0
    n = -t * np.eye(b, dtype=np.complex128)
    exact = _chain_surface(z, h0, t)
    xs, sig, steps = obc_sancho_rubio(m, n, n)
    assert _rel(xs, exact) < 1e-12, steps
    assert _rel(sig, t * t * exact) < 1e-12
    # Eq. (naive) contracts by about |lambda|^2 per iteration
    xf, sigf, upd = obc_fixed_point(m, n, n, np.zeros((b, b), np.complex128), 4000)
    assert _rel(xf, exact) < 1e-10
    assert upd < 1e-12


@pytest.mark.parametrize("E", [-3.1, 2.7])
def test_boundary_block_matches_chain_self_energy_outside_band(E):
    b, t = 5, 1.0
    rng = np.random.default_rng(11)
    X = synth.cn(rng, (b, b), 0.2 / b)
    h0 = 0.5 * (X + X.conj().T)
    m = E * np.eye(b) - h0
    n = -t * np.eye(b, dtype=np.complex128)
    _, sig, _ = obc_sancho_rubio(m, n, n)
    assert _rel(sig, chain_lead_self_energy(E, h0, t)) < 1e-12


@pytest.mark.parametrize("b,E,eta", [(3, 0.2, 0.3), (8, -0.7, 0.25)])
def test_general_lead_matches_dense_finite_lead(b, E, eta):
    m, n, np_ = synth.lead_blocks(5 + b, b, [E], eta=eta)
    m = m[0]
    xs, _, _ = obc_sancho_rubio(m, n, np_)
    x_dense = _finite_lead_surface(m, n, np_, 120)
    assert _rel(xs, x_dense) < 1e-11
    xf, _, _ = obc_fixed_point(m, n, np_, np.zeros((b, b), np.complex128), 400)
    assert _rel(xf, x_dense) < 1e-11


def test_non_hermitian_couplings_solve_the_defining_equation():
    rng = np.random.default_rng(3)
    b = 6
    m = (0.4 + 0.3j) * np.eye(b) + synth.cn(rng, (b, b), 0.1 / b)
    n = synth.cn(rng, (b, b), 0.2 / b)
    np_ = synth.cn(rng, (b, b), 0.2 / b)          # not n^dagger
    xs, sig, _ = obc_sancho_rubio(m, n, np_)
    assert _rel(xs, np.linalg.inv(m - n @ xs @ np_)) < 1e-13
    assert _rel(sig, n @ xs @ np_) < 1e-15
    xf, _, _ = obc_fixed_point(m, n, np_, np.zeros((b, b), np.complex128), 200)
    assert _rel(xf, xs) < 1e-12


def test_retarded_surface_function_has_nonpositive_imaginary_part():
    m, n, np_ = synth.lead_blocks(21, 10, [-0.4, 0.0, 0.9], eta=0.05)
    for e in range(3):
        xs, _, _ = obc_sancho_rubio(m[e], n, np_)
        im = (xs - xs.conj().T) / 2j
        assert np.linalg.eigvalsh(im).max() < 1e-12


def test_memoized_start_is_a_fixed_point():
    m, n, np_ = synth.lead_blocks(4, 12, [0.5], eta=0.05)
    xs, sig_s, _ = obc_sancho_rubio(m[0], n, np_)
    x3, sig3, upd = obc_fixed_point(m[0], n, np_, xs, 3)
    assert _rel(x3, xs) < 1e-12
    assert _rel(sig3, sig_s) < 1e-12
    assert upd < 1e-12


def test_fixed_point_first_iteration_and_update_definition():
    m, n, np_ = synth.lead_blocks(9, 4, [0.1], eta=0.2)
    x0 = np.zeros((4, 4), np.complex128)
    x1, sig1, upd1 = obc_fixed_point(m[0], n, np_, x0, 1)
    assert np.allclose(x1, np.linalg.inv(m[0]), rtol=0, atol=1e-15)
    assert upd1 == pytest.approx(1.0, abs=1e-15)        # ||x1 - 0|| / ||x1||
    x2, _, upd2 = obc_fixed_point(m[0], n, np_, x0, 2)
    assert upd2 == pytest.approx(np.linalg.norm(x2 - x1) / np.linalg.norm(x2), rel=1e-12)
    with pytest.raises(ValueError):
        obc_fixed_point(m[0], n, np_, x0, 0)


def test_fixed_step_decimation_agrees_with_converged_run():
    from oracle import obc_sancho_rubio_steps
    m, n, np_ = synth.lead_blocks(14, 10, [0.3], eta=0.05)
    xs, sig_s, k = obc_sancho_rubio(m[0], n, np_)
    x, sig, rest = obc_sancho_rubio_steps(m[0], n, np_, k + 3)
    assert _rel(x, xs) < 1e-13 and _rel(sig, sig_s) < 1e-13 and rest < 1e-15
    # one step: m_surf = m - n m^-1 n'
    x1, _, rest1 = obc_sancho_rubio_steps(m[0], n, np_, 1)
    g = np.linalg.inv(m[0])
    assert _rel(x1, np.linalg.inv(m[0] - n @ g @ np_)) < 1e-13
    a1, c1 = -(n @ g @ n), -(np_ @ g @ np_)
    assert rest1 == pytest.approx((np.linalg.norm(a1) + np.linalg.norm(c1))
                                  / (np.linalg.norm(n) + np.linalg.norm(np_)), rel=1e-12)
    with pytest.raises(ValueError):
        obc_sancho_rubio_steps(m[0], n, np_, 0)


# ------------------------------------------------- lesser/greater boundary blocks

def _chain_setup(b=5, t=1.0, seed=19):
    rng = np.random.default_rng(seed)
    X = synth.cn(rng, (b, b), 1.0 / b)
    return 0.5 * (X + X.conj().T), t


@pytest.mark.parametrize("E", [-0.9, 0.35])
def test_lesser_greater_in_the_chain_eigenbasis(E):
    """Each scalar channel k of the uniform chain has broadening
    -2 Im(t lambda_k); the matrix form must agree with it channel by channel."""
    from oracle import obc_lesser_greater
    h0, t = _chain_setup()
    sig = chain_lead_self_energy(E, h0, t)
    f = float(synth.fermi(np.array([E]))[0])
    omf = float(synth.one_minus_fermi(np.array([E]))[0])
    sl, sg = obc_lesser_greater(sig, f, omf)
    eps, U = np.linalg.eigh(h0)
    d = np.diag(U.conj().T @ sig @ U)
    gam = -2.0 * np.imag(d)
    assert _rel(sl, (U * (1j * f * gam)) @ U.conj().T) < 1e-13
    assert _rel(sg, (U * (-1j * omf * gam)) @ U.conj().T) < 1e-13
    assert _rel(sg - sl, sig - sig.conj().T) < 1e-13
    assert _rel(sl, -sl.conj().T) < 1e-15 and _rel(sg, -sg.conj().T) < 1e-15


def test_equilibrium_device_with_lesser_boundary_blocks():
    """A chain device closed by its exact leads, both at occupation f: the
    lesser function from the (pinned) recursion equals the closed form and
    the equilibrium relation G^< = -f (G^R - G^A)."""
    from oracle import obc_lesser_greater, rgf_selected, chain_closed_form
    h0, t = _chain_setup(b=4, seed=23)
    n, E = 6, 0.2
    b = h0.shape[0]
    sig = chain_lead_self_energy(E, h0, t)
    f = float(synth.fermi(np.array([E]))[0])
    omf = float(synth.one_minus_fermi(np.array([E]))[0])
    sl, sg = obc_lesser_greater(sig, f, omf)
    I = np.eye(b)
    d = np.stack([E * I - h0] * n)
    d[0] -= sig
    d[-1] -= sig
    u = np.stack([-t * I] * (n - 1)).astype(np.complex128)
    A = (d.astype(np.complex128), u, u.copy())
    z = np.zeros((n - 1, b, b), np.complex128)
    bl = np.zeros((n, b, b), np.complex128)
    bl[0] = sl
    bl[-1] = sl
    XR, XS = rgf_selected(A, [(bl, z, z)])
    XL = XS[0]
    (CR, CL) = chain_closed_form(E, h0, t, n, f, f)
    for k in range(3):
        assert _rel(XR[k], CR[k]) < 1e-12
        assert _rel(XL[k], CL[k]) < 1e-12
    gl_eq = -f * (XR[0] - np.conj(np.swapaxes(XR[0], 1, 2)))
    assert _rel(XL[0], gl_eq) < 1e-12


# ------------------------------------------------ Lyapunov (W lesser/greater)

def _lyap_direct(a, q):
    """Brute force: (I + conj(a) kron a) vec(w) = vec(q), column-major vec."""
    b = a.shape[0]
    K = np.eye(b * b) + np.kron(a.conj(), a)
    v = np.linalg.solve(K, q.reshape(-1, order="F"))
    return v.reshape((b, b), order="F")


def _contraction(b, seed, rho=0.6):
    rng = np.random.default_rng(seed)
    a = synth.cn(rng, (b, b), 1.0)
    a *= rho / np.max(np.abs(np.linalg.eigvals(a)))
    q = synth.cn(rng, (b, b), 1.0)
    return a, q


@pytest.mark.parametrize("b", [1, 3, 7])
def test_lyapunov_solvers_match_kronecker_solve(b):
    from oracle import obc_lyapunov_fixed_point, obc_lyapunov_doubling
    a, q = _contraction(b, 50 + b)
    exact = _lyap_direct(a, q)
    wf, upd = obc_lyapunov_fixed_point(a, q, np.zeros((b, b), np.complex128), 200)
    assert _rel(wf, exact) < 1e-12 and upd < 1e-13
    wd, rest = obc_lyapunov_doubling(a, q, 8)
    assert _rel(wd, exact) < 1e-12 and rest < 1e-12


def test_lyapunov_scalar_closed_form_and_symmetry():
    from oracle import obc_lyapunov_doubling
    a, q = np.array([[0.5 + 0.2j]]), np.array([[1.3 - 0.4j]])
    wd, _ = obc_lyapunov_doubling(a, q, 10)
    assert abs(wd[0, 0] - q[0, 0] / (1 + abs(a[0, 0]) ** 2)) < 1e-14
    # anti-Hermitian q (a lesser/greater quantity) gives anti-Hermitian w
    A, Q = _contraction(5, 9)
    Q = Q - Q.conj().T
    w, _ = obc_lyapunov_doubling(A, Q, 8)
    assert _rel(w, -w.conj().T) < 1e-13


def test_lyapunov_partial_sums_and_memoized_start():
    from oracle import obc_lyapunov_fixed_point, obc_lyapunov_doubling
    a, q = _contraction(4, 3, rho=0.9)
    ah = a.conj().T
    # doubling step k holds the first 2^k terms of the alternating series
    s4 = sum((-1) ** j * np.linalg.matrix_power(a, j) @ q @ np.linalg.matrix_power(ah, j)
             for j in range(4))
    w2, _ = obc_lyapunov_doubling(a, q, 2)
    assert _rel(w2, s4) < 1e-13
    # the plain iteration from zero after N steps holds the first N terms
    w3, _ = obc_lyapunov_fixed_point(a, q, np.zeros((4, 4), np.complex128), 3)
    s3 = sum((-1) ** j * np.linalg.matrix_power(a, j) @ q @ np.linalg.matrix_power(ah, j)
             for j in range(3))
    assert _rel(w3, s3) < 1e-13
    exact = _lyap_direct(a, q)
    wm, upd = obc_lyapunov_fixed_point(a, q, exact, 2)
    assert _rel(wm, exact) < 1e-13 and upd < 1e-13
