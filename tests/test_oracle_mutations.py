"""Planted mistakes in the oracle modules must fail their pins.

Each case copies one oracle module, plants one plausible mistake (a flipped
sign, a dropped term, a transposed or swapped operand, a wrong band), and
runs a check built on the module's independent pins (closed forms, dense
brute force, Kronecker solves, Landauer's formula, sparsity-pattern counts).
The unmodified module must pass the same check, and every mutant must fail
it by a wide margin.  The recursion itself (oracle/rgf.py) has its own cases
in test_oracle.py.
"""

import os
import types

import numpy as np
import pytest

import oracle
from oracle import chain_closed_form, chain_lead_self_energy, dense_selected
from paper_2508_19138_amd import synth
from test_oracle import _assembly_g_error, _w_products_by_pattern
from test_oracle_obc import _contraction, _finite_lead_surface, _lyap_direct
from test_oracle_nested import _bt


def _load(module, old=None, new=None):
    path = os.path.join(os.path.dirname(oracle.__file__), module + ".py")
    with open(path) as fh:
        src = fh.read()
    if old is not None:
        assert old in src, (module, old)
        src = src.replace(old, new, 1)
    mod = types.ModuleType("mutant_" + module)
    exec(compile(src, "mutant_" + module, "exec"), mod.__dict__)
    return mod


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ------------------------------------------------------------------ checks

def _check_assembly(m):
    err = _assembly_g_error(m.assemble_g)
    # W-type against the dense masked products (Sec. 3.2.2)
    rng = np.random.default_rng(5)
    n, b = 4, 3
    V = synth.hermitian_bt(rng, n, b)
    Pr = synth.random_bt(rng, n, b)
    Ps = synth.random_bt(rng, n, b)
    Mt, (B,) = m.assemble_w(V, Pr, [Ps])
    place = lambda t: oracle.dense_from_bt(*t)
    mask = np.kron(np.array([[1.0 if abs(i - j) <= 1 else 0.0 for j in range(n)]
                             for i in range(n)]), np.ones((b, b)))
    Vd = place(V)
    refM = (np.eye(n * b) - Vd @ place(Pr)) * mask
    refB = (Vd @ place(Ps) @ Vd.conj().T) * mask
    return max(err, float(np.abs(place(Mt) - refM).max()),
               float(np.abs(place(B) - refB).max()))


def _check_flops(m):
    bad = 0
    for n in (1, 2, 3, 5, 8):
        for n_rhs in (0, 2):
            bad = max(bad, abs(m.gemm_eq_w_assembly(n, n_rhs, True)
                               - _w_products_by_pattern(n, n_rhs, True)))
    return float(bad)


def _check_obc(m):
    worst = 0.0
    for b, E, eta in ((3, 0.2, 0.3), (5, -0.7, 0.25)):
        mm, n, np_ = synth.lead_blocks(5 + b, b, [E], eta=eta)
        ref = _finite_lead_surface(mm[0], n, np_, 120)
        xs, _, _ = m.obc_sancho_rubio(mm[0], n, np_, max_iter=200)
        xf, _, _ = m.obc_fixed_point(mm[0], n, np_, np.zeros((b, b), np.complex128), 400)
        worst = max(worst, _rel(xs, ref), _rel(xf, ref))
    return worst


def _check_lesser_greater(m):
    rng = np.random.default_rng(19)
    b, t, E = 5, 1.0, 0.35
    X = synth.cn(rng, (b, b), 1.0 / b)
    h0 = 0.5 * (X + X.conj().T)
    sig = chain_lead_self_energy(E, h0, t)
    f, omf = 0.3, 0.7
    sl, sg = m.obc_lesser_greater(sig, f, omf)
    eps, U = np.linalg.eigh(h0)
    gam = -2.0 * np.imag(np.diag(U.conj().T @ sig @ U))
    return max(_rel(sl, (U * (1j * f * gam)) @ U.conj().T),
               _rel(sg, (U * (-1j * omf * gam)) @ U.conj().T))


def _check_lyapunov(m):
    a, q = _contraction(4, 61)
    exact = _lyap_direct(a, q)
    wf, _ = m.obc_lyapunov_fixed_point(a, q, np.zeros((4, 4), np.complex128), 200)
    wd, _ = m.obc_lyapunov_doubling(a, q, 8)
    return max(_rel(wf, exact), _rel(wd, exact))


def _check_observables(m):
    E, fL, fR = 0.3, 0.9, 0.2
    b, t, n = 3, 1.0, 5
    rng = np.random.default_rng(1)
    X = synth.cn(rng, (b, b), 0.5 / b)
    h0 = 0.5 * (X + X.conj().T)
    eps = np.linalg.eigvalsh(h0)
    T = int(np.sum(np.abs((E - eps) / t) < 2.0))
    CR, CL = chain_closed_form(E, h0, t, n, fL, fR)
    gd = CL[0] + (CR[0] - np.conj(np.swapaxes(CR[0], 1, 2)))
    H_up = np.stack([t * np.eye(b, dtype=np.complex128)] * (n - 1))
    dos, dens, cur = m.observables(CL, (gd, None, None), H_up)
    want_cur = T * (fL - fR) / (2 * np.pi)
    want_dos = -np.imag(np.trace(CR[0], axis1=1, axis2=2)) / np.pi
    want_dens = np.real(np.trace(-1j * CL[0], axis1=1, axis2=2)) / (2 * np.pi)
    return max(float(np.max(np.abs(cur - want_cur)) / abs(want_cur)),
               float(np.max(np.abs(dos - want_dos)) / np.max(np.abs(want_dos))),
               float(np.max(np.abs(dens - want_dens)) / np.max(np.abs(want_dens))))


def _check_nested(m):
    worst = 0.0
    for n, b, P in ((9, 2, 3), (11, 2, 4)):
        Mt = _bt(300 + n, n, b)
        Bs = [_bt(301 + n, n, b)]
        r = m.nested_dissection_selected(Mt, P, Bs)
        refR, refS = dense_selected(Mt, Bs)
        for k in range(3):
            worst = max(worst, _rel(r["XR"][k], refR[k]), _rel(r["XS"][0][k], refS[0][k]))
    return worst


def _check_nested_blocks(m):
    """The block form against the dense definition, the Schur identity
    S^{-1} = (A^{-1})_SS and the separators' block of the dense X^s."""
    worst = 0.0
    for n, b, P in ((9, 2, 3), (12, 2, 4)):
        Mt = _bt(310 + n, n, b)
        Bs = [_bt(311 + n, n, b)]
        r = m.nested_dissection_blocks(Mt, P, Bs)
        refR, refS = dense_selected(Mt, Bs)
        for k in range(3):
            worst = max(worst, _rel(r["XR"][k], refR[k]), _rel(r["XS"][0][k], refS[0][k]))
        A = oracle.dense_from_bt(*Mt)
        B = oracle.dense_from_bt(*Bs[0])
        rows = np.concatenate([np.arange(k * b, (k + 1) * b) for k in r["sep"]])
        Ai = np.linalg.inv(A)
        Si = np.linalg.inv(r["S"])
        worst = max(worst, _rel(Si, Ai[np.ix_(rows, rows)]),
                    _rel(Si @ r["BS"][0] @ Si.conj().T,
                         (Ai @ B @ Ai.conj().T)[np.ix_(rows, rows)]))
    return worst


def _check_convolution(m):
    """Worst deviation of the energy convolution from its pins: the
    geometric closed form (scaled, shifted window), a shifted delta through
    the reversed X1, and numpy's convolution."""
    rng = np.random.default_rng(4)
    a = 0.6 * np.exp(1j * rng.uniform(0, 2 * np.pi, 3)) + 0.2
    c = 0.9 * np.exp(1j * rng.uniform(0, 2 * np.pi, 3)) - 0.1
    n1, n2, n_out, shift, s = 9, 7, 10, 3, 0.4 + 0.9j
    X1 = a[None, :] ** np.arange(n1)[:, None]
    X2 = c[None, :] ** np.arange(n2)[:, None]
    got = m.energy_convolution(X1, X2, n_out, shift, s)
    r = c / a
    worst = 0.0
    for k in range(n_out):
        mm = k + shift
        lo, hi = max(0, mm - n1 + 1), min(mm, n2 - 1)
        ref = s * a ** mm * (r ** lo - r ** (hi + 1)) / (1.0 - r) if lo <= hi else 0.0 * a
        worst = max(worst, float(np.max(np.abs(got[k] - ref))))
    D = np.zeros((n2, 3), np.complex128)
    D[2] = 1.0
    Y = synth.cn(rng, (n1, 3), 1.0)
    gotd = m.energy_convolution(Y, D, n_out, shift, 1.0, True)
    for k in range(n_out):
        j = k + shift - 2
        ref = Y[::-1][j] if 0 <= j < n1 else 0.0 * Y[0]
        worst = max(worst, float(np.max(np.abs(gotd[k] - ref))))
    Z = synth.cn(rng, (n2, 3), 1.0)
    full = m.energy_convolution(Y, Z, n1 + n2 - 1, 0, 1.0)
    for i in range(3):
        worst = max(worst, float(np.max(np.abs(full[:, i] - np.convolve(Y[:, i], Z[:, i])))))
    return worst


# --------------------------------------------------------------- mutations

_CASES = [
    # Table quantities / Sec. 3.2.2
    ("assembly", "sign of E S upper", "u = u + E * Su", "u = u - E * Su", _check_assembly),
    ("assembly", "sign of Sigma^R upper", "u = u - Ru", "u = u + Ru", _check_assembly),
    ("assembly", "sign of Sigma^R lower", "l = l - Rl", "l = l + Rl", _check_assembly),
    ("assembly", "S lower from S upper", "l = l + E * Sl", "l = l + E * Su", _check_assembly),
    ("assembly", "V^dagger without conjugation",
     "else _bt_get(V, j, i, n).conj().T)", "else _bt_get(V, j, i, n).T)", _check_assembly),
    ("assembly", "truncation keeps second off-diagonal", "        elif j == i + 1:\n            u[i] = blk",
     "        elif j == i + 1 or j == i + 2:\n            u[i] = blk", _check_assembly),
    # flop model of the W assembly
    ("flops", "left band too wide", "lhs += nprod(i, j, 1, 1)", "lhs += nprod(i, j, 2, 1)",
     _check_flops),
    ("flops", "V P^s block k = i + 2 dropped",
     "for k in (i - 1, i, i + 1, i + 2):          # blocks of T = V P^s",
     "for k in (i - 1, i, i + 1):          # blocks of T = V P^s", _check_flops),
    ("flops", "W^R end blocks miscounted", "total += sum(1 + (i > 0) + (i < n - 1) for i in range(n))",
     "total += 3 * n", _check_flops),
    # Sec. "Retarded OBC"
    ("obc", "sign of the decimated coupling", "a = -(a @ g @ a)", "a = (a @ g @ a)", _check_obc),
    ("obc", "surface update from the other product", "ms = ms - agc", "ms = ms - cga", _check_obc),
    ("obc", "couplings transposed in Eq. naive", "x = np.linalg.inv(m - n @ x @ np_)",
     "x = np.linalg.inv(m - np_ @ x @ n)", _check_obc),
    # Sec. "Lesser/Greater OBC"
    ("obc", "sign of Sigma^<", "return 1j * f * gamma, -1j * one_minus_f * gamma",
     "return -1j * f * gamma, -1j * one_minus_f * gamma", _check_lesser_greater),
    ("obc", "Gamma transposed without conjugation", "gamma = 1j * (sigma_r - sigma_r.conj().T)",
     "gamma = 1j * (sigma_r - sigma_r.T)", _check_lesser_greater),
    ("obc", "sign of the Lyapunov iteration", "w = q - a @ w @ ah", "w = q + a @ w @ ah",
     _check_lyapunov),
    ("obc", "sign of the doubling update", "S = S + A @ S @ A.conj().T",
     "S = S - A @ S @ A.conj().T", _check_lyapunov),
    ("obc", "a^dagger without conjugation", "ah = a.conj().T", "ah = a.T", _check_lyapunov),
    # Sec. "Observables"
    ("observables", "Im for Re in the current", "2.0 * np.real(np.trace(H_upper[i] @ gl_l[i]))",
     "2.0 * np.imag(np.trace(H_upper[i] @ gl_l[i]))", _check_observables),
    ("observables", "upper for lower block", "gl_d, _, gl_l = (np.asarray(t) for t in GL)",
     "gl_d, gl_l, _ = (np.asarray(t) for t in GL)", _check_observables),
    ("observables", "sign in the spectral function", "1j * (gg_d[i] - gl_d[i])",
     "1j * (gl_d[i] - gg_d[i])", _check_observables),
    # Sec. "Energy Convolutions" (Eq. interaction)
    ("convolution", "energy index of X2 with the wrong sign", "j = k + shift - kp",
     "j = k + shift + kp", _check_convolution),
    ("convolution", "difference grid shift dropped", "j = k + shift - kp", "j = k - kp",
     _check_convolution),
    ("convolution", "prefactor dropped", "B[k] = scale * acc", "B[k] = acc", _check_convolution),
    ("convolution", "reversal ignored", "X1p = X1[::-1] if reverse1 else X1", "X1p = X1",
     _check_convolution),
    ("convolution", "last X1 sample left out", "if 0 <= j < n1:", "if 0 <= j < n1 - 1:",
     _check_convolution),
    # Sec. 4.4 (nested dissection)
    ("nested", "sign of X_IS", "X_IS = -a @ A_IS @ X_SS", "X_IS = a @ A_IS @ X_SS", _check_nested),
    ("nested", "sign of the Schur complement", "S = A_SS - A_SI @ a @ A_IS",
     "S = A_SS + A_SI @ a @ A_IS", _check_nested),
    ("nested", "dropped correction of X_II", "X_II = a + a @ A_IS @ X_SS @ A_SI @ a",
     "X_II = a", _check_nested),
    ("nested", "reduced right-hand side without the B_II term",
     " + A_SI @ a @ B_II @ h(a) @ h(A_SI)\n", "\n", _check_nested),
    ("nested", "X^s_IS without the separator term", "XS_IS = C_IS - a @ A_IS @ XS_SS",
     "XS_IS = C_IS", _check_nested),
    ("nested", "X^s_SI with A_SI for A_IS^dagger", "XS_SI = C_SI - XS_SS @ h(A_IS) @ h(a)",
     "XS_SI = C_SI - XS_SS @ A_SI @ h(a)", _check_nested),
    # Sec. 4.4 in block form (per-partition elimination with fill-in)
    ("nested", "sign of the fill-in column", "qn = -ln @ q", "qn = ln @ q", _check_nested_blocks),
    ("nested", "fill-in row with the lower coupling", "rn = -lT @ A(c, nx)",
     "rn = -lT @ A(nx, c)", _check_nested_blocks),
    ("nested", "top separator's block not updated", "STT = STT - lT @ q", "STT = STT",
     _check_nested_blocks),
    ("nested", "right-hand side fill-in without its x^s term",
     "RnT = [-ln @ RkT[s] - blk(B, nx, c) @ h(lT) + ln @ Rkk[s] @ h(lT)",
     "RnT = [-ln @ RkT[s] - blk(B, nx, c) @ h(lT)", _check_nested_blocks),
    ("nested", "backward X^s_kk without the Z terms",
     " + Zk @ xs[s] + xs[s] @ h(Zk)\n", "\n", _check_nested_blocks),
    ("nested", "backward X^s_kN without the right-hand side coupling",
     "XskN.append(-Pk @ XsNN[s] - xs[s] @ h(XNN @ MNk) + x @ RkN[s] @ h(XNN))",
     "XskN.append(-Pk @ XsNN[s] - xs[s] @ h(XNN @ MNk))", _check_nested_blocks),
]


@pytest.mark.parametrize("module,check", sorted({(c[0], c[4]) for c in _CASES},
                                                key=lambda t: (t[0], t[1].__name__)),
                         ids=lambda v: v if isinstance(v, str) else v.__name__)
def test_unmodified_module_passes_its_check(module, check):
    assert check(_load(module)) < 1e-10


@pytest.mark.parametrize("module,name,old,new,check", _CASES, ids=[c[1] for c in _CASES])
def test_planted_mistake_is_caught(module, name, old, new, check):
    assert check(_load(module, old, new)) > 1e-3, name
