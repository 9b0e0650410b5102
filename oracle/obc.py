"""Retarded open-boundary surface function of a lead (Sec. "Retarded OBC").

TEST INFRASTRUCTURE ONLY (see the package header): nothing on the product
path may import, call or link this module.

A semi-infinite lead attached to a device contact gives the surface matrix
x^R, the solution of Eq. (retarded-recursion)

    x = (m - n x n')^{-1},

where m, n and n' are b x b blocks of M - B^R_scatt for the contact: the
lead's on-site block and its two couplings (n couples a layer to the next
one into the lead, n' back).  The contact's non-zero block of B^R_OBC is
n x n' (same section).

* ``obc_fixed_point`` - Eq. (naive), x_{i+1} = (m - n x_i n')^{-1}, for a
  fixed number of iterations from a given start.  Starting from the previous
  self-consistent iteration's x is the memoized mode of Sec. "OBC
  Memoization", where a fixed iteration count keeps all energies in step.
  Returns x_N, the boundary block n x_N n' and the relative size of the last
  update, ||x_N - x_{N-1}||_F / ||x_N||_F.
* ``obc_sancho_rubio`` - the decimation method the paper cites for fewer
  iterations (Lopez Sancho et al., 1985), written for M blocks.  Layers of
  the lead obey  n' X_{j-1} + m X_j + n X_{j+1} = delta_j;  eliminating every
  other layer with g = m_bulk^{-1} leaves a lead of half the layers with
      n_new  = -n g n,      n'_new = -n' g n',
      m_bulk_new = m_bulk - n g n' - n' g n,
      m_surf_new = m_surf - n g n'          (the surface has no layer -1).
  The couplings shrink geometrically; once they vanish, x = m_surf^{-1}.
* ``obc_lesser_greater`` - Sec. "Lesser/Greater OBC" for electrons: the
  lesser/greater blocks from the retarded one by fluctuation-dissipation.
* ``obc_lyapunov_fixed_point``, ``obc_lyapunov_doubling`` - the same section
  for the screened interaction: Eq. (lyapunov), w = q - a w a^dagger, by the
  plain iteration (memoized start) and by doubling.

All arithmetic is complex128 on the host; inverses are LAPACK via NumPy.
Parity pins: tests/test_oracle_obc.py.
"""

import numpy as np


def _fro(a):
    return float(np.sqrt(np.sum(np.abs(a) ** 2)))


def obc_fixed_point(m, n, np_, x0, n_iter):
    """Eq. (naive) for a fixed number of iterations.

    m, n, np_: [b, b] complex blocks (m, n, n'); x0: start [b, b] (zeros for
    a cold start).  Returns (x_N, n x_N n', ||x_N - x_{N-1}||_F / ||x_N||_F).
    """
    if n_iter < 1:
        raise ValueError("n_iter must be >= 1")
    x = np.array(x0, dtype=np.complex128)
    prev = x
    for _ in range(n_iter):
        prev = x
        x = np.linalg.inv(m - n @ x @ np_)
    upd = _fro(x - prev) / max(_fro(x), np.finfo(float).tiny)
    return x, n @ x @ np_, upd


def _decimate(m, n, np_, steps, tol):
    """Decimation steps; stops after `steps` (if given) or once the remaining
    coupling ||n_k||_F + ||n'_k||_F is at most tol times its start."""
    a = np.array(n, dtype=np.complex128)
    c = np.array(np_, dtype=np.complex128)
    ms = np.array(m, dtype=np.complex128)
    mb = np.array(m, dtype=np.complex128)
    scale = _fro(a) + _fro(c)
    k = 0
    while True:
        rest = (_fro(a) + _fro(c)) / scale if scale > 0.0 else 0.0
        if steps is not None and k == steps:
            break
        if steps is None and rest <= tol:
            break
        g = np.linalg.inv(mb)
        agc = a @ g @ c
        cga = c @ g @ a
        ms = ms - agc
        mb = mb - agc - cga
        a = -(a @ g @ a)
        c = -(c @ g @ c)
        k += 1
        if steps is None and k > 10000:
            raise RuntimeError("Sancho-Rubio decimation did not converge")
    x = np.linalg.inv(ms)
    return x, n @ x @ np_, k, rest


def obc_sancho_rubio(m, n, np_, max_iter=100, tol=1e-15):
    """Decimation until ||n_k||_F + ||n'_k||_F <= tol (||n||_F + ||n'||_F).

    Returns (x, n x n', steps taken).  Raises if it does not converge in
    max_iter steps.
    """
    x, sig, k, rest = _decimate(m, n, np_, None, tol)
    if k > max_iter:
        raise RuntimeError("Sancho-Rubio decimation did not converge in %d steps" % max_iter)
    return x, sig, k


def obc_sancho_rubio_steps(m, n, np_, steps):
    """Exactly `steps` decimation steps (the fixed count a batched solver
    runs for every energy).  Returns (x, n x n', remaining coupling
    (||n_N||_F + ||n'_N||_F) / (||n||_F + ||n'||_F))."""
    if steps < 1:
        raise ValueError("steps must be >= 1")
    x, sig, _, rest = _decimate(m, n, np_, steps, 0.0)
    return x, sig, rest


def obc_lesser_greater(sigma_r, f, one_minus_f):
    """Lesser/greater boundary blocks of a contact in equilibrium (Sec.
    "Lesser/Greater OBC"): by the fluctuation-dissipation theorem, with the
    broadening Gamma = i (Sigma^R - Sigma^R^dagger) of the retarded block,
        Sigma^< = i f Gamma,     Sigma^> = -i (1 - f) Gamma,
    f the contact's occupation at this energy (1 - f passed separately so
    that neither rounds to zero).  Returns (Sigma^<, Sigma^>)."""
    gamma = 1j * (sigma_r - sigma_r.conj().T)
    return 1j * f * gamma, -1j * one_minus_f * gamma


def obc_lyapunov_fixed_point(a, q, w0, n_iter):
    """Eq. (lyapunov), w = q - a w a^dagger (the W system's lesser/greater
    surface function), by the plain iteration w_{i+1} = q - a w_i a^dagger
    from a given start (zeros, or the previous self-consistent iteration's w
    as in Sec. "OBC Memoization").  Returns (w_N, ||w_N - w_{N-1}||_F /
    ||w_N||_F)."""
    if n_iter < 1:
        raise ValueError("n_iter must be >= 1")
    w = np.array(w0, dtype=np.complex128)
    prev = w
    ah = a.conj().T
    for _ in range(n_iter):
        prev = w
        w = q - a @ w @ ah
    return w, _fro(w - prev) / max(_fro(w), np.finfo(float).tiny)


def obc_lyapunov_doubling(a, q, steps):
    """Eq. (lyapunov) by doubling (Smith's method): the solution is the
    series w = sum_j (-1)^j a^j q (a^dagger)^j; with A_k = a^(2^k),
        S_1 = q - a q a^dagger,   S_{k+1} = S_k + A_k S_k A_k^dagger  (k >= 1),
    S_k holds the first 2^k terms.  Returns (S_steps, ||A_steps||_F / ||a||_F)."""
    if steps < 1:
        raise ValueError("steps must be >= 1")
    A = np.array(a, dtype=np.complex128)
    S = q - A @ q @ A.conj().T
    for _ in range(1, steps):
        A = A @ A
        S = S + A @ S @ A.conj().T
    A = A @ A
    na = _fro(a)
    return S, (_fro(A) / na if na > 0 else 0.0)
