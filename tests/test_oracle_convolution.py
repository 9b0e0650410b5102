"""Pins of the energy-convolution oracle (Sec. "Energy Convolutions",
Eq. interaction): B[k] = s * sum_{k'} X1'[k + shift - k'] X2[k'], element
by element, X1' = X1 or X1 reversed in energy.

* Closed form: geometric sequences X1[j] = a^j, X2[k] = c^k (a different
  ratio per element) have the partial geometric sums as their convolution.
* A shifted delta in X2 copies X1' shifted.
* The library's convolution and correlation (numpy.convolve,
  numpy.correlate) element by element, on windows of the full result.
* The Fourier theorem: the full linear convolution is the inverse FFT of
  the product of the zero-padded FFTs.
"""

import numpy as np
import pytest

from oracle import energy_convolution
from paper_2508_19138_amd import synth


def _geometric_window(a, c, n1, n2, n_out, shift, scale):
    """Closed form of the window of the full convolution of a^j (j < n1) and
    c^k (k < n2): full[m] = sum_{k=lo}^{hi} a^(m-k) c^k, lo = max(0, m-n1+1),
    hi = min(m, n2-1), a geometric series in c/a."""
    out = np.zeros((n_out,) + a.shape, dtype=np.complex128)
    r = c / a
    for k in range(n_out):
        m = k + shift
        lo, hi = max(0, m - n1 + 1), min(m, n2 - 1)
        if m < 0 or lo > hi:
            continue
        out[k] = scale * a ** m * (r ** lo - r ** (hi + 1)) / (1.0 - r)
    return out


@pytest.mark.parametrize("n1,n2,n_out,shift", [(7, 5, 11, 0), (9, 9, 9, 4), (12, 6, 8, 7),
                                               (5, 10, 6, -3), (4, 4, 3, 9)])
def test_geometric_sequences_closed_form(n1, n2, n_out, shift):
    rng = np.random.default_rng(n1 * 31 + n2)
    a = 0.6 * np.exp(1j * rng.uniform(0, 2 * np.pi, 5)) + 0.2
    c = 0.9 * np.exp(1j * rng.uniform(0, 2 * np.pi, 5)) - 0.1
    X1 = a[None, :] ** np.arange(n1)[:, None]
    X2 = c[None, :] ** np.arange(n2)[:, None]
    s = 0.3 - 1.7j
    got = energy_convolution(X1, X2, n_out, shift, s)
    ref = _geometric_window(a, c, n1, n2, n_out, shift, s)
    assert np.max(np.abs(got - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("reverse1", [False, True])
def test_shifted_delta_copies_x1(reverse1):
    rng = np.random.default_rng(3)
    n1, n2, n_out, shift, d = 10, 8, 12, 3, 5
    X1 = synth.cn(rng, (n1, 2, 3), 1.0)
    X2 = np.zeros((n2, 2, 3), np.complex128)
    X2[d] = 1.0
    got = energy_convolution(X1, X2, n_out, shift, 2.0, reverse1)
    X1p = X1[::-1] if reverse1 else X1
    for k in range(n_out):
        j = k + shift - d
        ref = 2.0 * X1p[j] if 0 <= j < n1 else np.zeros((2, 3))
        assert np.array_equal(got[k], ref)


@pytest.mark.parametrize("n1,n2,n_out,shift", [(16, 16, 16, 0), (16, 16, 16, 8), (20, 13, 32, 0),
                                               (11, 17, 5, 14)])
def test_library_convolution_and_correlation(n1, n2, n_out, shift):
    rng = np.random.default_rng(n1 + 7 * n2 + shift)
    X1 = synth.cn(rng, (n1, 6), 1.0)
    X2 = synth.cn(rng, (n2, 6), 1.0)
    s = 0.05j
    conv = energy_convolution(X1, X2, n_out, shift, s)
    corr = energy_convolution(X1, X2, n_out, shift, s, reverse1=True)
    for i in range(6):
        full = np.convolve(X1[:, i], X2[:, i])                   # length n1 + n2 - 1
        # reversed X1: sum_k' X1[n1-1-(k+shift-k')] X2[k'] = sum_n X1[n] X2[n + k + shift - n1 + 1],
        # which numpy.correlate(X2, conj(X1), "full") holds at index k + shift
        # (it conjugates its second argument)
        fullr = np.correlate(X2[:, i], np.conj(X1[:, i]), mode="full")
        for k in range(n_out):
            m = k + shift
            ref = s * full[m] if 0 <= m < full.size else 0.0
            assert abs(conv[k, i] - ref) < 1e-13
            refr = s * fullr[m] if 0 <= m < fullr.size else 0.0
            assert abs(corr[k, i] - refr) < 1e-13


def test_fourier_theorem():
    rng = np.random.default_rng(11)
    n1, n2 = 24, 19
    X1 = synth.cn(rng, (n1, 4, 5), 1.0)
    X2 = synth.cn(rng, (n2, 4, 5), 1.0)
    L = 64
    full = np.fft.ifft(np.fft.fft(X1, L, axis=0) * np.fft.fft(X2, L, axis=0), axis=0)
    got = energy_convolution(X1, X2, n1 + n2 - 1, 0, 1.0)
    assert np.max(np.abs(got - full[:n1 + n2 - 1])) < 1e-12
