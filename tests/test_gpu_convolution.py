"""GPU parity of the element-wise energy convolution (Sec. "Energy
Convolutions", Eq. interaction) against the oracle (oracle.convolution,
pinned by closed forms and library routines): random inputs over ragged
element counts, output ranges off the 8- and 16-output tiles, shifts that
leave part or all of the window outside X1, the reversed (correlation)
form, sequences short enough to be staged in LDS and longer ones, and the
solver's own lesser/greater outputs convolved over energy.

Bound: each output is a sum of n2 products computed in FP64 with fused
multiply-adds (the oracle rounds each product first), so the difference is
held to 1e-14 * n2 * max|s X1| * max|X2|."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import energy_convolution  # noqa: E402
from paper_2508_19138_amd import synth  # noqa: E402
from paper_2508_19138_amd import qtx_rgf as Q  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = Q.Context(0)
    yield c
    c.close()


def _gh():
    import gpu_helpers
    return gpu_helpers


def _run(ctx, X1, X2, n_out, shift, s, rev):
    gh = _gh()
    n_elem = int(np.prod(X1.shape[1:]))
    d1, d2 = gh.dev(X1), gh.dev(X2)
    dB = torch.full((n_out,) + X1.shape[1:], complex("nan"), dtype=torch.complex128, device=gh.DEV)
    print("convolution n_elem %d n1 %d n2 %d n_out %d shift %d rev %d"
          % (n_elem, X1.shape[0], X2.shape[0], n_out, shift, rev), flush=True)
    ctx.energy_convolution(n_elem, d1, X1.shape[0], d2, X2.shape[0], dB, n_out, shift, s, rev)
    torch.cuda.synchronize()
    return dB.cpu().numpy()


def _close(got, ref, X1, X2, s):
    bound = 1e-14 * X2.shape[0] * abs(s) * np.max(np.abs(X1)) * np.max(np.abs(X2)) + 1e-300
    return np.max(np.abs(got - ref)) <= bound


@pytest.mark.parametrize("n_elem,n1,n2,n_out,shift,rev", [
    (1, 5, 4, 8, 0, 0),
    (255, 31, 16, 16, 15, 0),
    (1000, 63, 32, 37, 31, 0),
    (4097, 20, 45, 50, 3, 1),
    (300, 17, 17, 33, -5, 1),
    (513, 9, 40, 20, 60, 0),         # the window leaves X1 for the later outputs
    (77, 6, 6, 12, 40, 0),           # every output outside: zeros
    # sequences longer than 400 samples in total: the kernel without LDS staging
    (300, 260, 150, 170, 100, 0),
    (129, 301, 120, 64, -7, 1),
    (1000, 255, 128, 128, 127, 0),   # the shape of the benchmark on 1000 entries (staged in LDS)
])
def test_random_inputs_match_oracle(ctx, n_elem, n1, n2, n_out, shift, rev):
    rng = np.random.default_rng(n_elem + 3 * n1 + 7 * n2 + shift)
    X1 = synth.cn(rng, (n1, n_elem), 1.0)
    X2 = synth.cn(rng, (n2, n_elem), 1.0)
    s = 0.25 - 0.5j
    got = _run(ctx, X1, X2, n_out, shift, s, rev)
    ref = energy_convolution(X1, X2, n_out, shift, s, bool(rev))
    assert not np.any(np.isnan(got))
    assert _close(got, ref, X1, X2, s)


def test_solver_outputs_convolved_over_energy(ctx):
    """G^< and G^> of a CPU-size solve (8 blocks of 32, 16 energies),
    selected diagonal blocks: B(E_k) = s sum_k' G^>(E_k' - E_k) G^<(E_k'),
    the correlation form, on the 31 energy differences."""
    gh = _gh()
    p = synth.g_problem(1234, 8, 32, n_e=16)
    prob, XR, XL, XG = gh.solve_g(ctx, p)
    assert prob.status == 0
    GL = XL[0]                               # host [16, 8, 32, 32]
    GG = XG[0]
    s = 1j * (4.0 / 15) / (2 * np.pi)
    n_e = GL.shape[0]
    got = _run(ctx, GG, GL, 2 * n_e - 1, 0, s, 1)
    ref = energy_convolution(GG, GL, 2 * n_e - 1, 0, s, True)
    assert _close(got, ref, GG, GL, s)


def test_invalid_arguments(ctx):
    gh = _gh()
    X = gh.dev(np.zeros((4, 10), np.complex128))
    B = gh.empty((4, 10))
    with pytest.raises(Q.QtxError) as ei:               # output overlaps an input
        ctx.energy_convolution(10, X, 4, X, 4, X, 4, 0)
    assert ei.value.status == Q.QTX_ERR_INVALID_ARG
    with pytest.raises(Q.QtxError) as ei:
        ctx.energy_convolution(10, X, 0, X, 4, B, 4, 0)
    assert ei.value.status == Q.QTX_ERR_INVALID_ARG
