"""GPU checks of qtx_rgf_zinv_noalloc, the allocation-free inverse: its
results equal qtx_rgf_zinv's bit for bit (same kernels, same order) on two
calls in a row, the second smaller than the first, so the shared static
scratch carries the first call's contents into the second; oversized calls
are refused; failures are reported per matrix as by qtx_rgf_zinv."""

import numpy as np
import pytest
import torch

from paper_2508_19138_amd import qtx_rgf as Q
from paper_2508_19138_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("needs the GPU")
    c = Q.Context(0)
    yield c
    c.close()


def _batch(seed, b, batch):
    rng = np.random.default_rng(seed)
    return np.stack([synth.cn(rng, (b, b), 1.0) + 0.5 * np.sqrt(b) * np.eye(b)
                     for _ in range(batch)])


def _both(ctx, A):
    """Inverse of every matrix of A by qtx_rgf_zinv and by the allocation-free
    entry point, each on its own copy of A (both overwrite it)."""
    batch, b = A.shape[0], A.shape[1]
    host = torch.from_numpy(np.ascontiguousarray(A))
    a1, a2 = host.to(DEV), host.to(DEV)
    x1 = torch.empty_like(a1)
    x2 = torch.full_like(a2, complex(np.nan, np.nan))
    i1 = torch.full((batch,), 7, dtype=torch.int32, device=DEV)
    i2 = torch.full((batch,), 7, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    ctx.zinv(b, a1, x1, i1, batch)
    ctx.zinv_noalloc(b, a2, x2, i2, batch)
    torch.cuda.synchronize()
    return x1.cpu().numpy(), x2.cpu().numpy(), i1.cpu().numpy(), i2.cpu().numpy()


def test_noalloc_equals_zinv_two_calls_second_smaller(ctx):
    for seed, b, batch in ((11, 512, 6), (12, 200, 3)):
        print("zinv_noalloc case: seed %d b %d batch %d" % (seed, b, batch), flush=True)
        A = _batch(seed, b, batch)
        x1, x2, i1, i2 = _both(ctx, A)
        assert np.all(i1 == 0) and np.all(i2 == 0)
        assert np.array_equal(x1.view(np.float64), x2.view(np.float64)), (b, batch)
        ref = np.linalg.inv(A)
        for e in range(batch):
            err = np.linalg.norm(x2[e] - ref[e]) / np.linalg.norm(ref[e])
            assert err < 1e-12, (b, e, err)


def test_noalloc_equals_zinv_one_launch_sizes(ctx):
    """Up to 128 rows both entry points take the one-launch inverse (no
    scratch at all, so a batch far beyond what the panel buffers would allow
    is accepted); calls in a row, each smaller than the one before."""
    for seed, b, batch in ((21, 128, 700), (22, 100, 7), (23, 64, 3), (24, 17, 2)):
        print("zinv_noalloc case: seed %d b %d batch %d" % (seed, b, batch), flush=True)
        A = _batch(seed, b, batch)
        x1, x2, i1, i2 = _both(ctx, A)
        assert np.all(i1 == 0) and np.all(i2 == 0)
        assert np.array_equal(x1.view(np.float64), x2.view(np.float64)), (b, batch)
        ref = np.linalg.inv(A)
        for e in range(batch):
            # the rounding bound of every inverse test: 1e-15 * cond_1 * b
            cond = np.linalg.norm(A[e], 1) * np.linalg.norm(ref[e], 1)
            err = np.linalg.norm(x2[e] - ref[e]) / np.linalg.norm(ref[e])
            assert err < 1e-15 * cond * b + 1e-13, (b, e, err, cond)


def _work_bytes(b, batch):
    """Scratch bytes of one call, as the header states them."""
    up = lambda x: (x + 255) // 256 * 256
    w = 64 if b <= 256 else 256
    return 2 * up(batch * b * 16 * 16) + 2 * up(batch * b * w * 16) + 2 * up(batch * b * 4)


def _largest_batch(b):
    n = 1
    while _work_bytes(b, n + 1) <= Q.QTX_NOALLOC_SCRATCH_BYTES:
        n += 1
    return n


def test_noalloc_largest_batch_that_fits(ctx):
    b = 512
    batch = _largest_batch(b)                  # 15 matrices of 512 fill 64 MiB
    assert batch == 15
    A = _batch(13, b, batch)
    x1, x2, i1, i2 = _both(ctx, A)
    assert np.all(i2 == 0)
    assert np.array_equal(x1.view(np.float64), x2.view(np.float64))


def test_noalloc_refuses_oversized_call(ctx):
    b = 512
    batch = _largest_batch(b) + 1
    a = torch.zeros((batch, b, b), dtype=torch.complex128, device=DEV)
    x = torch.empty_like(a)
    info = torch.zeros(batch, dtype=torch.int32, device=DEV)
    with pytest.raises(Q.QtxError) as ei:
        ctx.zinv_noalloc(b, a, x, info, batch)
    assert ei.value.status == Q.QTX_ERR_INVALID_ARG
    assert "scratch" in str(ei.value)
    # the context still works afterwards
    A = _batch(14, 64, 2)
    x1, x2, i1, i2 = _both(ctx, A)
    assert np.array_equal(x1.view(np.float64), x2.view(np.float64))


def test_noalloc_reports_singular_matrix(ctx):
    A = _batch(15, 40, 3)
    A[1][:, 23] = 0.0                                 # exactly singular
    x1, x2, i1, i2 = _both(ctx, A)
    assert i2[0] == 0 and i2[2] == 0 and i2[1] > 0
    assert np.array_equal(i1, i2)
    for e in (0, 2):
        assert np.array_equal(x1[e].view(np.float64), x2[e].view(np.float64))
