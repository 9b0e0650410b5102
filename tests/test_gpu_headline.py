"""GPU parity at the benchmark's launch shapes (32 blocks of 512).

The product kernel picks its tile per merged launch: the 128x64 tile is only
kept when a launch covers the chip twice (512 or more tiles), which at
b = 512 takes 16 or more energies per launch.  These tests solve at that
size so the wide tile runs in every operand orientation, and check:

* two sampled energies of a 16-energy solve against the oracle, block by
  block, at 1e-10 (Eqs. forward-pass / backward-pass);
* the same two energies solved as a 2-energy batch (where the launches fall
  back to the 32x32 tile) give identical bits: the tile does not change the
  result;
* the product kernel alone at 512^3 x 16 in all four orientations, with the
  128x64 tile and the two smaller ones, against NumPy;
* the same products with edge tiles in m, n and k (loaded through registers)
  give the bits of whole tiles (loaded straight into LDS), in FP64 and on
  the FP32 matrix cores.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import assemble_g, rgf_selected  # noqa: E402
from paper_2508_19138_amd import synth  # noqa: E402
from paper_2508_19138_amd import qtx_rgf as Q  # noqa: E402
from blockcmp import triple_err  # noqa: E402

DEV = "cuda:0"
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = Q.Context(0)
    yield c
    c.close()


def _device_inputs(p, idx):
    """H and the block-diagonal self-energies of energies `idx`, expanded on
    the device from the generator's per-block scalars."""
    b = p["b"]
    H = tuple(torch.from_numpy(np.ascontiguousarray(t)).to(DEV) for t in p["H"])
    eye = torch.eye(b, dtype=torch.complex128, device=DEV)
    sig = []
    for sc in p["sigma_scalars"]:
        s = torch.from_numpy(np.ascontiguousarray(sc[idx])).to(DEV)
        sig.append((s[:, :, None, None] * eye, None, None))
    return H, sig


def _outs(n_e, n, b):
    mk = lambda k: torch.empty((n_e, k, b, b), dtype=torch.complex128, device=DEV)
    return [(mk(n), mk(n - 1), mk(n - 1)) for _ in range(3)]


def _solve(ctx, p, idx):
    n, b = p["n"], p["b"]
    E = np.ascontiguousarray(p["energies"][idx])
    H, (sr, sl, sg) = _device_inputs(p, idx)
    XR, XL, XG = _outs(len(idx), n, b)
    torch.cuda.synchronize()
    prob = Q.make_g_problem(E, H, sr, sl, sg, XR, XL, XG)
    ctx.solve_batch([prob])
    assert prob.status == 0, prob.status
    return XR, XL, XG


def _at(T, e):
    return tuple(t[e].cpu().numpy() for t in T)


def _oracle(p, e):
    n, b = p["n"], p["b"]
    sr, sl, sg = p["sigma_scalars"]
    A = assemble_g(p["energies"][e], p["H"], (synth.eye_blocks(sr[e], b), None, None))
    z = np.zeros((n - 1, b, b), np.complex128)
    return rgf_selected(A, [(synth.eye_blocks(sl[e], b), z, z),
                            (synth.eye_blocks(sg[e], b), z, z)])


def test_wide_tile_solve_matches_oracle_and_small_tile_bits(ctx, monkeypatch):
    n, b = 32, 512
    grid = synth.energy_grid(128)
    idx16 = np.arange(0, 128, 8)             # 16 energies, both signs of E
    p = synth.g_problem(2024, n, b, energies=grid[idx16], expand=False)
    monkeypatch.setenv("QTX_GEMM_CFG", "1")  # start every product at 128x64
    XR, XL, XG = _solve(ctx, p, np.arange(16))
    monkeypatch.delenv("QTX_GEMM_CFG")
    sample = (0, 9)
    for e in sample:
        OR, (OL, OG) = _oracle(p, e)
        for got, ref in ((XR, OR), (XL, OL), (XG, OG)):
            err = triple_err(_at(got, e), ref)
            assert err < TOL, (e, err)
    # the same two energies alone: every launch is too small for the wide
    # tile, yet the bits are the same
    XR2, XL2, XG2 = _solve(ctx, p, np.array(sample))
    for j, e in enumerate(sample):
        for big, small in ((XR, XR2), (XL, XL2), (XG, XG2)):
            for tb, ts in zip(big, small):
                assert torch.equal(tb[e], ts[j]), e


@pytest.mark.parametrize("cfg", ["1", "0", "2"])
@pytest.mark.parametrize("opa,opb", [("N", "N"), ("N", "C"), ("C", "N"), ("C", "C")])
def test_zgemm_512_batch16_matches_numpy(ctx, monkeypatch, cfg, opa, opb):
    b, batch = 512, 16
    rng = np.random.default_rng(17 + ord(opa) + 2 * ord(opb))
    A = synth.cn(rng, (batch, b, b), 1.0)
    B = synth.cn(rng, (batch, b, b), 1.0)
    C = synth.cn(rng, (batch, b, b), 1.0)
    dA, dB, dC = (torch.from_numpy(x).to(DEV) for x in (A, B, C))
    dD = torch.empty((batch, b, b), dtype=torch.complex128, device=DEV)
    alpha, beta = 0.6 + 0.3j, -1.0 + 0.0j
    monkeypatch.setenv("QTX_GEMM_CFG", cfg)
    ctx.zgemm(opa, opb, b, b, b, alpha, dA, b, b * b, dB, b, b * b, beta, dC, b, b * b,
              dD, b, b * b, batch)
    monkeypatch.delenv("QTX_GEMM_CFG")
    D = dD.cpu().numpy()
    opA = A if opa == "N" else np.conj(np.swapaxes(A, 1, 2))
    opB = B if opb == "N" else np.conj(np.swapaxes(B, 1, 2))
    ref = alpha * (opA @ opB) + beta * C
    err = np.linalg.norm(D - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
    assert err.max() < 1e-14, err.max()


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("cfg", ["1", "0", "2"])
@pytest.mark.parametrize("opa,opb", [("N", "N"), ("N", "C"), ("C", "N"), ("C", "C")])
def test_zgemm_edge_tiles_give_the_bits_of_whole_tiles(ctx, monkeypatch, cfg, opa, opb, fp32):
    """Tiles inside the matrices load their operands from HBM straight into
    LDS; tiles that cross an edge (in m, n or k) load through registers with
    zeros outside.  Both fill the same layout and sum over k in the same
    order, so a product whose operands are zero past k = 509 gives the same
    bits computed as 512^3 (every tile whole), as 500 x 497 x 512 (edge tiles
    in m and n) and as 512 x 512 x 509 (every tile ragged in k); the same
    for the FP32 matrix-core products, which round the loaded complex128
    fragments to complex64 as they read them."""
    b, batch, kk, mm, nn = 512, 16, 509, 500, 497
    rng = np.random.default_rng(3 + ord(opa) + 5 * ord(opb))
    A = synth.cn(rng, (batch, b, b), 1.0)
    B = synth.cn(rng, (batch, b, b), 1.0)
    C = synth.cn(rng, (batch, b, b), 1.0)
    # zero the operands past k = kk (A is m x k stored, or k x m for "C")
    if opa == "N":
        A[:, :, kk:] = 0
    else:
        A[:, kk:, :] = 0
    if opb == "N":
        B[:, kk:, :] = 0
    else:
        B[:, :, kk:] = 0
    dA, dB, dC = (torch.from_numpy(x).to(DEV) for x in (A, B, C))
    alpha, beta = 0.6 + 0.3j, -1.0 + 0.5j
    monkeypatch.setenv("QTX_GEMM_CFG", cfg)
    outs = []
    for m, n, k in ((b, b, b), (mm, nn, b), (b, b, kk)):
        dD = torch.zeros((batch, b, b), dtype=torch.complex128, device=DEV)
        print("zgemm %s%s cfg %s fp32 %d %d x %d x %d" % (opa, opb, cfg, fp32, m, n, k), flush=True)
        ctx.zgemm(opa, opb, m, n, k, alpha, dA, b, b * b, dB, b, b * b, beta, dC, b, b * b,
                  dD, b, b * b, batch, fp32=fp32)
        outs.append(dD)
    monkeypatch.delenv("QTX_GEMM_CFG")
    torch.cuda.synchronize()
    whole, edge, ragk = outs
    assert torch.equal(edge[:, :mm, :nn], whole[:, :mm, :nn])
    assert torch.count_nonzero(edge[:, mm:, :]) == 0 and torch.count_nonzero(edge[:, :, nn:]) == 0
    assert torch.equal(ragk, whole)
    D = whole.cpu().numpy()
    opA = A if opa == "N" else np.conj(np.swapaxes(A, 1, 2))
    opB = B if opb == "N" else np.conj(np.swapaxes(B, 1, 2))
    ref = alpha * (opA @ opB) + beta * C
    err = np.linalg.norm(D - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
    # FP64: rounding of the 3M form; FP32: complex64 operands, FP32 sums
    assert err.max() < (2e-6 if fp32 else 1e-14), err.max()
