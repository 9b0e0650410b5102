"""Helpers for the GPU parity tests: move seeded synthetic inputs to the
device, call the C ABI through the binding, and bring outputs back."""

import numpy as np
import torch

from paper_2508_19138_amd import qtx_rgf as Q

DEV = "cuda:0"


def dev(a):
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(DEV)


def empty(shape):
    return torch.empty(shape, dtype=torch.complex128, device=DEV)


def outputs(n_e, n, b, with_lower=True):
    d = empty((n_e, n, b, b))
    u = empty((n_e, max(n - 1, 0), b, b))
    l = empty((n_e, max(n - 1, 0), b, b)) if with_lower else None
    return (d, u, l)


def host(T):
    return tuple(None if t is None else t.cpu().numpy() for t in T)


def solve_g(ctx, p, want=("L", "G"), S=None, precision=Q.QTX_FP64,
            h_lower=True):
    """Run a G-type problem dict from synth.g_problem on the GPU.

    Returns (status, XR, XL, XG) with numpy triples (XL/XG None if skipped).
    """
    n, b = p["n"], p["b"]
    E = np.ascontiguousarray(p["energies"], dtype=np.float64)
    n_e = E.shape[0]
    H = (dev(p["H"][0]), dev(p["H"][1]), dev(p["H"][2]) if h_lower else None)
    sr = tuple(dev(t) for t in p["sigma_r"])
    sl = (dev(p["sigma_l"][0]), dev(p["sigma_l"][1]), None)
    sg = (dev(p["sigma_g"][0]), dev(p["sigma_g"][1]), None)
    XR = outputs(n_e, n, b)
    XL = outputs(n_e, n, b) if "L" in want else None
    XG = outputs(n_e, n, b) if "G" in want else None
    Sd = None if S is None else tuple(dev(t) for t in S)
    prob = Q.make_g_problem(E, H, sr, sl, sg, XR, XL, XG, S=Sd, precision=precision)
    st = ctx.solve_batch([prob])
    torch.cuda.synchronize()
    return (prob, host(XR), host(XL) if XL else None, host(XG) if XG else None)


def solve_w(ctx, p, want=("L", "G"), want_wr=True, v_lower=True,
            precision=Q.QTX_FP64):
    n, b = p["n"], p["b"]
    n_e = p["energies"].shape[0]
    V = (dev(p["V"][0]), dev(p["V"][1]), dev(p["V"][2]) if v_lower else None)
    Pr = tuple(dev(t) for t in p["P_r"])
    Pl = (dev(p["P_l"][0]), dev(p["P_l"][1]), None)
    Pg = (dev(p["P_g"][0]), dev(p["P_g"][1]), None)
    XR = outputs(n_e, n, b)
    XL = outputs(n_e, n, b) if "L" in want else None
    XG = outputs(n_e, n, b) if "G" in want else None
    WR = empty((n_e, n, b, b)) if want_wr else None
    prob = Q.make_w_problem(V, Pr, Pl, Pg, XR, XL, XG, WR, precision=precision)
    ctx.solve_batch([prob])
    torch.cuda.synchronize()
    return (prob, host(XR), host(XL) if XL else None, host(XG) if XG else None,
            WR.cpu().numpy() if WR is not None else None)
