"""Benchmark: batched FP64 RGF selected inversion on one MI355X.

Workload (one "step" = one full solve of every energy):
  G-type block-tridiagonal complex128 system, 32 blocks of 512 x 512,
  128 energies on linspace(-2, 2); H Hermitian BT random (seeded),
  S = I, Sigma^R = -0.01i I (+ -0.1i I on the two contact blocks),
  Sigma^< = i f Gamma, Sigma^> = -i (1-f) Gamma (block-diagonal), outputs the
  diagonal, upper and lower blocks of G^R, G^<, G^>.
Inputs and outputs are resident in HBM before the clock starts.

Prints one JSON line: energy-points/s, ms per step, the roofline of the
dominant kernel (complex FP64 GEMM on the matrix cores, HIP-event timed on
its launch stream inside the library) and the CPU oracle's rate on a bounded
sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
HBM_PEAK_GBS = 8000.0

# HBM traffic factor of the dominant kernel from rocprofv3 PMC counters
# (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by the copy-kernel
# calibration); None until measured for the current kernel.
MEASURED_TRAFFIC_BYTES_PER_LAUNCH = None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-blocks", type=int, default=32)
    ap.add_argument("--block-size", type=int, default=512)
    ap.add_argument("--energies", type=int, default=128)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--cpu-energies", type=int, default=2,
                    help="energies in the CPU-oracle sample (0 = skip)")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-launch HIP events")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy a 1 GiB device buffer three times "
                         "(reference kernel for HBM byte counters)")
    return ap.parse_args()


def build_inputs(n, b, n_e, seed):
    import torch
    from paper_2508_19138_amd import synth
    p = synth.g_problem(seed, n, b, n_e=n_e, expand=False)
    dev = "cuda:0"
    H = tuple(torch.from_numpy(np.ascontiguousarray(t)).to(dev) for t in p["H"])
    eye = torch.eye(b, dtype=torch.complex128, device=dev)
    sig = []
    for sc in p["sigma_scalars"]:
        s = torch.from_numpy(np.ascontiguousarray(sc)).to(dev)       # [n_e, n]
        sig.append(s[:, :, None, None] * eye)                         # [n_e, n, b, b]
    return p, H, sig


def cpu_baseline(p, n_cpu):
    """Time the oracle (as it stands) on `n_cpu` energies of the workload."""
    from oracle import rgf_selected, assemble_g
    from paper_2508_19138_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    n, b = p["n"], p["b"]
    E_all = p["energies"]
    idx = [0, len(E_all) - 1][:n_cpu] if n_cpu <= 2 else list(
        np.linspace(0, len(E_all) - 1, n_cpu).astype(int))
    sr, sl, sg = p["sigma_scalars"]
    z = np.zeros((n - 1, b, b), np.complex128)
    t0 = time.perf_counter()
    for e in idx:
        A = assemble_g(E_all[e], p["H"], (synth.eye_blocks(sr[e], b), None, None))
        rgf_selected(A, [(synth.eye_blocks(sl[e], b), z, z),
                         (synth.eye_blocks(sg[e], b), z, z)])
    dt = time.perf_counter() - t0
    return {"value": len(idx) / dt, "unit": "energy-points/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "%d of the %d energies (indices %s) of the same workload, "
                      "assembly + full forward/backward recursion, NumPy/OpenBLAS, "
                      "%.1f s" % (len(idx), len(E_all), idx, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU; --gpus %d is not supported "
              "(energies shard across GPUs with no exchange, see the design notes)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    n, b, n_e = args.n_blocks, args.block_size, args.energies

    p, H, (sr, sl, sg) = build_inputs(n, b, n_e, args.seed)
    E = np.ascontiguousarray(p["energies"])
    mk = lambda: (torch.empty((n_e, n, b, b), dtype=torch.complex128, device="cuda:0"),
                  torch.empty((n_e, n - 1, b, b), dtype=torch.complex128, device="cuda:0"),
                  torch.empty((n_e, n - 1, b, b), dtype=torch.complex128, device="cuda:0"))
    XR, XL, XG = mk(), mk(), mk()
    torch.cuda.synchronize()

    ctx = Q.Context(0, profile=not args.no_profile)
    prob = Q.make_g_problem(E, H, (sr, None, None), (sl, None, None),
                            (sg, None, None), XR, XL, XG)
    for _ in range(args.warmup):
        ctx.solve_batch([prob])
        assert prob.status == 0, prob.status
    torch.cuda.synchronize()
    ctx.reset_stats()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.solve_batch([prob])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert prob.status == 0, prob.status

    ms_step = 1000.0 * dt / args.steps
    eps = n_e * args.steps / dt
    flops_e = Q.flops_per_energy(Q.QTX_KIND_G, n, b, 2, False)
    tflops = flops_e * n_e * args.steps / dt / 1e12
    roof = None
    if not args.no_profile:
        st = ctx.kernel_stats("zgemm")
        if st["launches"]:
            avg_ms = st["ms"] / st["launches"]
            fl_launch = st["flops"] / st["launches"]
            ach = fl_launch / (avg_ms * 1e-3) / 1e12
            roof = {"bound": "mfma", "kernel": "zgemm_kernel (complex FP64, 4 real MFMA per complex product)",
                    "achieved": round(ach, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(ach / FP64_MFMA_PEAK_TFLOPS, 4),
                    "traffic": MEASURED_TRAFFIC_BYTES_PER_LAUNCH,
                    "launches": st["launches"], "avg_launch_ms": round(avg_ms, 4),
                    "algorithmic_flops_per_launch": fl_launch,
                    "algorithmic_bytes_per_launch": st["bytes"] / st["launches"]}
        inv = ctx.kernel_stats("inverse")
        elem = ctx.kernel_stats("elementwise")
    ctx.close()
    if args.copy_calibration:
        x = torch.empty(1 << 26, dtype=torch.complex128, device="cuda:0")   # 1 GiB
        x.fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    cpu = None
    if args.cpu_energies > 0:
        cpu = cpu_baseline(p, args.cpu_energies)

    out = {
        "metric": "RGF energy-points/s + % FP64 MFMA peak; p50/p99 solve latency",
        "value": round(eps, 4), "unit": "energy-points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "plain FP64 batched RGF (G-type): complex128 block-tridiagonal, "
                               "%d blocks of %dx%d, %d energies on [-2,2], block-diagonal Sigma, "
                               "outputs G^R/G^</G^> diag+upper+lower" % (n, b, b, n_e),
                   "n_blocks": n, "block_size": b, "n_energies": n_e, "seed": args.seed},
        "tflops": round(tflops, 3),
        "pct_fp64_mfma_peak": round(100.0 * tflops / FP64_MFMA_PEAK_TFLOPS, 2),
        "flops_per_energy": flops_e,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if not args.no_profile:
        out["kernel_time_ms"] = {"zgemm": round(st["ms"], 1), "inverse": round(inv["ms"], 1),
                                 "elementwise": round(elem["ms"], 1)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
