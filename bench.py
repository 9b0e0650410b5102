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

Other workloads (one JSON line each, not part of the default run):
  --mode mixed   the same workload with complex64 FP32-matrix-core products
                 and FP64 inverses; per-output error against the FP64 path on
                 every energy and against the CPU oracle on sampled energies.
  --mode uneven  512 independent single-energy solves of mixed block size
                 {64..768}, block count 8..128, half G-type, half W-type:
                 merged batches against a per-solve loop.
  --mode serve   a Poisson stream of G-type requests of mixed shape through
                 the request loop (qtx_rgf_submit/poll) against a per-solve
                 loop on the same arrival trace: throughput, p50/p99 latency.
  --mode nested  one long device at one energy (128 blocks of 512) by the
                 partitioned solve (nested dissection) for several partition
                 counts, against the plain solve of the same problem.
  --mode gemm    the dominant kernel alone at the workload's shape (complex
                 FP64 products D = A op(B) + C of 512 x 512 blocks, 128 per
                 launch, each operand orientation), then three copies of a
                 1 GiB buffer: the run that HBM byte counters are read on.
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

# Measured HBM bytes of the dominant kernel per algorithmic byte: rocprofv3
# --pmc FETCH_SIZE and WRITE_SIZE runs of this default workload (the
# recursion's real launch mix, 810 product launches), each scaled by the
# same counter on a 1 GiB device copy in the same run (FETCH_SIZE reads 0.500
# of the copied bytes, WRITE_SIZE 1.000): 1618018 KiB x 2 read + 968317 KiB
# written per launch against 3.3445e9 algorithmic bytes (A, B, D, and C or
# the assembled C's sources).  Taken on the kernel whose operand tiles go
# from HBM straight into LDS; None once the kernel changes.
MEASURED_TRAFFIC_FACTOR = (1618018.0 * 2.0 + 968317.0) * 1024.0 / 3344506940.68


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", default="plain",
                    choices=["plain", "mixed", "uneven", "serve", "gemm", "obc",
                             "observables", "nested", "convolution"])
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-blocks", type=int, default=32)
    ap.add_argument("--block-size", type=int, default=512)
    ap.add_argument("--energies", type=int, default=128)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--cpu-energies", type=int, default=2,
                    help="energies in the CPU-oracle sample (0 = skip)")
    ap.add_argument("--cpu-reps", type=int, default=3,
                    help="repetitions of the CPU-oracle sample (median reported)")
    ap.add_argument("--upper-only", action="store_true",
                    help="plain: lesser/greater outputs as diagonal + upper blocks only")
    ap.add_argument("--bt-sigma", action="store_true",
                    help="plain/mixed: self-energies with block-tridiagonal parts (general "
                         "path, F_BT flop model); use --energies 96 to fit HBM")
    ap.add_argument("--obc-iters", type=int, default=20,
                    help="obc: fixed-point iterations (or decimation steps) per call")
    ap.add_argument("--obc-method", default="fixed",
                    choices=["fixed", "sancho", "lyap-fixed", "lyap-doubling"],
                    help="obc: retarded surface function by memoized fixed-point iterations "
                         "or Sancho-Rubio decimation; or the W system's lesser/greater "
                         "surface function (Eq. lyapunov) by memoized iterations or doubling")
    ap.add_argument("--per-b", action="store_true",
                    help="uneven: also time the merged batch of each block size alone")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-launch HIP events")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy a 1 GiB device buffer three times "
                         "(reference kernel for HBM byte counters)")
    ap.add_argument("--solves", type=int, default=512, help="uneven: solve count")
    ap.add_argument("--only-b", type=int, default=0,
                    help="uneven: keep only the solves of this block size (0: all)")
    ap.add_argument("--skip-loop", action="store_true",
                    help="uneven: time the merged batches only")
    ap.add_argument("--repeat", type=int, default=1,
                    help="uneven: solve each wave this many times and time the last "
                         "(repeated batches replay captured graphs, as in a "
                         "self-consistent loop that re-solves the same shapes)")
    ap.add_argument("--order", default="cost", choices=["given", "length", "cost"],
                    help="uneven: order of the solves before they are cut into memory waves: "
                         "as drawn, by block count (longest chains first) or by flops "
                         "(most expensive first, the default: waves of similar solves end "
                         "with shorter tails)")
    ap.add_argument("--wave-gib", type=float, default=140.0,
                    help="uneven: device memory for the inputs/outputs of one wave")
    ap.add_argument("--requests", type=int, default=1000, help="serve: requests per rate")
    ap.add_argument("--rates", default="50,100,200,400", help="serve: arrivals per second")
    ap.add_argument("--serve-sizes", default="scaled", choices=["scaled", "matched", "literal"],
                    help="serve: request sizes: scaled (n 8..64, b in {128,192,256}, 1..16 "
                         "energies), matched (n 8..32, b in {128,256}, 16..64 energies) or "
                         "literal (n 8..64, b in {128,256,...,768}, 16..256 energies)")
    ap.add_argument("--serve-cap-s", type=float, default=0.0,
                    help="serve: stop each replay this many seconds after its first arrival "
                         "(0: serve every request)")
    ap.add_argument("--chunk-gib", type=float, default=16.0,
                    help="serve: the client splits a request into energy chunks of at most "
                         "this many GiB of self-energies and outputs, one problem each")
    ap.add_argument("--partitions", default="2,4,8,16",
                    help="nested: partition counts to time")
    ap.add_argument("--nested-blocks", type=int, default=128, help="nested: block count")
    ap.add_argument("--conv-blocks", type=int, default=16,
                    help="convolution: blocks of b x b entries convolved over energy")
    ap.add_argument("--nested-energies", type=int, default=1, help="nested: energies")
    ap.add_argument("--pool-gib", type=float, default=150.0,
                    help="serve: device memory for requests admitted by the client")
    ap.add_argument("--ws-gib", type=float, default=64.0,
                    help="uneven/serve: library workspace budget")
    return ap.parse_args()


def build_inputs(n, b, n_e, seed, bt_sigma=False):
    """H on the host generator; self-energies expanded on the device.

    Returns (problem dict, H triple, [(diag, upper, lower)] for Sigma^R,
    Sigma^<, Sigma^>).  With bt_sigma the broadening gets an energy-independent
    Hermitian block-tridiagonal part K (diagonal and coupling entries
    CN(0, 0.005/b), drawn on the device from the seed):  Gamma -> Gamma + K,
    Sigma^R = -i Gamma/2, Sigma^< = i f Gamma, Sigma^> = -i (1-f) Gamma, so
    Sigma^> - Sigma^< = Sigma^R - Sigma^A still holds block by block.
    """
    import torch
    from paper_2508_19138_amd import synth
    p = synth.g_problem(seed, n, b, n_e=n_e, expand=False)
    dev = "cuda:0"
    H = tuple(torch.from_numpy(np.ascontiguousarray(t)).to(dev) for t in p["H"])
    eye = torch.eye(b, dtype=torch.complex128, device=dev)
    sig = []
    for sc in p["sigma_scalars"]:
        s = torch.from_numpy(np.ascontiguousarray(sc)).to(dev)       # [n_e, n]
        sig.append([s[:, :, None, None] * eye, None, None])           # [n_e, n, b, b]
    if bt_sigma:
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed + 1)
        X = _cn_dev(gen, (n, b, b), 0.005 / b)
        Kd = 0.5 * (X + X.conj().transpose(1, 2))
        del X
        Ku = _cn_dev(gen, (n - 1, b, b), 0.005 / b)
        E = p["energies"]
        f = torch.from_numpy(synth.fermi(E)).to(dev)[:, None, None, None]
        fb = torch.from_numpy(synth.one_minus_fermi(E)).to(dev)[:, None, None, None]
        one = torch.ones_like(f)
        for k, coef in ((0, -0.5j * one), (1, 1j * f), (2, -1j * fb)):
            sig[k][0] += coef * Kd[None]
            sig[k][1] = (coef * Ku[None]).contiguous()
        sig[0][2] = (-0.5j * one * Ku.conj().transpose(1, 2)[None]).contiguous()
        del Kd, Ku
    return p, H, sig


def cpu_baseline(p, n_cpu, reps=3):
    """Time the oracle (as it stands) on `n_cpu` energies of the workload,
    `reps` times; the median repetition is reported.  Also returns the
    oracle's selected blocks of those energies (from the first repetition)
    so the caller can compare the GPU results with them."""
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
    times, results = [], {}
    for r in range(max(1, reps)):
        t0 = time.perf_counter()
        for e in idx:
            A = assemble_g(E_all[e], p["H"], (synth.eye_blocks(sr[e], b), None, None))
            out = rgf_selected(A, [(synth.eye_blocks(sl[e], b), z, z),
                                   (synth.eye_blocks(sg[e], b), z, z)])
            if r == 0:
                results[e] = out
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    info = {"value": len(idx) / dt, "unit": "energy-points/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "%d of the %d energies (indices %s) of the same workload, "
                      "assembly + full forward/backward recursion, NumPy/OpenBLAS; "
                      "median of %d repetitions (%s s)"
                      % (len(idx), len(E_all), idx, len(times),
                         ", ".join("%.2f" % t for t in times))}
    return info, results


def oracle_max_error(results, XR, XL, XG):
    """Largest per-block relative Frobenius error of the device outputs
    against the oracle over the sampled energies (all nine outputs)."""
    worst = 0.0
    for e, (OR, OS) in results.items():
        for X, R in zip((XR, XL, XG), (OR,) + tuple(OS)):
            for x, r in zip(X, R):
                if x is None:                  # lower blocks not written
                    continue
                g = x[e].cpu().numpy()
                num = np.linalg.norm(g - r, axis=(-2, -1))
                den = np.linalg.norm(r, axis=(-2, -1))
                den = np.where(den < 1e-13 * den.max(), den.max(), den)
                worst = max(worst, float(np.max(num / np.where(den == 0, 1.0, den))))
    return worst


def _gemm_roofline(ctx, cls, peak, label):
    st = ctx.kernel_stats(cls)
    if not st["launches"]:
        return None
    avg_ms = st["ms"] / st["launches"]
    fl_launch = st["flops"] / st["launches"]
    ach = fl_launch / (avg_ms * 1e-3) / 1e12
    # algorithmic flops are the conventional 8 b^3 per complex product; the
    # FP64 kernel's 3M form executes 6 b^3 of them on the matrix cores, so
    # its matrix cores' own utilisation is 3/4 of `frac` (frac may exceed 1)
    ex = 0.75 if cls == "zgemm" else 1.0
    return {"bound": "mfma", "kernel": label,
            "achieved": round(ach, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(ach / peak, 4),
            "mfma_utilisation": round(ex * ach / peak, 4),
            "executed_flops_per_launch": ex * fl_launch,
            "traffic": (round(MEASURED_TRAFFIC_FACTOR * st["bytes"] / st["launches"])
                        if cls == "zgemm" and MEASURED_TRAFFIC_FACTOR else None),
            "launches": st["launches"], "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_flops_per_launch": fl_launch,
            "algorithmic_bytes_per_launch": st["bytes"] / st["launches"]}


def run_plain(args, mixed=False):
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    n, b, n_e = args.n_blocks, args.block_size, args.energies

    p, H, (sr, sl, sg) = build_inputs(n, b, n_e, args.seed, args.bt_sigma)
    E = np.ascontiguousarray(p["energies"])
    mk = lambda lower=True: (
        torch.empty((n_e, n, b, b), dtype=torch.complex128, device="cuda:0"),
        torch.empty((n_e, n - 1, b, b), dtype=torch.complex128, device="cuda:0"),
        torch.empty((n_e, n - 1, b, b), dtype=torch.complex128, device="cuda:0") if lower else None)
    # --upper-only: the lesser/greater lower blocks are not written (they are
    # -upper^dagger, Sec. 4.2), which saves their HBM
    XR, XL, XG = mk(), mk(not args.upper_only), mk(not args.upper_only)
    torch.cuda.synchronize()

    ctx = Q.Context(0, profile=not args.no_profile)
    prec = Q.QTX_MIXED if mixed else Q.QTX_FP64
    prob = Q.make_g_problem(E, H, tuple(sr), tuple(sl), tuple(sg), XR, XL, XG,
                            precision=prec)
    for _ in range(args.warmup):
        ctx.solve_batch([prob])
        assert prob.status == 0, prob.status
    torch.cuda.synchronize()
    ctx.reset_stats()
    step_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        ctx.solve_batch([prob])               # synchronous: returns when done
        step_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert prob.status == 0, prob.status

    ms_step = 1000.0 * dt / args.steps
    eps = n_e * args.steps / dt
    flops_e = Q.flops_per_energy(Q.QTX_KIND_G, n, b, 2, args.bt_sigma)
    tflops = flops_e * n_e * args.steps / dt / 1e12
    roof, kt = None, None
    if not args.no_profile:
        if mixed:
            roof = _gemm_roofline(ctx, "cgemm", FP32_MFMA_PEAK_TFLOPS,
                                  "cgemm_kernel (complex64 operands, 4 real FP32 MFMA per complex product)")
        else:
            roof = _gemm_roofline(ctx, "zgemm", FP64_MFMA_PEAK_TFLOPS,
                                  "zgemm_kernel (complex FP64, 3M form: 3 real MFMA per complex product)")
        kt = {k: round(ctx.kernel_stats(k)["ms"], 1)
              for k in ("zgemm", "cgemm", "inverse", "elementwise")}
        if mixed:
            kt["fp64_zgemm_tflops"] = _tf(ctx.kernel_stats("zgemm"))
            kt["fp32_cgemm_tflops"] = _tf(ctx.kernel_stats("cgemm"))
    ctx.close()
    errors = None
    if mixed and args.bt_sigma:
        errors = "not computed for --bt-sigma (see the parity tests)"
    elif mixed:
        with Q.Context(0, budget_bytes=8 << 30) as ctx64:
            errors = mixed_errors(ctx64, p, E, H, (sr, sl, sg), (XR, XL, XG), args)
    if args.copy_calibration:
        x = torch.empty(1 << 26, dtype=torch.complex128, device="cuda:0")   # 1 GiB
        x.fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    cpu, oracle_err = None, None
    if args.cpu_energies > 0 and not mixed and not args.bt_sigma:
        cpu, ref = cpu_baseline(p, args.cpu_energies, args.cpu_reps)
        oracle_err = oracle_max_error(ref, XR, XL, XG)

    out = {
        "metric": "RGF energy-points/s + % FP64 MFMA peak; p50/p99 solve latency",
        "value": round(eps, 4), "unit": "energy-points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64-mfma/f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": "%s batched RGF (G-type): complex128 block-tridiagonal, "
                               "%d blocks of %dx%d, %d energies on [-2,2], %s Sigma, "
                               "outputs G^R/G^</G^> diag+upper+lower"
                               % ("mixed-precision" if mixed else "plain FP64", n, b, b, n_e,
                                  "block-tridiagonal" if args.bt_sigma else "block-diagonal"),
                   "n_blocks": n, "block_size": b, "n_energies": n_e, "seed": args.seed},
        "tflops": round(tflops, 3),
        "pct_fp64_mfma_peak": round(100.0 * tflops / FP64_MFMA_PEAK_TFLOPS, 2),
        "flops_per_energy": flops_e,
        "roofline": roof,
        "cpu_baseline": cpu,
        "latency_s": {"p50": round(float(np.percentile(step_s, 50)), 4),
                      "p99": round(float(np.percentile(step_s, 99)), 4),
                      "what": "wall time of one solve_batch call (all %d energies) "
                              "over the %d timed steps" % (n_e, args.steps)},
        "oracle_max_block_rel_err": oracle_err,
        "context": PAPER_CONTEXT,
    }
    if args.upper_only:
        blk = 16.0 * b * b
        out["symmetric_storage"] = {
            "lower_blocks_not_written": 2 * (n - 1) * n_e,
            "hbm_saved_bytes": 2 * (n - 1) * n_e * blk,
            "output_bytes_written": ((3 * n - 2) + 2 * (2 * n - 1)) * n_e * blk,
            "energies_per_lane": n_e,
            "what": "X^< and X^> lower blocks left to the caller as -upper^dagger (Sec. 4.2)"}
    if mixed:
        out["mode"] = "mixed"
        out["errors"] = errors
    if kt is not None:
        out["kernel_time_ms"] = kt
    print(json.dumps(out), flush=True)


def _tf(st):
    return round(st["flops"] / (st["ms"] * 1e-3) / 1e12, 3) if st["ms"] else None


def _rel_blocks(x, y):
    """Per-block ||x - y||_F / ||y||_F (blocks on the last two axes), flat."""
    import torch
    d = torch.linalg.matrix_norm(x - y)
    r = torch.linalg.matrix_norm(y)
    return (d / torch.clamp(r, min=1e-300)).reshape(-1).cpu()


def mixed_errors(ctx, p, E, H, sig, Xmix, args):
    """Per-output error of the mixed-precision result: against the FP64
    library path on every energy, and against the CPU oracle on sampled
    energies."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    from paper_2508_19138_amd import synth
    from oracle import rgf_selected, assemble_g
    n, b, n_e = p["n"], p["b"], len(E)
    sr, sl, sg = sig
    names = ("G^R", "G^<", "G^>")
    parts = ("diag", "upper", "lower")
    per = {}
    ch = 8                                    # FP64 reference in energy chunks
    for e0 in range(0, n_e, ch):
        e1 = min(n_e, e0 + ch)
        X64 = tuple(tuple(torch.empty_like(t[e0:e1]) for t in T) for T in Xmix)
        Ec = np.ascontiguousarray(E[e0:e1])
        prob = Q.make_g_problem(Ec, H, (sr[0][e0:e1], None, None), (sl[0][e0:e1], None, None),
                                (sg[0][e0:e1], None, None), *X64)
        ctx.solve_batch([prob])
        torch.cuda.synchronize()
        for nm, A, B in zip(names, Xmix, X64):
            for pt, a, bb in zip(parts, A, B):
                k = "%s %s" % (nm, pt)
                per.setdefault(k, []).append(_rel_blocks(a[e0:e1], bb))
        del X64
    vs_fp64 = {k: {"max": float(torch.cat(v).max()), "median": float(torch.cat(v).median())}
               for k, v in per.items()}
    per = {}
    idx = [0, n_e // 2]
    srs, sls, sgs = p["sigma_scalars"]
    z = np.zeros((n - 1, b, b), np.complex128)
    for e in idx:
        A = assemble_g(E[e], p["H"], (synth.eye_blocks(srs[e], b), None, None))
        XR, XS = rgf_selected(A, [(synth.eye_blocks(sls[e], b), z, z),
                                  (synth.eye_blocks(sgs[e], b), z, z)])
        for nm, ref, mix in zip(names, [XR] + list(XS), Xmix):
            for pt, r, m in zip(parts, ref, mix):
                key = "%s %s" % (nm, pt)
                per.setdefault(key, []).append(_rel_blocks(m[e].cpu(), torch.from_numpy(np.asarray(r))))
    vs_oracle = {k: {"max": float(torch.cat(v).max()), "median": float(torch.cat(v).median())}
                 for k, v in per.items()}
    return {"metric": "per-block ||X_mixed - X_ref||_F / ||X_ref||_F: max and median over blocks",
            "vs_fp64_library_all_energies": vs_fp64,
            "vs_cpu_oracle": vs_oracle, "oracle_energy_indices": idx}


# ------------------------------------------------------------ uneven batch --

def _cn_dev(gen, shape, var):
    import torch
    z = torch.randn(shape, dtype=torch.complex128, device="cuda:0", generator=gen)
    return z * np.sqrt(var)


def _herm_bt_dev(gen, n, b, scale=1.0):
    """Device draw of the Hermitian block-tridiagonal generator: H_ii =
    (X + X^dagger)/2, X ~ CN(0, 1/b); H_{i,i+1} ~ CN(0, 0.25/b); lower =
    upper^dagger (left to the library: passed as NULL)."""
    X = _cn_dev(gen, (n, b, b), 1.0 / b)
    d = 0.5 * (X + X.conj().transpose(1, 2))
    del X
    u = _cn_dev(gen, (max(n - 1, 0), b, b), 0.25 / b)
    if scale != 1.0:
        d, u = d * scale, u * scale
    return d.contiguous(), u.contiguous()


def _eye_dev(scal, b):
    """[n_e, n] complex scalars -> [n_e, n, b, b] multiples of the identity."""
    import torch
    s = torch.from_numpy(np.ascontiguousarray(scal)).to("cuda:0")
    out = torch.zeros(s.shape + (b, b), dtype=torch.complex128, device="cuda:0")
    out.diagonal(dim1=-2, dim2=-1).copy_(s[..., None].expand(s.shape + (b,)))
    return out


def _outs_dev(n_e, n, b):
    import torch
    e = lambda k: torch.empty((n_e, k, b, b), dtype=torch.complex128, device="cuda:0")
    return (e(n), e(n - 1), e(n - 1))


def _solve_bytes(spec, n_e=1):
    n, b = spec["n"], spec["b"]
    blk = 16 * b * b
    if spec["kind"] == "G":
        return blk * (2 * n + 3 * n * n_e + 9 * n * n_e)
    return blk * (2 * n + 5 * n * n_e + 9 * n * n_e)


def _uneven_problem(spec):
    """Inputs/outputs of one single-energy solve drawn on the device with the
    G-type / W-type generators (same distributions as the seeded host
    generators used by the tests)."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    from paper_2508_19138_amd import synth
    n, b = spec["n"], spec["b"]
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(spec["seed"])
    E = np.array([spec["E"]])
    keep = {"E": E}
    if spec["kind"] == "G":
        Hd, Hu = _herm_bt_dev(gen, n, b)
        sr, sl, sg = synth.g_sigma_scalars(E, n)
        keep["ins"] = ((Hd, Hu, None), (_eye_dev(sr, b), None, None),
                       (_eye_dev(sl, b), None, None), (_eye_dev(sg, b), None, None))
        keep["outs"] = (_outs_dev(1, n, b), _outs_dev(1, n, b), _outs_dev(1, n, b))
        keep["prob"] = Q.make_g_problem(E, *keep["ins"], *keep["outs"])
    else:
        Vd, Vu = _herm_bt_dev(gen, n, b, 0.5)
        Phd, Phu = _herm_bt_dev(gen, n, b, 0.5)
        eye = torch.eye(b, dtype=torch.complex128, device="cuda:0")
        Prd = (0.5 * (Phd + 0.1 * spec["E"] * eye) - 0.01j * eye)[None].contiguous()
        Pru = (0.5 * Phu)[None].contiguous()
        Prl = Pru[0].conj().transpose(1, 2)[None].contiguous()
        del Phd, Phu
        f = synth.fermi(E)
        fb = synth.one_minus_fermi(E)
        Pl = _eye_dev(np.broadcast_to((1j * 0.02 * f)[:, None], (1, n)), b)
        Pg = _eye_dev(np.broadcast_to((-1j * 0.02 * fb)[:, None], (1, n)), b)
        keep["ins"] = ((Vd, Vu, None), (Prd, Pru, Prl), (Pl, None, None), (Pg, None, None))
        keep["outs"] = (_outs_dev(1, n, b), _outs_dev(1, n, b), _outs_dev(1, n, b))
        keep["prob"] = Q.make_w_problem(*keep["ins"], *keep["outs"])
    return keep


def _waves(specs, cap):
    waves, cur, used = [], [], 0
    for sp in specs:
        by = _solve_bytes(sp)
        if cur and used + by > cap:
            waves.append(cur)
            cur, used = [], 0
        cur.append(sp)
        used += by
    if cur:
        waves.append(cur)
    return waves


def _spec_flops(Q, sp):
    return Q.flops_per_energy(Q.QTX_KIND_G if sp["kind"] == "G" else Q.QTX_KIND_W,
                              sp["n"], sp["b"], 2, sp["kind"] == "W", False)


def run_uneven(args):
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    from paper_2508_19138_amd import synth
    specs = synth.uneven_specs(args.seed, args.solves)
    if args.only_b:
        specs = [sp for sp in specs if sp["b"] == args.only_b]
        if not specs:
            raise SystemExit("no solve of block size %d in the workload" % args.only_b)
    cap = int(args.wave_gib * 2 ** 30)
    flops = {id(sp): _spec_flops(Q, sp) for sp in specs}
    if args.order == "length":
        specs = sorted(specs, key=lambda sp: -sp["n"])
    elif args.order == "cost":
        specs = sorted(specs, key=lambda sp: -flops[id(sp)])
    waves = _waves(specs, cap)
    ws = int(args.ws_gib * 2 ** 30)
    # without --repeat every wave is a different batch: no launch segment
    # repeats, so graph capture (done on a segment's second sight) would only
    # add its cost
    os.environ["QTX_GRAPHS"] = "1" if args.repeat > 1 else "0"
    ctx = Q.Context(0, budget_bytes=ws, profile=False)
    # warm-up: tile tuning for every block size and both kinds, then the
    # first wave once (workspace growth) -- untimed
    for b in sorted({sp["b"] for sp in specs}):
        for kind in ("G", "W"):
            w = _uneven_problem({"kind": kind, "n": 3, "b": b, "E": 0.1, "seed": 1})
            ctx.solve_batch([w["prob"]])
    t_merged, t_loop, tf_total = 0.0, 0.0, 0.0
    for wi, wave in enumerate(waves):
        probs = [_uneven_problem(sp) for sp in wave]
        torch.cuda.synchronize()
        if wi == 0 and args.repeat == 1:
            ctx.solve_batch([k["prob"] for k in probs])
            torch.cuda.synchronize()
        for _ in range(args.repeat - 1):          # untimed: first sight, capture
            ctx.solve_batch([k["prob"] for k in probs])
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.solve_batch([k["prob"] for k in probs])
        torch.cuda.synchronize()
        t_merged += time.perf_counter() - t0
        assert st == Q.QTX_OK, st
        if not args.skip_loop:
            t0 = time.perf_counter()
            for k in probs:
                ctx.solve_batch([k["prob"]])
            torch.cuda.synchronize()
            t_loop += time.perf_counter() - t0
        tf_total += sum(flops[id(sp)] for sp in wave)
        print("wave %d/%d: %d solves, merged %.3f s, loop %.3f s (cumulative)"
              % (wi + 1, len(waves), len(wave), t_merged, t_loop), file=sys.stderr, flush=True)
        del probs
        torch.cuda.empty_cache()
    per_b = None
    if args.per_b:
        per_b = {}
        for b in sorted({sp["b"] for sp in specs}):
            sub = [sp for sp in specs if sp["b"] == b]
            tb, fb = 0.0, 0.0
            for wave in _waves(sub, cap):
                probs = [_uneven_problem(sp) for sp in wave]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                assert ctx.solve_batch([k["prob"] for k in probs]) == Q.QTX_OK
                torch.cuda.synchronize()
                tb += time.perf_counter() - t0
                fb += sum(_spec_flops(Q, sp) for sp in wave)
                del probs
                torch.cuda.empty_cache()
            per_b[str(b)] = {"solves": len(sub), "s": round(tb, 3),
                             "tflops": round(fb / tb / 1e12, 3),
                             "pct_fp64_mfma_peak": round(100 * fb / tb / 1e12 / FP64_MFMA_PEAK_TFLOPS, 2)}
            print("b=%d alone: %s" % (b, per_b[str(b)]), file=sys.stderr, flush=True)
    ctx.close()
    n_sol = len(specs)
    out = {
        "mode": "uneven",
        "metric": "RGF energy-points/s + % FP64 MFMA peak; p50/p99 solve latency",
        "value": round(n_sol / t_merged, 3), "unit": "energy-points/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batched uneven solves: %d independent single-energy complex128 "
                               "RGF solves, b from %s, n from 8..128, "
                               "half G-type half W-type (W with W^< W^> outputs), merged "
                               "batches in %d memory waves"
                               % (n_sol, "{%d}" % args.only_b if args.only_b
                                  else "{64,128,256,384,512,768}", len(waves)),
                   "solves": n_sol, "waves": len(waves), "order": args.order, "seed": args.seed,
                   "timed_solve_of_each_wave": args.repeat},
        "merged": {"s": round(t_merged, 3), "energy_points_per_s": round(n_sol / t_merged, 3),
                   "tflops": round(tf_total / t_merged / 1e12, 3),
                   "pct_fp64_mfma_peak": round(100 * tf_total / t_merged / 1e12 / FP64_MFMA_PEAK_TFLOPS, 2)},
        "per_solve_loop": None if args.skip_loop else {
            "s": round(t_loop, 3), "energy_points_per_s": round(n_sol / t_loop, 3),
            "tflops": round(tf_total / t_loop / 1e12, 3)},
        "speedup_merged_vs_loop": None if args.skip_loop else round(t_loop / t_merged, 3),
        "total_canonical_tflop": round(tf_total / 1e12, 3),
        "merged_per_block_size": per_b,
    }
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------------- serving --

def _serve_trace(args, rate):
    rng = np.random.default_rng(args.seed + int(rate))
    R = args.requests
    gaps = rng.exponential(1.0 / rate, size=R)
    arr = np.cumsum(gaps) - gaps[0]
    reqs = []
    n_lo, n_hi, bs, e_lo, e_hi = _SERVE_SIZES[args.serve_sizes]
    for i in range(R):
        reqs.append({"n": int(rng.integers(n_lo, n_hi + 1)), "b": int(rng.choice(bs)),
                     "ne": int(rng.integers(e_lo, e_hi + 1)), "t": float(arr[i]),
                     "e0": float(rng.uniform(-2.0, 1.0))})
    return reqs


# request sizes: (n min, n max, block sizes, energies min, energies max)
_SERVE_SIZES = {
    "scaled": (8, 64, (128, 192, 256), 1, 16),
    "matched": (8, 32, (128, 256), 16, 64),
    "literal": (8, 64, (128, 256, 384, 512, 640, 768), 16, 256),
}


def _chunks(r, i, cap_elems):
    """The client's split of request i into energy chunks (one problem each)
    of at most cap_elems complex128 elements of self-energies and outputs."""
    per_e = _req_elems(dict(r, ne=1))
    k = max(1, min(r["ne"], cap_elems // per_e))
    E = np.linspace(r["e0"], r["e0"] + 1.0, r["ne"])
    return [{"req": i, "n": r["n"], "b": r["b"], "ne": len(E[j:j + k]), "E": E[j:j + k]}
            for j in range(0, r["ne"], k)]


class _Arena:
    """The client's request memory: one device allocation made up front and
    carved first-fit into per-request regions (in complex128 elements), so
    that admitting a request calls no allocator.  A caching allocator that
    runs short of memory frees its cached blocks, and each free waits for
    the whole device, i.e. for the library's queued work."""

    ALIGN = 16                                  # elements (256 bytes)

    def __init__(self, gib):
        import torch
        self.n = int(gib * 2 ** 30) // 16 // self.ALIGN * self.ALIGN
        self.buf = torch.empty(self.n, dtype=torch.complex128, device="cuda:0")
        self.free = [(0, self.n)]               # sorted (offset, length)

    def _round(self, n):
        return (n + self.ALIGN - 1) // self.ALIGN * self.ALIGN

    def alloc(self, n):
        n = self._round(n)
        for k, (o, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    del self.free[k]
                else:
                    self.free[k] = (o + n, l - n)
                return o
        return None

    def release(self, o, n):
        import bisect
        n = self._round(n)
        k = bisect.bisect(self.free, (o, 0))
        self.free.insert(k, (o, n))
        if k + 1 < len(self.free) and o + n == self.free[k + 1][0]:
            self.free[k] = (o, n + self.free[k + 1][1])
            del self.free[k + 1]
        if k > 0 and self.free[k - 1][0] + self.free[k - 1][1] == o:
            self.free[k - 1] = (self.free[k - 1][0], self.free[k - 1][1] + self.free[k][1])
            del self.free[k]


def _req_elems(r):
    """complex128 elements of one request's self-energies and outputs."""
    bb, n, ne = r["b"] * r["b"], r["n"], r["ne"]
    return bb * ne * (3 * n + 3 * (n + 2 * (n - 1)))


class _ServeInputs:
    """Shared read-only H per block size (prefix views per block count);
    per-request self-energies and outputs are views of a region of the
    client's arena, filled when the client admits the request."""

    def __init__(self, seed, arena, sizes="scaled"):
        import torch
        self.arena = arena
        self.H = {}
        n_hi, bs = _SERVE_SIZES[sizes][1], _SERVE_SIZES[sizes][2]
        for b in bs:
            gen = torch.Generator(device="cuda:0")
            gen.manual_seed(seed + b)
            self.H[b] = _herm_bt_dev(gen, n_hi, b)

    def make(self, r):
        """The request's problem, or None while the arena has no room."""
        import torch
        from paper_2508_19138_amd import qtx_rgf as Q
        from paper_2508_19138_amd import synth
        n, b, ne = r["n"], r["b"], r["ne"]
        size = _req_elems(r)
        off = self.arena.alloc(size)
        if off is None:
            return None
        buf = self.arena.buf
        pos = [off]

        def take(k):
            t = buf[pos[0]:pos[0] + ne * k * b * b].view(ne, k, b, b)
            pos[0] += ne * k * b * b
            return t

        E = np.ascontiguousarray(r["E"] if "E" in r else np.linspace(r["e0"], r["e0"] + 1.0, ne))
        sig = []
        for scal in synth.g_sigma_scalars(E, n):
            t = take(n)
            t.zero_()
            sc = torch.from_numpy(np.ascontiguousarray(scal)).to("cuda:0")
            t.diagonal(dim1=-2, dim2=-1).copy_(sc[..., None].expand(ne, n, b))
            sig.append(t)
        outs = tuple((take(n), take(n - 1), take(n - 1)) for _ in range(3))
        Hd, Hu = self.H[b]
        ins = ((Hd[:n], Hu[:n - 1], None), (sig[0], None, None),
               (sig[1], None, None), (sig[2], None, None))
        return {"E": E, "ins": ins, "outs": outs, "off": off, "size": size,
                "prob": Q.make_g_problem(E, *ins, *outs)}

    def release(self, k):
        self.arena.release(k["off"], k["size"])


def _lat_summary(lat, n_e_tot, t_span):
    lat = np.asarray(lat)
    out = {"energy_points_per_s": round(n_e_tot / t_span, 2),
           "requests_per_s": round(len(lat) / t_span, 2), "span_s": round(t_span, 3)}
    if len(lat):
        out.update({"p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                    "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                    "mean_latency_s": round(float(lat.mean()), 4)})
    return out


def _serve_run(ctx, inputs, reqs, served, cap_elems, cap_s=0.0):
    """Replay the arrival trace.  A request becomes its energy chunks when
    it arrives (the client's split, one problem each) and completes with its
    last chunk.  served: chunks are submitted to the request loop in arrival
    order while the client's arena has room; otherwise each chunk is solved
    alone, in arrival order, as soon as the previous one is done.  With
    cap_s > 0 the replay stops cap_s seconds after the first arrival (work
    then in flight is drained and not counted).  Returns the latencies of
    the completed requests, the span, diagnostics, and the energy points,
    flops and arrived-but-unfinished requests of the span."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    R = len(reqs)
    lat = [None] * R
    left = [0] * R
    diag = {"client_wait": [], "lib_queue": [], "lib_latency": []}
    queue, nxt = [], 0
    st = {"req": 0, "e": 0, "flops": 0.0, "last": 0.0}
    live = {}
    t0 = time.perf_counter()
    st["last"] = t0

    def finish(ch, tn):
        i = ch["req"]
        left[i] -= 1
        st["e"] += ch["ne"]
        st["flops"] += ch["ne"] * Q.flops_per_energy(Q.QTX_KIND_G, ch["n"], ch["b"], 2, False)
        st["last"] = tn
        if left[i] == 0:
            lat[i] = (tn - t0) - reqs[i]["t"]
            st["req"] += 1
            if st["req"] % 1000 == 0:
                print("  %s %d/%d" % ("served" if served else "per-solve loop", st["req"], R),
                      file=sys.stderr, flush=True)

    def in_cap(tn):
        return not cap_s or tn - t0 <= cap_s

    while st["req"] < R:
        now = time.perf_counter() - t0
        if cap_s and now >= cap_s:
            break
        while nxt < R and reqs[nxt]["t"] <= now:
            chs = _chunks(reqs[nxt], nxt, cap_elems)
            left[nxt] = len(chs)
            queue.extend(chs)
            nxt += 1
        if served:
            while queue:
                k = inputs.make(queue[0])
                if k is None:
                    assert live, "request chunk larger than the client arena"
                    break
                ch = queue.pop(0)
                torch.cuda.current_stream().synchronize()     # inputs written
                diag["client_wait"].append(time.perf_counter() - t0 - reqs[ch["req"]]["t"])
                live[ctx.submit(k["prob"])] = (ch, k)
            wait = 1 if (cap_s or nxt < R or queue) else 50
            cs, _ = ctx.poll(cap=64, wait_ms=wait)
            tn = time.perf_counter()
            for c in cs:
                ch, k = live.pop(c["ticket"])
                assert c["status"] == 0, c
                diag["lib_queue"].append(c["queue_s"])
                diag["lib_latency"].append(c["latency_s"])
                inputs.release(k)
                if in_cap(tn):
                    finish(ch, tn)
        else:
            if not queue:
                dt = reqs[nxt]["t"] - (time.perf_counter() - t0)
                if cap_s:
                    dt = min(dt, cap_s - (time.perf_counter() - t0))
                if dt > 0:
                    time.sleep(dt)
                continue
            ch = queue.pop(0)
            k = inputs.make(ch)
            torch.cuda.current_stream().synchronize()         # inputs written
            ctx.solve_batch([k["prob"]])
            assert k["prob"].status == 0
            tn = time.perf_counter()
            inputs.release(k)
            if in_cap(tn):
                finish(ch, tn)
    while live:                                               # drain, not counted
        cs, _ = ctx.poll(cap=64, wait_ms=50)
        for c in cs:
            ch, k = live.pop(c["ticket"])
            inputs.release(k)
    span = cap_s if cap_s else st["last"] - t0
    done = [x for x in lat if x is not None]
    return done, span, diag, st["e"], st["flops"], nxt - st["req"]


def run_serve(args):
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    rates = [float(x) for x in args.rates.split(",") if x]
    ws = int(args.ws_gib * 2 ** 30)
    inputs = _ServeInputs(args.seed, _Arena(args.pool_gib), args.serve_sizes)
    cap_elems = int(args.chunk_gib * 2 ** 30) // 16
    results = []
    ctx_s = Q.Context(0, budget_bytes=ws)
    ctx_l = Q.Context(0, budget_bytes=ws)
    # warm-up (tile tuning, workspace, request-loop start): untimed
    warm = [{"n": 8, "b": b, "ne": 2, "t": 0.0, "e0": -0.5} for b in _SERVE_SIZES[args.serve_sizes][2]]
    for r in warm:
        k = inputs.make(r)
        torch.cuda.synchronize()
        ctx_l.solve_batch([k["prob"]])
        t = ctx_s.submit(k["prob"])
        while True:
            cs, _ = ctx_s.poll(cap=4, wait_ms=100)
            if any(c["ticket"] == t for c in cs):
                break
        inputs.release(k)
    for rate in rates:
        reqs = _serve_trace(args, rate)
        n_e_tot = sum(r["ne"] for r in reqs)
        req_flops = np.mean([Q.flops_per_energy(Q.QTX_KIND_G, r["n"], r["b"], 2, False) * r["ne"]
                             for r in reqs])
        row = {"rate_per_s": rate, "requests": len(reqs), "energy_points": n_e_tot,
               "mean_request_tflop": round(req_flops / 1e12, 4)}
        for name, ctx, served in (("served", ctx_s, True), ("per_solve_loop", ctx_l, False)):
            lat, span, diag, e_done, fl_done, unfinished = _serve_run(
                ctx, inputs, reqs, served, cap_elems, args.serve_cap_s)
            row[name] = _lat_summary(lat, e_done, span)
            row[name]["tflops"] = round(fl_done / span / 1e12, 3)
            if args.serve_cap_s:
                row[name]["requests_completed"] = len(lat)
                row[name]["requests_arrived_not_completed"] = unfinished
            if served:
                # where the time goes: arrival -> submit in the client (input
                # set-up, memory admission), submit -> first lane admitted and
                # submit -> complete inside the library
                row[name]["p50_p99_s"] = {
                    k: [round(float(np.percentile(v, 50)), 4), round(float(np.percentile(v, 99)), 4)]
                    for k, v in diag.items() if v}
            print("rate %g %s: %s" % (rate, name, row[name]), file=sys.stderr, flush=True)
            torch.cuda.synchronize()
        row["throughput_ratio_served_vs_loop"] = round(
            row["served"]["energy_points_per_s"] / max(row["per_solve_loop"]["energy_points_per_s"], 1e-9), 3)
        results.append(row)
    ctx_s.close()
    ctx_l.close()
    # offered load: arrival rate x mean request work over the largest served
    # throughput measured (the loop's capacity)
    cap_tf = max(r["served"]["tflops"] for r in results)
    for r in results:
        r["offered_load_vs_served_capacity"] = round(
            r["rate_per_s"] * r["mean_request_tflop"] / cap_tf, 3)
    top = results[-1]
    out = {
        "mode": "serve",
        "metric": "RGF energy-points/s + % FP64 MFMA peak; p50/p99 solve latency",
        "value": top["served"]["energy_points_per_s"], "unit": "energy-points/s",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "serving stream (%s sizes): Poisson arrivals, %d G-type requests "
                               "per rate, each n in %d..%d blocks of b in {%s}, %d..%d energies "
                               "in a window of width 1 in [-2,2], split by the client into energy "
                               "chunks of at most %.0f GiB; chunks admitted in arrival order into "
                               "a %.0f GiB device arena allocated up front; latency = arrival to "
                               "observed completion of the last chunk%s"
                               % ((args.serve_sizes, args.requests) + _SERVE_SIZES[args.serve_sizes][:2]
                                  + (",".join(str(x) for x in _SERVE_SIZES[args.serve_sizes][2]),)
                                  + _SERVE_SIZES[args.serve_sizes][3:]
                                  + (args.chunk_gib, args.pool_gib,
                                     "; each replay stopped %.0f s after its first arrival "
                                     "(work then in flight not counted)" % args.serve_cap_s
                                     if args.serve_cap_s else "")),
                   "rates_per_s": rates, "seed": args.seed, "sizes": args.serve_sizes,
                   "time_cap_s": args.serve_cap_s or None},
        "rates": results,
    }
    print(json.dumps(out), flush=True)


FP32_MFMA_PEAK_TFLOPS = 157.3     # MI355X dense FP32 matrix peak

# The paper's own figures, for context only (other hardware, other inputs):
# per-GPU RGF rates derived as workload / time from its per-kernel table, and
# its whole-application run.
PAPER_CONTEXT = {
    "paper_rgf_single_gpu_best": "G-type RGF, NR-23 (b=3408, n=23) on one GH200: "
                                 "244.077 Tflop in 5.963 s = 40.9 TFLOP/s, 61% of its "
                                 "FP64 tensor-core peak",
    "paper_rgf_single_gcd_mi250x": "G-type RGF, NR-16 (b=3408, n=16) on one MI250X GCD: "
                                   "167.704 Tflop in 7.873 s = 21.3 TFLOP/s, 44.5% of peak",
    "paper_full_application": "1.15 Eflop/s FP64 on 37,600 MI250X (75,200 GCDs), "
                              "42.1 s per SCBA iteration, 42,240 atoms",
}


def run_lyapunov(args):
    """w = q - a w a^dagger for all energies per call (memoized iterations
    from the previous call's w, or doubling from scratch)."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    from paper_2508_19138_amd import synth
    b, ne, it = args.block_size, args.energies, args.obc_iters
    dbl = args.obc_method == "lyap-doubling"
    a, q = synth.lyapunov_blocks(args.seed, b, ne)
    da, dq = torch.from_numpy(a).to("cuda:0"), torch.from_numpy(q).to("cuda:0")
    w = torch.zeros((ne, b, b), dtype=torch.complex128, device="cuda:0")
    out = torch.empty(ne, dtype=torch.float64, device="cuda:0")
    n_prod = (2 + 3 * (it - 1) + 1) if dbl else 2 * it
    flops_call = ne * n_prod * 8.0 * b ** 3

    def run(ctx):
        if dbl:
            ctx.obc_lyapunov_doubling(b, ne, da, b * b, dq, b * b, w, out, it)
        else:
            ctx.obc_lyapunov_fixed_point(b, ne, da, b * b, dq, b * b, w, out, it)

    with Q.Context(0, profile=not args.no_profile) as ctx:
        torch.cuda.synchronize()
        for _ in range(max(1, args.warmup)):
            run(ctx)
        torch.cuda.synchronize()
        ctx.reset_stats()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run(ctx)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        roof = None if args.no_profile else _gemm_roofline(
            ctx, "zgemm", FP64_MFMA_PEAK_TFLOPS,
            "zgemm_kernel (complex FP64, 3M form: 3 real MFMA per complex product)")
        if roof is not None:
            roof["traffic"] = None
    o = out.cpu().numpy()
    cpu = None
    if args.cpu_energies > 0:
        from oracle import obc_lyapunov_fixed_point, obc_lyapunov_doubling
        k = min(ne, max(args.cpu_energies, 32))
        idx = [int(i) for i in np.linspace(0, ne - 1, k).round()]
        t1 = time.perf_counter()
        for e in idx:
            if dbl:
                obc_lyapunov_doubling(a[e], q[e], it)
            else:
                obc_lyapunov_fixed_point(a[e], q[e], np.zeros((b, b), np.complex128), it)
        dc = time.perf_counter() - t1
        cpu = {"value": len(idx) / dc, "unit": "energy-points/s",
               "cores": os.cpu_count() or 1, "kind": "oracle",
               "sample": "%d of the %d energies (evenly spaced), %d %s each, NumPy/OpenBLAS, "
                         "%.1f s" % (len(idx), ne, it, "steps" if dbl else "iterations", dc)}
    res = {
        "mode": "obc", "metric": "W lesser/greater surface functions/s (energy-points/s) + "
                                 "% FP64 MFMA peak",
        "value": round(ne / dt, 3), "unit": "energy-points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Eq. lyapunov w = q - a w a^dagger by %d %s per call, b=%d, "
                               "%d energies, a ~ CN(0, 0.64/b), q anti-Hermitian"
                               % (it, "doubling steps (from scratch)" if dbl else
                                  "fixed-point iterations (memoized start)", b, ne),
                   "block_size": b, "n_energies": ne, "method": args.obc_method,
                   "iterations": it, "seed": args.seed},
        "tflops": round(flops_call / dt / 1e12, 3),
        "pct_fp64_mfma_peak": round(100 * flops_call / dt / 1e12 / FP64_MFMA_PEAK_TFLOPS, 2),
        "flops_per_call": flops_call,
        ("remaining_max" if dbl else "last_update_max"): float(o.max()),
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def run_obc(args):
    """Lead surface function (retarded OBC) in the memoized mode: every call
    runs a fixed number of fixed-point iterations over all energies, starting
    from the previous call's result, and returns x, n x n' and the update."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    from paper_2508_19138_amd import synth
    b, ne, it = args.block_size, args.energies, args.obc_iters
    E = synth.energy_grid(ne)
    m, n, np_ = synth.lead_blocks(args.seed, b, E, eta=0.05)
    dev = lambda a: torch.from_numpy(a).to("cuda:0")
    dm, dn, dnp = dev(m), dev(n), dev(np_)
    x = torch.zeros((ne, b, b), dtype=torch.complex128, device="cuda:0")
    sig = torch.empty_like(x)
    upd = torch.empty(ne, dtype=torch.float64, device="cuda:0")
    info = torch.zeros(ne, dtype=torch.int32, device="cuda:0")
    sancho = args.obc_method == "sancho"
    # fixed point: two products and one inverse per iteration; decimation:
    # six products and one inverse per step and one final inverse; both end
    # with the two products of n x n' (an inverse counts as 8 b^3)
    flops_call = ne * ((7 * it + 3) if sancho else (3 * it + 2)) * 8.0 * b ** 3

    def run(ctx):
        if sancho:
            ctx.obc_sancho_rubio(b, ne, dm, b * b, dn, 0, dnp, 0, x, sig, upd, info, it)
        else:
            ctx.obc_fixed_point(b, ne, dm, b * b, dn, 0, dnp, 0, x, sig, upd, info, it)

    with Q.Context(0, profile=not args.no_profile) as ctx:
        torch.cuda.synchronize()
        for _ in range(max(1, args.warmup)):        # also brings x near the solution
            run(ctx)
        torch.cuda.synchronize()
        ctx.reset_stats()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run(ctx)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        roof = None if args.no_profile else _gemm_roofline(
            ctx, "zgemm", FP64_MFMA_PEAK_TFLOPS,
            "zgemm_kernel (complex FP64, 3M form: 3 real MFMA per complex product)")
        if roof is not None:
            roof["traffic"] = None           # no counter run of this workload
        kt = None if args.no_profile else {
            k: round(ctx.kernel_stats(k)["ms"] / args.steps, 2)
            for k in ("zgemm", "inverse", "elementwise")}
        # lesser/greater boundary blocks from n x n' (HBM-bound); algorithmic
        # bytes: read the retarded block once, write the two outputs
        f_h, omf_h = synth.fermi(E), synth.one_minus_fermi(E)
        sl, sg = torch.empty_like(sig), torch.empty_like(sig)
        ctx.obc_lesser_greater(b, ne, sig, b * b, f_h, omf_h, sl, sg)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            ctx.obc_lesser_greater(b, ne, sig, b * b, f_h, omf_h, sl, sg)
        torch.cuda.synchronize()
        lg_s = (time.perf_counter() - t2) / args.steps
        lg_bytes = 3.0 * 16.0 * b * b * ne
    assert int(info.max().item()) == 0 and int(info.min().item()) == 0
    upd_h = upd.cpu().numpy()
    cpu = None
    if args.cpu_energies > 0:
        from oracle import obc_fixed_point, obc_sancho_rubio_steps
        # about 10 s of host work: evenly spaced energies, both ends included
        k = min(ne, max(args.cpu_energies, 20 if sancho else 48))
        idx = [int(i) for i in np.linspace(0, ne - 1, k).round()]
        x0 = np.zeros((b, b), np.complex128)
        t1 = time.perf_counter()
        for e in idx:
            if sancho:
                obc_sancho_rubio_steps(m[e], n, np_, it)
            else:
                obc_fixed_point(m[e], n, np_, x0, it)
        dc = time.perf_counter() - t1
        cpu = {"value": len(idx) / dc, "unit": "energy-points/s",
               "cores": os.cpu_count() or 1, "kind": "oracle",
               "sample": "%d of the %d energies (evenly spaced, both ends), %d iterations "
                         "each, NumPy/OpenBLAS, %.1f s" % (len(idx), ne, it, dc)}
    out = {
        "mode": "obc",
        "metric": "lead surface functions/s (energy-points/s) + % FP64 MFMA peak",
        "value": round(ne / dt, 3), "unit": "energy-points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "retarded OBC surface function x = (m - n x n')^-1 by %d "
                               "%s per call, b=%d, %d energies on [-2,2], eta 0.05, "
                               "shared couplings"
                               % (it, "Sancho-Rubio decimation steps (from scratch)" if sancho
                                  else "fixed-point iterations (memoized start)", b, ne),
                   "block_size": b, "n_energies": ne, "method": args.obc_method,
                   "iterations": it, "seed": args.seed},
        "tflops": round(flops_call / dt / 1e12, 3),
        "pct_fp64_mfma_peak": round(100 * flops_call / dt / 1e12 / FP64_MFMA_PEAK_TFLOPS, 2),
        "flops_per_call": flops_call,
        ("remaining_coupling_max" if sancho else "last_update_max"): float(upd_h.max()),
        ("remaining_coupling_median" if sancho else "last_update_median"):
            float(np.median(upd_h)),
        "roofline": roof, "kernel_time_ms_per_call": kt, "cpu_baseline": cpu,
        "lesser_greater": {"ms_per_call": round(lg_s * 1e3, 3),
                           "algorithmic_bytes": lg_bytes,
                           "GB_per_s": round(lg_bytes / lg_s / 1e9, 1),
                           "note": "host-timed call incl. launch; Sigma^< and Sigma^> for all "
                                   "energies"},
    }
    print(json.dumps(out), flush=True)


def run_observables(args):
    """Density of states, density and current per block from G^</G^> of the
    device-size shape (random contents: the reduction does not depend on
    them).  HBM-bound: reports GB/s on algorithmic bytes."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    n, b, ne = args.n_blocks, args.block_size, min(args.energies, 64)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(args.seed)
    mk = lambda *sh: torch.randn(sh, dtype=torch.complex128, device="cuda:0", generator=g)
    gl_d, gg_d, gl_l, hu = mk(ne, n, b, b), mk(ne, n, b, b), mk(ne, n - 1, b, b), mk(n - 1, b, b)
    dos = torch.empty((ne, n), dtype=torch.float64, device="cuda:0")
    dens = torch.empty_like(dos)
    cur = torch.empty((ne, n - 1), dtype=torch.float64, device="cuda:0")
    with Q.Context(0) as ctx:
        torch.cuda.synchronize()
        for _ in range(max(1, args.warmup)):
            ctx.observables(n, b, ne, gl_d, gg_d, gl_l, hu, dos, dens, cur)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.observables(n, b, ne, gl_d, gg_d, gl_l, hu, dos, dens, cur)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
    # per energy: the diagonals of G^<_ii and G^>_ii, every G^<_{i+1,i};
    # per call: H_{i,i+1} read and its adjoint written once
    by = ne * (2.0 * n * b * 16 + (n - 1) * b * b * 16.0) + 2.0 * (n - 1) * b * b * 16
    out = {"mode": "observables",
           "metric": "observables energy-points/s + HBM GB/s",
           "value": round(ne / dt, 2), "unit": "energy-points/s", "n_gpus": 1,
           "steps": args.steps, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "density of states, density (n blocks) and current (n-1 "
                                  "interfaces) per energy from G^</G^> blocks, %d blocks of "
                                  "%d, %d energies" % (n, b, ne), "n_blocks": n,
                      "block_size": b, "n_energies": ne},
           "roofline": {"bound": "hbm", "achieved": round(by / dt / 1e9, 1), "peak": 8000.0,
                        "unit": "GB/s", "frac": round(by / dt / 1e9 / 8000.0, 4),
                        "traffic": None, "algorithmic_bytes_per_call": by,
                        "note": "host-timed call (adjoint of H, then one reduction launch)"}}
    print(json.dumps(out), flush=True)


def run_convolution(args):
    """Element-wise energy convolution (Eq. interaction) of the diagonal
    blocks of a device: X2 = a descriptor on N energies, X1 = the other on
    the 2N - 1 energy differences, B on the N energies (every term inside
    X1's range).  Random contents; FP64 vector arithmetic."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    nb, b, N = args.conv_blocks, args.block_size, args.energies
    n_elem = nb * b * b
    g = torch.Generator(device="cuda:0")
    g.manual_seed(args.seed)
    X1 = torch.randn((2 * N - 1, n_elem), dtype=torch.complex128, device="cuda:0", generator=g)
    X2 = torch.randn((N, n_elem), dtype=torch.complex128, device="cuda:0", generator=g)
    B = torch.empty((N, n_elem), dtype=torch.complex128, device="cuda:0")
    s = 1j / (2 * np.pi)
    with Q.Context(0) as ctx:
        torch.cuda.synchronize()
        for _ in range(max(1, args.warmup)):
            ctx.energy_convolution(n_elem, X1, 2 * N - 1, X2, N, B, N, N - 1, s)
        ts = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            ctx.energy_convolution(n_elem, X1, 2 * N - 1, X2, N, B, N, N - 1, s)
            ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    flops = 8.0 * n_elem * N * N
    by = 16.0 * n_elem * (3 * N - 1 + N)
    # CPU baseline: the oracle on a bounded sample of the elements
    from oracle import energy_convolution
    m = 4096
    x1 = X1[:, :m].cpu().numpy()
    x2 = X2[:, :m].cpu().numpy()
    t0 = time.perf_counter()
    energy_convolution(x1, x2, N, N - 1, s)
    tc = time.perf_counter() - t0
    out = {"mode": "convolution",
           "metric": "element-wise energy convolutions: energy-points/s + % of FP64 vector peak",
           "value": round(N / dt, 2), "unit": "energy-points/s", "n_gpus": 1,
           "steps": args.steps, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "B(E_k) = s sum_k' X1(E_k - E_k') X2(E_k') element by element "
                                  "over %d blocks of %dx%d entries, %d energies, X1 on the %d "
                                  "energy differences" % (nb, b, b, N, 2 * N - 1),
                      "n_elem": n_elem, "n_energies": N},
           "roofline": {"bound": "alu", "achieved": round(flops / dt / 1e12, 3),
                        "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(flops / dt / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
                        "traffic": None, "algorithmic_flops_per_call": flops,
                        "algorithmic_bytes_per_call": by,
                        "note": "host-timed call; peak = the FP64 vector rate (equal to the "
                                "FP64 matrix rate on MI355X)"},
           "cpu_baseline": {"value": round(N * m / n_elem / tc, 4), "unit": "energy-points/s",
                            "cores": 1, "kind": "oracle",
                            "sample": "%d of the %d elements (all energies), scaled to the whole "
                                      "workload; NumPy, %.1f s" % (m, n_elem, tc)}}
    print(json.dumps(out), flush=True)


def run_nested(args):
    """Partitioned solve (qtx_rgf_solve_nested) of one long device at few
    energies, for several partition counts, against the plain solve of the
    same problem (the tests pin both against the oracle)."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    n, b, n_e = args.nested_blocks, args.block_size, args.nested_energies
    parts = [int(x) for x in args.partitions.split(",") if x]
    p, H, (sr, sl, sg) = build_inputs(n, b, n_e, args.seed)
    E = np.ascontiguousarray(p["energies"])
    mk = lambda: tuple(torch.empty((n_e, m, b, b), dtype=torch.complex128, device="cuda:0")
                       for m in (n, n - 1, n - 1))
    ref = (mk(), mk(), mk())
    out = (mk(), mk(), mk())
    torch.cuda.synchronize()
    flops_e = Q.flops_per_energy(Q.QTX_KIND_G, n, b, 2, False)

    def timed(call):
        for _ in range(max(1, args.warmup)):
            call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            call()
            ts.append(time.perf_counter() - t0)
        return ts

    rows = []
    with Q.Context(0) as ctx:
        plain = Q.make_g_problem(E, H, tuple(sr), tuple(sl), tuple(sg), *ref)
        tp = timed(lambda: ctx.solve_batch([plain]))
        assert plain.status == 0
        t_plain = float(np.median(tp))
        for P in parts:
            prob = Q.make_g_problem(E, H, tuple(sr), tuple(sl), tuple(sg), *out)
            t = float(np.median(timed(lambda: ctx.solve_nested(prob, P))))
            assert prob.status == 0, prob.status
            worst = 0.0
            for X, R in zip(out, ref):
                for x, r in zip(X, R):
                    d = torch.linalg.matrix_norm(x - r)
                    nr = torch.linalg.matrix_norm(r)
                    big = nr.max()
                    nr = torch.where(nr < 1e-13 * big, big, nr)
                    worst = max(worst, float((d / nr).max()))
            rows.append({"partitions": P, "ms_per_solve": round(t * 1e3, 2),
                         "speedup_vs_plain": round(t_plain / t, 3),
                         "energy_points_s": round(n_e / t, 3),
                         "tflops_on_plain_count": round(flops_e * n_e / t / 1e12, 2),
                         "max_block_rel_diff_vs_plain": worst})
    best = max(rows, key=lambda r: r["energy_points_s"]) if rows else None
    res = {"mode": "nested",
           "metric": "partitioned RGF energy-points/s vs the plain solve",
           "value": best["energy_points_s"] if best else None, "unit": "energy-points/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "one long device, G-type, %d blocks of %d, %d energies, "
                                  "block-diagonal Sigma, all nine outputs; partitions %s"
                                  % (n, b, n_e, parts),
                      "n_blocks": n, "block_size": b, "n_energies": n_e},
           "plain": {"ms_per_solve": round(t_plain * 1e3, 2),
                     "energy_points_s": round(n_e / t_plain, 3),
                     "tflops": round(flops_e * n_e / t_plain / 1e12, 2)},
           "partitioned": rows}
    print(json.dumps(res), flush=True)


def run_gemm(args):
    """Product kernel alone; HIP-event time per launch and algorithmic bytes."""
    import torch
    from paper_2508_19138_amd import qtx_rgf as Q
    b, batch = args.block_size, args.energies
    g = torch.Generator(device="cuda:0")
    g.manual_seed(args.seed)
    mk = lambda: torch.randn((batch, b, b), dtype=torch.complex128, device="cuda:0", generator=g)
    A, B, C = mk(), mk(), mk()
    D = torch.empty_like(C)
    torch.cuda.synchronize()
    rows = []
    with Q.Context(0, profile=True) as ctx:
        for opa, opb in (("N", "N"), ("N", "C"), ("C", "N"), ("C", "C")):
            ctx.zgemm(opa, opb, b, b, b, 1 + 0j, A, b, b * b, B, b, b * b, 1 + 0j, C, b, b * b,
                      D, b, b * b, batch)
            ctx.reset_stats()
            for _ in range(max(1, args.steps)):
                ctx.zgemm(opa, opb, b, b, b, 1 + 0j, A, b, b * b, B, b, b * b, 1 + 0j, C, b,
                          b * b, D, b, b * b, batch)
            st = ctx.kernel_stats("zgemm")
            ms = st["ms"] / st["launches"]
            rows.append({"op": opa + opb, "avg_launch_ms": round(ms, 4),
                         "tflops": round(st["flops"] / st["launches"] / (ms * 1e-3) / 1e12, 3),
                         "algorithmic_bytes_per_launch": st["bytes"] / st["launches"]})
    x = torch.empty(1 << 26, dtype=torch.complex128, device="cuda:0")   # 1 GiB
    x.fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "gemm", "block_size": b, "batch": batch, "products": rows,
                      "copy_calibration_bytes": 1 << 30}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU; --gpus %d is not supported "
              "(energies shard across GPUs with no exchange, see the design notes)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.mode == "plain":
        run_plain(args)
    elif args.mode == "mixed":
        run_plain(args, mixed=True)
    elif args.mode == "uneven":
        run_uneven(args)
    elif args.mode == "convolution":
        run_convolution(args)
    elif args.mode == "gemm":
        run_gemm(args)
    elif args.mode == "obc" and args.obc_method.startswith("lyap"):
        run_lyapunov(args)
    elif args.mode == "obc":
        run_obc(args)
    elif args.mode == "observables":
        run_observables(args)
    elif args.mode == "nested":
        run_nested(args)
    else:
        run_serve(args)


if __name__ == "__main__":
    main()
