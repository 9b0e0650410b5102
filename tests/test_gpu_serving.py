"""GPU tests of the request loop (qtx_rgf_submit / qtx_rgf_poll): problems
submitted one by one, some while others are already running, must each give
exactly the result of solving them alone with qtx_rgf_solve_batch, and that
result must match the CPU oracle (1e-10 per block); failures stay with their
problem; completions carry consistent timings."""

import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import assemble_g, assemble_w, rgf_selected  # noqa: E402
from paper_2508_19138_amd import synth  # noqa: E402
from paper_2508_19138_amd import qtx_rgf as Q  # noqa: E402
from blockcmp import triple_err  # noqa: E402
import gpu_helpers as G  # noqa: E402

TOL = 1e-10


class Job:
    """Device inputs/outputs and the Problem structure of one request."""

    def __init__(self, spec):
        self.spec = spec
        n, b, ne, seed = spec["n"], spec["b"], spec["ne"], spec["seed"]
        if spec["kind"] == "G":
            self.p = synth.g_problem(seed, n, b, n_e=ne)
        else:
            E = synth.energy_grid(ne)
            self.p = synth.w_problem(seed, n, b, E)
        self.alloc()

    def alloc(self):
        p, n, b, ne = self.p, self.spec["n"], self.spec["b"], self.spec["ne"]
        self.XR, self.XL, self.XG = (G.outputs(ne, n, b), G.outputs(ne, n, b),
                                     G.outputs(ne, n, b))
        for T in (self.XR, self.XL, self.XG):
            for t in T:
                t.fill_(complex(float("nan"), 0.0))
        if self.spec["kind"] == "G":
            self.E = np.ascontiguousarray(p["energies"])
            self.ins = ((G.dev(p["H"][0]), G.dev(p["H"][1]), G.dev(p["H"][2])),
                        tuple(G.dev(t) for t in p["sigma_r"]),
                        (G.dev(p["sigma_l"][0]), None, None),
                        (G.dev(p["sigma_g"][0]), None, None))
            self.prob = Q.make_g_problem(self.E, *self.ins, self.XR, self.XL, self.XG)
        else:
            self.ins = ((G.dev(p["V"][0]), G.dev(p["V"][1]), None),
                        tuple(G.dev(t) for t in p["P_r"]),
                        (G.dev(p["P_l"][0]), None, None),
                        (G.dev(p["P_g"][0]), None, None))
            self.prob = Q.make_w_problem(*self.ins, self.XR, self.XL, self.XG)
        torch.cuda.synchronize()          # fills done before the library's stream reads

    def results(self):
        torch.cuda.synchronize()
        return [G.host(T) for T in (self.XR, self.XL, self.XG)]

    def oracle_error(self):
        """Largest per-block error of the device results against the oracle
        over every energy and output."""
        p, n = self.p, self.spec["n"]
        got = self.results()
        adj = lambda T: np.conj(np.swapaxes(T, -1, -2))
        worst = 0.0
        for e in range(self.spec["ne"]):
            if self.spec["kind"] == "G":
                A = assemble_g(p["energies"][e], p["H"], (p["sigma_r"][0][e], None, None))
                z = np.zeros((n - 1,) + p["sigma_l"][0].shape[-2:], np.complex128)
                Bs = [(p["sigma_l"][0][e], z, z), (p["sigma_g"][0][e], z, z)]
            else:
                at = lambda T: tuple(t[e] for t in T)
                A, Bs = assemble_w(p["V"], at(p["P_r"]), [at(p["P_l"]), at(p["P_g"])])
            OR, (OL, OG) = rgf_selected(A, Bs)
            for X, R in zip(got, (OR, OL, OG)):
                worst = max(worst, triple_err(tuple(t[e] for t in X), R))
        return worst


def _specs(seed, count, bs=(16, 40, 64, 96), ns=(1, 9), ne=(1, 6)):
    rng = np.random.default_rng(seed)
    out = []
    for s in synth.uneven_specs(seed, count, block_sizes=bs, n_range=ns):
        out.append({"kind": s["kind"], "n": s["n"], "b": s["b"], "seed": s["seed"],
                    "ne": int(rng.integers(ne[0], ne[1] + 1))})
    return out


def _alone(jobs):
    with Q.Context(0) as ctx:
        ref = []
        for j in jobs:
            assert ctx.solve_batch([j.prob]) == Q.QTX_OK, j.spec
            ref.append(j.results())
    return ref


def _equal(a, b, what):
    for X, Y in zip(a, b):
        for x, y in zip(X, Y):
            assert np.array_equal(x, y), what


def _drain(ctx, want, timeout_s=60.0):
    done = {}
    t0 = time.time()
    while len(done) < want:
        cs, pend = ctx.poll(cap=16, wait_ms=200)
        for c in cs:
            assert c["ticket"] not in done
            done[c["ticket"]] = c
        assert time.time() - t0 < timeout_s, "request loop did not finish"
        if not cs and pend == 0:
            break
    return done


def test_served_requests_equal_alone():
    jobs = [Job(s) for s in _specs(21, 12)]
    assert {j.spec["kind"] for j in jobs} == {"G", "W"}
    ref = _alone(jobs)
    for j in jobs:
        j.alloc()
    with Q.Context(0) as ctx:
        tickets = {}
        half = len(jobs) // 2
        for j in jobs[:half]:
            tickets[ctx.submit(j.prob)] = j
        first, _ = ctx.poll(cap=1, wait_ms=-1)      # some work has completed
        for j in jobs[half:]:                       # arrivals while others run
            tickets[ctx.submit(j.prob)] = j
        done = _drain(ctx, len(jobs) - len(first))
        for c in first:
            done[c["ticket"]] = c
        assert sorted(done) == sorted(tickets)
        for t, c in done.items():
            assert c["status"] == Q.QTX_OK, (tickets[t].spec, c)
            assert c["n_energies"] == tickets[t].spec["ne"]
            assert 0.0 <= c["queue_s"] <= c["latency_s"]
        cs, pend = ctx.poll(cap=4, wait_ms=0)
        assert cs == [] and pend == 0
    for j, r in zip(jobs, ref):
        _equal(j.results(), r, j.spec)
        assert j.oracle_error() < TOL, j.spec


def test_served_admission_into_small_workspace():
    """A workspace that holds a few lanes: later requests wait for memory in
    arrival order, energy chunks are admitted as others finish."""
    jobs = [Job(s) for s in _specs(22, 8, bs=(32, 64), ns=(3, 10), ne=(2, 8))]
    ref = _alone(jobs)
    for j in jobs:
        j.alloc()
    with Q.Context(0, budget_bytes=6 * 1024 * 1024) as ctx:
        tickets = [ctx.submit(j.prob) for j in jobs]
        done = _drain(ctx, len(jobs))
        assert sorted(done) == sorted(tickets)
        assert all(c["status"] == Q.QTX_OK for c in done.values())
    for j, r in zip(jobs, ref):
        _equal(j.results(), r, j.spec)
        assert j.oracle_error() < TOL, j.spec


def test_served_failure_stays_with_its_request():
    n, b = 4, 16
    good = Job({"kind": "G", "n": n, "b": b, "ne": 2, "seed": 31})
    bad = Job({"kind": "G", "n": n, "b": b, "ne": 2, "seed": 32})
    p = bad.p
    E1 = p["energies"][1]
    K = np.zeros((b, b), np.complex128)
    K[:, 1:] = synth.cn(np.random.default_rng(2), (b, b - 1), 1.0)
    d = p["H"][0].copy()
    d[2] = E1 * np.eye(b) - p["sigma_r"][0][1][2] - K
    p["H"] = (d, np.zeros_like(p["H"][1]), np.zeros_like(p["H"][2]))
    bad.alloc()
    ref = _alone([good])
    good.alloc()
    with Q.Context(0) as ctx:
        tg = ctx.submit(good.prob)
        tb = ctx.submit(bad.prob)
        done = _drain(ctx, 2)
    assert done[tg]["status"] == Q.QTX_OK
    assert done[tb]["status"] == Q.QTX_ERR_SINGULAR
    assert done[tb]["fail_energy"] == 1 and done[tb]["fail_block"] == 2
    _equal(good.results(), ref[0], "good")


def test_submit_checks_and_empty_poll():
    j = Job({"kind": "G", "n": 3, "b": 8, "ne": 1, "seed": 1})
    with Q.Context(0) as ctx:
        cs, pend = ctx.poll(cap=4, wait_ms=0)
        assert cs == [] and pend == 0
        bad = Q.make_g_problem(j.E, *j.ins, j.XR, j.XL, j.XG)
        bad.block_size = 0
        with pytest.raises(Q.QtxError) as ei:
            ctx.submit(bad)
        assert ei.value.status == Q.QTX_ERR_INVALID_ARG
    with Q.Context(0, budget_bytes=64 * 1024) as ctx:
        big = Job({"kind": "G", "n": 8, "b": 64, "ne": 1, "seed": 3})
        with pytest.raises(Q.QtxError) as ei:
            ctx.submit(big.prob)
        assert ei.value.status == Q.QTX_ERR_NOMEM


def test_close_drains_outstanding_requests():
    jobs = [Job(s) for s in _specs(23, 5, bs=(32, 48), ns=(2, 6))]
    ref = _alone(jobs)
    for j in jobs:
        j.alloc()
    ctx = Q.Context(0)
    for j in jobs:
        ctx.submit(j.prob)
    ctx.close()                                   # without polling
    for j, r in zip(jobs, ref):
        _equal(j.results(), r, j.spec)


def test_served_mixed_precision_and_wr_equal_alone():
    """Requests with options: FP32 matrix-core products, and a W-type
    request that also asks for W^R diagonal blocks."""
    n, b, ne = 5, 48, 3
    pg = synth.g_problem(41, n, b, n_e=ne)
    pw = synth.w_problem(42, n, b, synth.energy_grid(ne))

    def make():
        E = np.ascontiguousarray(pg["energies"])
        g_in = ((G.dev(pg["H"][0]), G.dev(pg["H"][1]), None),
                (G.dev(pg["sigma_r"][0]), None, None),
                (G.dev(pg["sigma_l"][0]), None, None),
                (G.dev(pg["sigma_g"][0]), None, None))
        g_out = (G.outputs(ne, n, b), G.outputs(ne, n, b), G.outputs(ne, n, b))
        w_in = ((G.dev(pw["V"][0]), G.dev(pw["V"][1]), None),
                tuple(G.dev(t) for t in pw["P_r"]),
                (G.dev(pw["P_l"][0]), None, None),
                (G.dev(pw["P_g"][0]), None, None))
        w_out = (G.outputs(ne, n, b), G.outputs(ne, n, b), G.outputs(ne, n, b))
        wr = G.empty((ne, n, b, b))
        probs = [Q.make_g_problem(E, *g_in, *g_out, precision=Q.QTX_MIXED),
                 Q.make_w_problem(*w_in, *w_out, WR_diag=wr)]
        torch.cuda.synchronize()
        return probs, (E, g_in, w_in), [g_out, w_out, wr]

    def host(outs):
        torch.cuda.synchronize()
        g_out, w_out, wr = outs
        return [G.host(T) for T in g_out + w_out] + [wr.cpu().numpy()]

    with Q.Context(0) as ctx:
        probs, keep, outs = make()
        for pr in probs:
            assert ctx.solve_batch([pr]) == Q.QTX_OK
        ref = host(outs)
        probs, keep2, outs2 = make()
        tickets = [ctx.submit(pr) for pr in probs]
        done = _drain(ctx, len(tickets))
        assert all(done[t]["status"] == Q.QTX_OK for t in tickets)
        got = host(outs2)
    for a, r in zip(got[:-1], ref[:-1]):
        for x, y in zip(a, r):
            assert np.array_equal(x, y)
    assert np.array_equal(got[-1], ref[-1])
