"""GPU tests of the batched runtime: independent solves of different block
size, block count and kind share merged launches; each result must be the
same alone and in the mix, agree with the oracle, survive graph replay and
admission of lanes into a workspace smaller than the batch."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import rgf_selected, assemble_g, assemble_w  # noqa: E402
from paper_2508_19138_amd import synth  # noqa: E402
from paper_2508_19138_amd import qtx_rgf as Q  # noqa: E402
from blockcmp import triple_err  # noqa: E402
import gpu_helpers as G  # noqa: E402

TOL = 1e-10


def _adj(T):
    return np.conj(np.swapaxes(T, -1, -2))


class Solve:
    """Inputs, outputs and the Problem structure of one solve on the GPU."""

    def __init__(self, spec, precision=Q.QTX_FP64):
        self.spec = spec
        n, b = spec["n"], spec["b"]
        E = np.array([spec["E"]])
        if spec["kind"] == "G":
            self.p = synth.g_problem(spec["seed"], n, b, energies=E)
        else:
            self.p = synth.w_problem(spec["seed"], n, b, E)
        self.precision = precision

    def problem(self):
        p, n, b = self.p, self.spec["n"], self.spec["b"]
        self.XR, self.XL, self.XG = G.outputs(1, n, b), G.outputs(1, n, b), G.outputs(1, n, b)
        if self.spec["kind"] == "G":
            self.E = np.ascontiguousarray(p["energies"])
            self.ins = ((G.dev(p["H"][0]), G.dev(p["H"][1]), G.dev(p["H"][2])),
                        tuple(G.dev(t) for t in p["sigma_r"]),
                        (G.dev(p["sigma_l"][0]), None, None),
                        (G.dev(p["sigma_g"][0]), None, None))
            return Q.make_g_problem(self.E, *self.ins, self.XR, self.XL, self.XG,
                                    precision=self.precision)
        self.ins = ((G.dev(p["V"][0]), G.dev(p["V"][1]), None),
                    tuple(G.dev(t) for t in p["P_r"]),
                    (G.dev(p["P_l"][0]), None, None),
                    (G.dev(p["P_g"][0]), None, None))
        return Q.make_w_problem(*self.ins, self.XR, self.XL, self.XG, precision=self.precision)

    def results(self):
        return [G.host(T) for T in (self.XR, self.XL, self.XG)]

    def oracle(self):
        p = self.p
        if self.spec["kind"] == "G":
            A = assemble_g(p["energies"][0], p["H"], (p["sigma_r"][0][0], None, None))
            Bs = [(p["sigma_l"][0][0], p["sigma_l"][1][0], -_adj(p["sigma_l"][1][0])),
                  (p["sigma_g"][0][0], p["sigma_g"][1][0], -_adj(p["sigma_g"][1][0]))]
        else:
            A, Bs = assemble_w(p["V"], tuple(t[0] for t in p["P_r"]),
                               [tuple(t[0] for t in p["P_l"]), tuple(t[0] for t in p["P_g"])])
        XR, XS = rgf_selected(A, Bs)
        return [XR] + list(XS)


def _specs(seed, count, bs=(16, 40, 64, 96), ns=(1, 9)):
    return synth.uneven_specs(seed, count, block_sizes=bs, n_range=ns)


def _first(T):
    return tuple(t[0] for t in T)


def test_mixed_batch_equals_alone_and_oracle():
    specs = _specs(11, 10)
    assert {s["kind"] for s in specs} == {"G", "W"}
    solves = [Solve(s) for s in specs]
    with Q.Context(0) as ctx:
        probs = [s.problem() for s in solves]
        assert ctx.solve_batch(probs) == Q.QTX_OK
        mixed = [s.results() for s in solves]
        alone = []
        for s in solves:
            pr = s.problem()
            assert ctx.solve_batch([pr]) == Q.QTX_OK
            alone.append(s.results())
    for s, m, a in zip(solves, mixed, alone):
        for X, Y in zip(m, a):
            for x, y in zip(X, Y):
                assert np.array_equal(x, y), s.spec        # tiles depend on b only
        for X, R in zip(m, s.oracle()):
            assert triple_err(_first(X), R) < TOL, s.spec


def test_graph_replay_matches_eager():
    """The same batch is solved repeatedly: the second call is captured as a
    graph and later calls replay it; eager work and synchronisation happen
    between replays, and every replay must reproduce the first result."""
    specs = _specs(12, 6, bs=(24, 48), ns=(2, 5))
    solves = [Solve(s) for s in specs]
    with Q.Context(0) as ctx:
        probs = [s.problem() for s in solves]
        ctx.solve_batch(probs)
        ref = [s.results() for s in solves]
        for rep in range(4):
            for s in solves:                          # scribble on the outputs
                for T in (s.XR, s.XL, s.XG):
                    for t in T:
                        t.fill_(complex(float("nan"), 0.0))
            junk = torch.randn(256, 256, dtype=torch.float64, device=G.DEV)
            (junk @ junk).sum().item()                # eager work in between
            torch.cuda.synchronize()
            assert ctx.solve_batch(probs) == Q.QTX_OK
            for s, r in zip(solves, ref):
                for X, Y in zip(s.results(), r):
                    for x, y in zip(X, Y):
                        assert np.array_equal(x, y), (rep, s.spec)


def test_admission_into_small_workspace():
    """A budget that holds only a few lanes: lanes wait for memory and are
    admitted as others finish; results are those of an unconstrained run."""
    specs = _specs(13, 12, bs=(32, 64), ns=(3, 12))
    solves = [Solve(s) for s in specs]
    with Q.Context(0) as ctx:
        probs = [s.problem() for s in solves]
        ctx.solve_batch(probs)
        ref = [s.results() for s in solves]
    budget = 6 * 1024 * 1024
    with Q.Context(0, budget_bytes=budget) as ctx:
        probs = [s.problem() for s in solves]
        assert ctx.solve_batch(probs) == Q.QTX_OK
        for s, r in zip(solves, ref):
            for X, Y in zip(s.results(), r):
                for x, y in zip(X, Y):
                    assert np.array_equal(x, y), s.spec


def test_one_energy_over_budget_is_nomem():
    s = Solve({"kind": "G", "b": 64, "n": 8, "E": 0.1, "seed": 3})
    with Q.Context(0, budget_bytes=64 * 1024) as ctx:
        with pytest.raises(Q.QtxError) as ei:
            ctx.solve_batch([s.problem()])
        assert ei.value.status == Q.QTX_ERR_NOMEM


def test_stream_pool_is_bitwise_neutral(monkeypatch):
    """The same mixed batch on one stream and on the default pool of
    streams (lanes grouped by class, launches split differently) gives the
    same bits."""
    specs = _specs(14, 10, bs=(16, 40, 64, 96), ns=(2, 9))
    solves = [Solve(s) for s in specs]
    out = {}
    for n in ("1", "4"):
        monkeypatch.setenv("QTX_STREAMS", n)
        with Q.Context(0) as ctx:
            probs = [s.problem() for s in solves]
            torch.cuda.synchronize()
            assert ctx.solve_batch(probs) == Q.QTX_OK
            out[n] = [s.results() for s in solves]
    for s, a, b in zip(solves, out["1"], out["4"]):
        for X, Y in zip(a, b):
            for x, y in zip(X, Y):
                assert np.array_equal(x, y), s.spec
