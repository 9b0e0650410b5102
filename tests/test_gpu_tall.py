"""Block sizes above 1024: the inverse's tournament path (each chunk of 768
rows proposes the rows its own elimination pivots on, one workgroup picks
the panel's pivot rows among them, every row then follows from the pivot
block's inverse).  The batched inverse against numpy for random, structured
and graded matrices, singular and non-finite columns past the first 1024,
and against the oracle at the FP64 bound (Sec. 3.2.3 recursion; Eq.
system-solve definition): G-type solves at b = 1100 and at the NW-2 block
size 2016 (Table tab:structure_param), a W-type solve with W^R at b = 1040,
and the partitioned solve (Sec. 4.4) at b = 1100."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import rgf_selected, assemble_g  # noqa: E402
from paper_2508_19138_amd import synth  # noqa: E402
from paper_2508_19138_amd import qtx_rgf as Q  # noqa: E402
from blockcmp import triple_err  # noqa: E402

TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = Q.Context(0)
    yield c
    c.close()


def _gh():
    import gpu_helpers
    return gpu_helpers


def _matrix(b, kind, rng):
    if kind == "random":
        return synth.cn(rng, (b, b), 1.0 / b) + 0.5 * np.eye(b)
    if kind == "zero_lead":
        # the first column's only entry sits in the second chunk: every other
        # chunk meets an all-zero column and proposes nothing for it
        M = synth.cn(rng, (b, b), 1.0 / b)
        M[:, 0] = 0.0
        M[b - 3, 0] = 1.0
        return M
    if kind == "perm_identity":
        P = np.eye(b, dtype=np.complex128)[rng.permutation(b)]
        return P * (1.0 - 0.25j)
    if kind == "graded":
        M = synth.cn(rng, (b, b), 1.0) + 2 * np.eye(b)
        return M * (10.0 ** (-np.arange(b) * 6.0 / (b - 1)))[:, None]
    raise ValueError(kind)


def _close(X, A, b):
    """The inverse's relative error within the rounding bound used for every
    inverse test (1e-15 * cond_1 * b)."""
    ref = np.linalg.inv(A)
    cond = np.linalg.norm(A, 1) * np.linalg.norm(ref, 1)
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    return err < 1e-15 * cond * b + 1e-13, (err, cond)


def _zinv(ctx, A):
    gh = _gh()
    batch, b = A.shape[0], A.shape[1]
    dA = gh.dev(A)
    dX = gh.empty((batch, b, b))
    info = torch.zeros(batch, dtype=torch.int32, device=gh.DEV)
    print("zinv b %d batch %d" % (b, batch), flush=True)
    ctx.zinv(b, dA, dX, info, batch)
    torch.cuda.synchronize()
    return dX.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("b", [1025, 1300, 2016, 2305])
@pytest.mark.parametrize("kind", ["random", "zero_lead", "perm_identity", "graded"])
def test_tall_zinv_matches_numpy(ctx, b, kind):
    rng = np.random.default_rng(b * 7 + len(kind))
    A = np.stack([_matrix(b, kind, rng) for _ in range(2)])
    X, info = _zinv(ctx, A)
    assert np.all(info == 0), info
    for e in range(2):
        ok, why = _close(X[e], A[e], b)
        assert ok, (e, why)


def test_tall_zinv_singular_column_past_1024(ctx):
    """An exactly zero column at 1100: every chunk and the final step meet
    only zeros there, so the status names that column; the other matrix of
    the batch is unaffected."""
    b = 1300
    rng = np.random.default_rng(5)
    A = np.stack([_matrix(b, "random", rng) for _ in range(2)])
    A[1][:, 1100] = 0.0
    X, info = _zinv(ctx, A)
    assert info[0] == 0
    assert info[1] == 1 + 1100
    ok, why = _close(X[0], A[0], b)
    assert ok, why


def test_tall_zinv_non_finite_entry(ctx):
    b = 1300
    rng = np.random.default_rng(6)
    A = np.stack([_matrix(b, "random", rng) for _ in range(2)])
    A[0][5, 1200] = np.nan
    X, info = _zinv(ctx, A)
    assert info[0] < 0
    assert info[1] == 0
    ok, why = _close(X[1], A[1], b)
    assert ok, why


def _oracle_g(p, e):
    E = p["energies"][e]
    sr = tuple(None if t is None else t[e] for t in p["sigma_r"])
    A = assemble_g(E, p["H"], sr)
    adj = lambda T: np.conj(np.swapaxes(T, -1, -2))
    Bs = []
    for key in ("sigma_l", "sigma_g"):
        d, u, _ = (t[e] for t in p[key])
        Bs.append((d, u, -adj(u)))
    return rgf_selected(A, Bs)


def _sel(T, e):
    return tuple(None if t is None else t[e] for t in T)


@pytest.mark.parametrize("n,b,bt", [(3, 1100, True), (2, 2016, False)])
def test_tall_block_solve_matches_oracle(ctx, n, b, bt):
    gh = _gh()
    p = synth.g_problem(300 + b, n, b, n_e=1, bt_sigma=bt)
    print("solve n %d b %d" % (n, b), flush=True)
    prob, XR, XL, XG = gh.solve_g(ctx, p)
    assert prob.status == 0
    OR, (OL, OG) = _oracle_g(p, 0)
    assert triple_err(_sel(XR, 0), OR) < TOL
    assert triple_err(_sel(XL, 0), OL) < TOL
    assert triple_err(_sel(XG, 0), OG) < TOL


def test_tall_block_w_type_solve(ctx):
    """W-type (I - V P^R) at b = 1040: the assembly products, the solve and
    W^R_ii on the tournament path."""
    from oracle import assemble_w, w_retarded_diag
    gh = _gh()
    n, b = 2, 1040
    E = np.array([0.7])
    p = synth.w_problem(17, n, b, E)
    V = (gh.dev(p["V"][0]), gh.dev(p["V"][1]), None)
    Pr = tuple(gh.dev(t) for t in p["P_r"])
    Pl = (gh.dev(p["P_l"][0]), gh.dev(p["P_l"][1]), None)
    Pg = (gh.dev(p["P_g"][0]), gh.dev(p["P_g"][1]), None)
    XR, XL, XG = gh.outputs(1, n, b), gh.outputs(1, n, b), gh.outputs(1, n, b)
    WR = gh.empty((1, n, b, b))
    prob = Q.make_w_problem(V, Pr, Pl, Pg, XR, XL, XG, WR)
    torch.cuda.synchronize()
    print("W solve n %d b %d" % (n, b), flush=True)
    ctx.solve_batch([prob])
    torch.cuda.synchronize()
    assert prob.status == 0
    A, Bs = assemble_w(p["V"], tuple(t[0] for t in p["P_r"]),
                       [tuple(t[0] for t in p["P_l"]), tuple(t[0] for t in p["P_g"])])
    OR, (OL, OG) = rgf_selected(A, Bs)
    for got, ref in ((gh.host(XR), OR), (gh.host(XL), OL), (gh.host(XG), OG)):
        assert triple_err(_sel(got, 0), ref) < TOL
    from blockcmp import max_rel_err
    assert max_rel_err(WR.cpu().numpy()[0], w_retarded_diag(OR, p["V"])) < TOL


def test_tall_block_partitioned_solve(ctx):
    """The partitioned solve (Sec. 4.4) at b = 1100: 5 blocks in 2
    partitions, one energy, against the oracle."""
    gh = _gh()
    n, b, P = 5, 1100, 2
    p = synth.g_problem(5, n, b, n_e=1)
    E = np.ascontiguousarray(p["energies"], dtype=np.float64)
    H = tuple(gh.dev(t) for t in p["H"])
    sr = tuple(gh.dev(t) for t in p["sigma_r"])
    sl = (gh.dev(p["sigma_l"][0]), gh.dev(p["sigma_l"][1]), None)
    sg = (gh.dev(p["sigma_g"][0]), gh.dev(p["sigma_g"][1]), None)
    XR, XL, XG = gh.outputs(1, n, b), gh.outputs(1, n, b), gh.outputs(1, n, b)
    prob = Q.make_g_problem(E, H, sr, sl, sg, XR, XL, XG)
    torch.cuda.synchronize()
    print("nested solve n %d b %d P %d" % (n, b, P), flush=True)
    ctx.solve_nested(prob, P)
    torch.cuda.synchronize()
    assert prob.status == 0
    OR, (OL, OG) = _oracle_g(p, 0)
    assert triple_err(_sel(gh.host(XR), 0), OR) < TOL
    assert triple_err(_sel(gh.host(XL), 0), OL) < TOL
    assert triple_err(_sel(gh.host(XG), 0), OG) < TOL
