"""Block sizes up to 128: the inverse done whole by one workgroup per matrix
in one launch (columns eliminated one by one with partial pivoting, the
matrix held in registers).  The batched inverse against numpy at sizes on
either side of its 64- and 128-row forms (and 129, the first size of the
blocked path), the exact status of a zero and of a non-finite column, bits
that do not depend on the batch, and RGF solves at b = 128 against the
oracle, G-type and W-type with W^R (Sec. 3.2.3 recursion; Eq. system-solve
definition)."""

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
        # column 0 has one nonzero entry, in the last rows: the first pivot
        # is far from the diagonal
        M = synth.cn(rng, (b, b), 1.0 / b)
        M[:, 0] = 0.0
        M[b - 1, 0] = 1.0
        return M
    if kind == "perm_identity":
        P = np.eye(b, dtype=np.complex128)[rng.permutation(b)]
        return P * (1.0 - 0.25j)
    if kind == "graded":
        M = synth.cn(rng, (b, b), 1.0) + 2 * np.eye(b)
        return M * (10.0 ** (-np.arange(b) * 6.0 / max(b - 1, 1)))[:, None]
    raise ValueError(kind)


def _close(X, A, b):
    """Relative error of the inverse within 1e-15 * cond_1 * b (+1e-13)."""
    ref = np.linalg.inv(A)
    cond = np.linalg.norm(A, 1) * np.linalg.norm(ref, 1)
    err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
    return err < 1e-15 * cond * b + 1e-13, (err, cond)


def _zinv(ctx, A):
    gh = _gh()
    batch, b = A.shape[0], A.shape[1]
    dA = gh.dev(A)
    dX = gh.empty((batch, b, b))
    info = torch.full((batch,), 7, dtype=torch.int32, device=gh.DEV)
    print("zinv b %d batch %d" % (b, batch), flush=True)
    ctx.zinv(b, dA, dX, info, batch)
    torch.cuda.synchronize()
    return dX.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("b", [2, 15, 16, 17, 33, 63, 64, 65, 96, 127, 128, 129])
@pytest.mark.parametrize("kind", ["random", "zero_lead", "perm_identity", "graded"])
def test_small_zinv_matches_numpy(ctx, b, kind):
    rng = np.random.default_rng(b * 11 + len(kind))
    A = np.stack([_matrix(b, kind, rng) for _ in range(3)])
    X, info = _zinv(ctx, A)
    assert np.all(info == 0), info                     # the status is reset
    for e in range(3):
        ok, why = _close(X[e], A[e], b)
        assert ok, (e, why)


@pytest.mark.parametrize("b,col", [(40, 23), (100, 77), (128, 127)])
def test_small_zinv_zero_column_status(ctx, b, col):
    """An exactly zero column: its search meets only zero candidates, so the
    status is +(1 + column); the other matrices are unaffected."""
    rng = np.random.default_rng(b + col)
    A = np.stack([_matrix(b, "random", rng) for _ in range(3)])
    A[1][:, col] = 0.0
    X, info = _zinv(ctx, A)
    assert info[0] == 0 and info[2] == 0
    assert info[1] == 1 + col
    for e in (0, 2):
        ok, why = _close(X[e], A[e], b)
        assert ok, (e, why)


@pytest.mark.parametrize("b", [50, 100])
def test_small_zinv_non_finite_entry(ctx, b):
    """A NaN at (5, 30): columns before 30 are eliminated normally and
    column 30 meets a non-finite candidate (row 5 itself, or every row once
    row 5 has been a pivot row), so the status is -(1 + 30)."""
    rng = np.random.default_rng(b)
    A = np.stack([_matrix(b, "random", rng) for _ in range(2)])
    A[0][5, 30] = np.nan
    X, info = _zinv(ctx, A)
    assert info[0] == -31
    assert info[1] == 0
    ok, why = _close(X[1], A[1], b)
    assert ok, why


@pytest.mark.parametrize("b", [37, 128])
def test_small_zinv_bits_do_not_depend_on_batch(ctx, b):
    rng = np.random.default_rng(3 * b)
    A = np.stack([_matrix(b, "random", rng) for _ in range(6)])
    X6, i6 = _zinv(ctx, A)
    X1, i1 = _zinv(ctx, A[4:5])
    assert i6[4] == 0 and i1[0] == 0
    assert np.array_equal(X6[4].view(np.float64), X1[0].view(np.float64))


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


@pytest.mark.parametrize("n,b,n_e,bt", [(5, 128, 3, True), (4, 64, 2, False), (3, 90, 1, True)])
def test_small_block_solve_matches_oracle(ctx, n, b, n_e, bt):
    gh = _gh()
    p = synth.g_problem(700 + b, n, b, n_e=n_e, bt_sigma=bt)
    print("solve n %d b %d energies %d" % (n, b, n_e), flush=True)
    prob, XR, XL, XG = gh.solve_g(ctx, p)
    assert prob.status == 0
    for e in range(n_e):
        OR, (OL, OG) = _oracle_g(p, e)
        for got, ref in ((XR, OR), (XL, OL), (XG, OG)):
            sel = tuple(None if t is None else t[e] for t in got)
            err = triple_err(sel, ref)
            assert err < TOL, (e, err)


def test_small_block_w_type_solve(ctx):
    """W-type (I - V P^R) at b = 128, with W^R_ii: the assembly products, the
    solve on the one-launch inverse and the retarded screened interaction."""
    from oracle import assemble_w, w_retarded_diag
    from blockcmp import max_rel_err
    gh = _gh()
    n, b = 4, 128
    E = np.array([0.4, -0.9])
    p = synth.w_problem(31, n, b, E)
    V = (gh.dev(p["V"][0]), gh.dev(p["V"][1]), None)
    Pr = tuple(gh.dev(t) for t in p["P_r"])
    Pl = (gh.dev(p["P_l"][0]), gh.dev(p["P_l"][1]), None)
    Pg = (gh.dev(p["P_g"][0]), gh.dev(p["P_g"][1]), None)
    n_e = E.shape[0]
    XR, XL, XG = gh.outputs(n_e, n, b), gh.outputs(n_e, n, b), gh.outputs(n_e, n, b)
    WR = gh.empty((n_e, n, b, b))
    prob = Q.make_w_problem(V, Pr, Pl, Pg, XR, XL, XG, WR)
    torch.cuda.synchronize()
    print("W solve n %d b %d energies %d" % (n, b, n_e), flush=True)
    ctx.solve_batch([prob])
    torch.cuda.synchronize()
    assert prob.status == 0
    hR, hL, hG = gh.host(XR), gh.host(XL), gh.host(XG)
    for e in range(n_e):
        A, Bs = assemble_w(p["V"], tuple(t[e] for t in p["P_r"]),
                           [tuple(t[e] for t in p["P_l"]), tuple(t[e] for t in p["P_g"])])
        OR, (OL, OG) = rgf_selected(A, Bs)
        for got, ref in ((hR, OR), (hL, OL), (hG, OG)):
            sel = tuple(None if t is None else t[e] for t in got)
            assert triple_err(sel, ref) < TOL, e
        assert max_rel_err(WR.cpu().numpy()[e], w_retarded_diag(OR, p["V"])) < TOL
