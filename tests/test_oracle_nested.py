"""Pins of the nested-dissection oracle (Sec. 4.4, partitioned solver).

* The selected blocks of X^R and of X^s = A^{-1} B A^{-dagger} equal the
  dense definition (Eq. system-solve) for general non-symmetric
  block-tridiagonal A and B, for 2..5 partitions, block sizes 1 to 3, and
  uneven partition sizes.
* The reduced right-hand side is what the separators see: X^s_SS =
  S^{-1} B~ S^{-dagger} equals the separator block of the dense X^s, and B~
  is block tridiagonal in separator order like S.
* The reduced system has the structure the scheme predicts: block
  tridiagonal in separator order, where the two separators of a middle
  partition are coupled only through fill-in (they are not neighbours in A),
  and it equals the inverse of the separator-restricted block of A^{-1}.
* The block form (each partition's elimination with fill-in, as one device
  would run it) gives the same selected blocks as the dense definition and
  the same reduced system and right-hand sides, including middle
  partitions of two blocks (no interior) and block size 1.
"""

import numpy as np
import pytest

from oracle import dense_selected
from oracle.nested import (nested_dissection_blocks, nested_dissection_selected, partitions,
                           separators)
from paper_2508_19138_amd import synth


def _bt(seed, n, b):
    rng = np.random.default_rng(seed)
    d = synth.cn(rng, (n, b, b), 1.0) + 4.0 * np.eye(b)
    u = synth.cn(rng, (n - 1, b, b), 1.0)
    l = synth.cn(rng, (n - 1, b, b), 1.0)
    return d, u, l


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,b,P", [(6, 1, 2), (7, 3, 2), (9, 3, 3), (11, 2, 4), (13, 3, 5),
                                   (10, 1, 3)])
def test_selected_blocks_match_dense(n, b, P):
    Mt = _bt(100 * n + P, n, b)
    Bs = [_bt(100 * n + P + 1, n, b), _bt(100 * n + P + 2, n, b)]
    r = nested_dissection_selected(Mt, P, Bs)
    refR, refS = dense_selected(Mt, Bs)
    for k in range(3):
        assert _rel(r["XR"][k], refR[k]) < 1e-12
        for s in range(2):
            assert _rel(r["XS"][s][k], refS[s][k]) < 1e-12


def test_partitions_and_separators():
    assert partitions(10, 3) == [(0, 4), (4, 7), (7, 10)]
    assert separators(10, 3) == [3, 4, 6, 7]
    assert separators(6, 2) == [2, 3]
    with pytest.raises(ValueError):
        partitions(4, 3)          # a middle partition needs two blocks
    with pytest.raises(ValueError):
        partitions(5, 1)


def test_reduced_system_structure_and_schur_identity():
    n, b, P = 12, 2, 4
    Mt = _bt(5, n, b)
    B = _bt(6, n, b)
    r = nested_dissection_selected(Mt, P, [B])
    S, sep, BS = r["S"], r["sep"], r["BS"][0]
    m = len(sep)
    Sb = lambda i, j: S[i * b:(i + 1) * b, j * b:(j + 1) * b]
    # block tridiagonal in separator order
    for i in range(m):
        for j in range(m):
            if abs(i - j) > 1:
                assert np.all(Sb(i, j) == 0)
    # the two separators of each middle partition: not neighbours in A, yet
    # coupled in S (fill-in)
    for lo, hi in partitions(n, P)[1:-1]:
        i, j = sep.index(lo), sep.index(hi - 1)
        assert hi - 1 - lo > 1 and np.linalg.norm(Sb(i, j)) > 0
    # S^{-1} is the separator block of A^{-1}
    d, u, l = Mt
    A = np.zeros((n * b, n * b), np.complex128)
    for i in range(n):
        A[i * b:(i + 1) * b, i * b:(i + 1) * b] = d[i]
        if i + 1 < n:
            A[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = u[i]
            A[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = l[i]
    rS = np.concatenate([np.arange(k * b, (k + 1) * b) for k in sep])
    Ai = np.linalg.inv(A)
    assert _rel(np.linalg.inv(S), Ai[np.ix_(rS, rS)]) < 1e-12
    # the reduced right-hand side: block tridiagonal in separator order, and
    # S^{-1} B~ S^{-dagger} is the separator block of the dense X^s
    Bb = lambda i, j: BS[i * b:(i + 1) * b, j * b:(j + 1) * b]
    for i in range(m):
        for j in range(m):
            if abs(i - j) > 1:
                assert np.linalg.norm(Bb(i, j)) < 1e-12 * np.linalg.norm(BS)
    Bdense = np.zeros_like(A)
    for i in range(n):
        Bdense[i * b:(i + 1) * b, i * b:(i + 1) * b] = B[0][i]
        if i + 1 < n:
            Bdense[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = B[1][i]
            Bdense[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = B[2][i]
    XSd = Ai @ Bdense @ Ai.conj().T
    Si = np.linalg.inv(S)
    assert _rel(Si @ BS @ Si.conj().T, XSd[np.ix_(rS, rS)]) < 1e-12


@pytest.mark.parametrize("n,b,P", [(6, 1, 2), (7, 3, 2), (9, 3, 3), (11, 2, 4), (13, 3, 5),
                                   (8, 2, 4), (2, 2, 2), (3, 2, 2), (12, 2, 6)])
def test_block_form_matches_dense_and_reduced_system(n, b, P):
    Mt = _bt(7 * n + P, n, b)
    Bs = [_bt(7 * n + P + 1, n, b), _bt(7 * n + P + 2, n, b)]
    r = nested_dissection_blocks(Mt, P, Bs)
    rd = nested_dissection_selected(Mt, P, Bs)
    refR, refS = dense_selected(Mt, Bs)
    for k in range(3):
        assert _rel(r["XR"][k], refR[k]) < 1e-12
        for s in range(2):
            assert _rel(r["XS"][s][k], refS[s][k]) < 1e-12
    assert r["sep"] == rd["sep"]
    assert _rel(r["S"], rd["S"]) < 1e-12
    for s in range(2):
        assert _rel(r["BS"][s], rd["BS"][s]) < 1e-12
