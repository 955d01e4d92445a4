"""Pins of the oracle's tournament pivoting (Sec. 7.3; no GPU).

* a 6 x 2 block column worked by hand: the tournament (blocks of 3 rows,
  rounds of 2 sets) keeps rows 0 and 3 where partial pivoting takes rows 0
  and 5, and the factors of the chosen order are fixed exactly (every value
  is a dyadic rational, so binary64 is exact);
* with one block (block >= m) the tournament is one local LU with partial
  pivoting, so its pivots are those of dgetrf;
* for v = 1 every round keeps the largest |a|, so the winner is the row of
  the column's largest magnitude (first on ties);
* on small random integer matrices, the orders agree with an exact-rational
  tournament written independently here (Fractions);
* the block-column factors satisfy P A = L U to rounding, the chosen rows
  are distinct, and |L| may exceed 1 (it does in the hand example).
"""
from fractions import Fraction

import numpy as np
import pytest

HAND = np.array([[-4, -1], [-3, -3], [-2, 0], [0, -4], [2, 0], [1, -4]], dtype=np.float64)


def test_hand_worked_tournament(oracle_mod):
    """Blocks {0,1,2} and {3,4,5}.  Block 0: pivot row 0 (|-4|); row 1
    becomes -3 - (3/4)(-1) = -9/4, row 2 becomes 0 - (1/2)(-1) = 1/2, so the
    candidates are [0, 1].  Block 1: pivot row 4 (|2|); rows 3 and 5 both
    become -4 (multipliers 0 and 1/2 against a zero), the tie goes to row 3:
    candidates [4, 3].  Final round over rows [0, 1, 4, 3]: pivot row 0;
    row 1 -> -9/4, row 4 -> 0 - (-1/2)(-1) = -1/2, row 3 -> -4: winner 3.
    Partial pivoting over all six rows instead finds row 5 at
    -4 - (-1/4)(-1) = -17/4 in the second column."""
    assert oracle_mod.tournament_pivots(HAND, 2, 3, 2) == [0, 3]
    assert oracle_mod.gepp_rows(HAND, range(6), 2) == [0, 5]
    lu, ipiv, info = oracle_mod.calu_panel(HAND, 2, 3, 2)
    assert info == 0 and list(ipiv) == [1, 4]
    # rows after the interchanges: 0, 3, 2, 1, 4, 5
    want = np.array([[-4, -1], [0, -4], [0.5, -0.125], [0.75, 0.5625], [-0.5, 0.125], [-0.25, 1.0625]])
    assert np.array_equal(lu, want)
    assert np.abs(np.tril(lu, -1)).max() > 1.0


def test_one_block_is_partial_pivoting(oracle_mod):
    rng = np.random.default_rng(11)
    a = rng.uniform(-1, 1, (300, 32))
    _, gp, _ = oracle_mod.dgetrf(a)
    assert oracle_mod.tournament_pivots(a, 32, 512, 8) == oracle_mod.gepp_rows(a, range(300), 32)
    lu, ipiv, info = oracle_mod.calu_panel(a, 32, 512, 8)
    assert info == 0 and np.array_equal(ipiv, gp)
    ref, _, _ = oracle_mod.dgetrf(a)
    assert np.abs(lu - ref).max() < 1e-13


@pytest.mark.parametrize("block,fanin", [(4, 2), (7, 3), (16, 8)])
def test_width_one_is_column_argmax(oracle_mod, block, fanin):
    rng = np.random.default_rng(block)
    for _ in range(20):
        col = rng.integers(-9, 10, (50, 1)).astype(np.float64)
        mag = np.abs(col[:, 0])
        assert oracle_mod.tournament_pivots(col, 1, block, fanin) == [int(np.argmax(mag))]


def _gepp_exact(rows, v):
    """Exact-rational LU with partial pivoting of [(row id, values)]: the ids
    of the rows it brings to the top, in pivot order (first on ties)."""
    r = [(i, list(x)) for i, x in rows]
    k = min(v, len(r))
    for j in range(k):
        best = j
        for i in range(j + 1, len(r)):
            if abs(r[i][1][j]) > abs(r[best][1][j]):
                best = i
        r[j], r[best] = r[best], r[j]
        piv = r[j][1][j]
        if piv == 0:
            continue
        for i in range(j + 1, len(r)):
            l = r[i][1][j] / piv
            r[i] = (r[i][0], [r[i][1][c] - l * r[j][1][c] if c > j else r[i][1][c] for c in range(len(r[i][1]))])
    return [x[0] for x in r[:k]]


def _tournament_exact(a, v, block, fanin):
    m = a.shape[0]
    rows = lambda ids: [(i, [Fraction(int(x)) for x in a[i]]) for i in ids]  # noqa: E731
    sets = [_gepp_exact(rows(range(s, min(m, s + block))), v) for s in range(0, m, block)]
    while len(sets) > 1:
        sets = [_gepp_exact(rows([r for st in sets[i:i + fanin] for r in st]), v)
                for i in range(0, len(sets), fanin)]
    return sets[0]


@pytest.mark.parametrize("m,v,block,fanin", [(12, 3, 4, 2), (20, 4, 5, 3), (17, 2, 3, 2), (9, 3, 9, 2)])
def test_against_exact_rational_tournament(oracle_mod, m, v, block, fanin):
    rng = np.random.default_rng(1000 + m)
    checked = 0
    for _ in range(30):
        a = rng.integers(-20, 21, (m, v)).astype(np.float64)
        exact = _tournament_exact(a, v, block, fanin)
        got = oracle_mod.tournament_pivots(a, v, block, fanin)
        assert got == exact
        checked += 1
    assert checked == 30


@pytest.mark.parametrize("fanin", [2, 8])
def test_block_column_reconstruction(oracle_mod, fanin):
    rng = np.random.default_rng(7 + fanin)
    m, n = 600, 96
    a = rng.uniform(-1, 1, (m, n))
    lu, ipiv, info = oracle_mod.calu_panel(a, 32, 256, fanin)
    assert info == 0
    perm = oracle_mod.ipiv_to_perm(ipiv, m)
    assert len(set(perm.tolist())) == m
    L = np.tril(lu, -1) + np.eye(m, n)
    U = np.triu(lu[:n])
    assert np.abs(a[perm] - L @ U).max() <= 1e-13 * np.abs(a).max() * n
    _, gp, _ = oracle_mod.dgetrf(a)
    assert not np.array_equal(ipiv, gp)  # several blocks: a different, equally valid order


def test_mixed_getrf_tournament_reduces_to_partial(oracle_mod):
    rng = np.random.default_rng(3)
    n = 200
    a = rng.uniform(-1, 1, (n, n))
    w0, p0, i0 = oracle_mod.mixed_getrf(a, 64, oracle_mod.FMT_BF16, 128, 128)
    w1, p1, i1 = oracle_mod.mixed_getrf(a, 64, oracle_mod.FMT_BF16, 128, 128, tournament=(32, 4096, 8))
    assert i0 == i1 == 0 and np.array_equal(p0, p1)
    assert np.abs(w0.astype(np.float64) - w1).max() <= 1e-5 * np.abs(w0).max()
