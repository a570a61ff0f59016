"""Pins of the oracle's re-bin statistics (paper Sec. 6.1: lifts per particle
and time step), checked against computations that share nothing with it:

  - the mechanism of the paper's PIT (Sec. 5.1, Algorithm 1): a particle that
    has left its cell is lifted to the parent cell until a cell covers it;
    counted here step by step with exact rational positions;
  - the same mechanism in the dual tree for PIDT: the dual cell of a level-l
    vertex b covers x when x - b 3^-l lies in [-3^-l/2, 3^-l/2) on every axis
    (periodic), and its parent is the level-(l-1) vertex nearest to it;
  - for adaptive PIDT trees, dual cells as explicit sets of finest vertices
    and a lift loop that stops at the first cell holding the new one;
  - a hand-computed case on a 9 x 9 tree.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W


def _cell_centres(cells, S):
    return ((np.asarray(cells, np.float64) + 0.5) / S).T.copy()


def test_hand_computed_lifts_on_a_9x9_tree():
    o = oracle.OracleTree(W.regular_tree(2, 2))
    S = 9
    # (2,4)->(3,4) crosses a level-1 boundary: lifted to the root (2 lifts);
    # (0,0)->(1,0) stays inside level-1 cell (0,0): 1 lift; (8,0)->(0,0)
    # wraps (distance 1, root); (5,5) stays; (0,0)->(6,3) tunnels 3 cells
    # (periodic distance min(6, 3) = 3 on axis 0, 3 on axis 1).
    before = [(2, 4), (0, 0), (8, 0), (5, 5), (0, 0)]
    after = [(3, 4), (1, 0), (0, 0), (5, 5), (6, 3)]
    x0, x1 = _cell_centres(before, S), _cell_centres(after, S)
    for scheme in (oracle.PIT, oracle.PIDT):
        xs, _, _, start, perm = oracle.initial_sort(o, x0, x0, None, scheme)
        nb = o.bin_of(x1[:, perm], scheme)
        st = o.rebin_stats(start, nb, scheme)
        assert st["particles"] == 5 and st["movers"] == 4
        assert st["max_tunnel"] == 3
        if scheme == oracle.PIT:
            assert st["lifts"] == 7
            assert st["lift_hist"][:4] == [1, 1, 3, 0]
        else:
            # the dual cells of finest vertices (cell centres round up to the
            # upper corner): (3,5)->(4,5) shares the level-1 dual cell of
            # vertex (1,2) (finest 2..4, 5..7): 1 lift; (1,1)->(2,1) crosses
            # the level-1 dual cells 0 and 1 (finest -1..1, 2..4): 2 lifts;
            # (0,1)->(1,1) shares level-1 cell 0: 1 lift; (1,1)->(7,4): 2 lifts
            assert st["lifts"] == 6
            assert st["lift_hist"][:4] == [1, 2, 2, 0]


def _contains_pit(level, a, x):
    n = 3 ** level
    return all(Fraction(int(a[k]), n) <= x[k] < Fraction(int(a[k]) + 1, n) for k in range(len(a)))


def _contains_dual(level, b, x):
    if level == 0:
        return True
    h = Fraction(1, 3 ** level)
    for k in range(len(b)):
        off = (x[k] - int(b[k]) * h) % 1
        if not (off < h / 2 or off >= 1 - h / 2):
            return False
    return True


def _literal_stats(o, scheme, x0_sorted, start, x1_sorted):
    """Per particle: its old bin from the offsets, then lifts by the paper's
    mechanism (parent after parent until the cell covers the new position)."""
    leaves, pidt = o.leaves(), o.pidt_bins()
    nb1 = o.bin_of(x1_sorted, scheme)
    n_bins = len(start) - 1
    old = np.repeat(np.arange(n_bins), np.diff(start))
    hist = np.zeros(oracle.STATS_LEVELS, np.int64)
    movers = lifts = 0
    max_tunnel = 0
    for p in range(x0_sorted.shape[1]):
        b0, b1 = int(old[p]), int(nb1[p])
        if b0 == b1:
            hist[0] += 1
            continue
        movers += 1
        x = [Fraction(float(v)) for v in x1_sorted[:, p]]
        if scheme == oracle.PIT:
            lev, a = int(leaves["level"][b0]), [int(v) for v in leaves["coord"][b0]]
            n = 0
            while not _contains_pit(lev, a, x):
                lev, a, n = lev - 1, [v // 3 for v in a], n + 1
            anc = lambda b: [int(v) * 3 ** (o.L - int(leaves["level"][b])) for v in leaves["coord"][b]]
        else:
            lev, b = int(pidt["level"][b0]), [int(v) for v in pidt["b"][b0]]
            n = 0
            while not _contains_dual(lev, b, x):
                b = [((v + 1) // 3) % 3 ** (lev - 1) for v in b]
                lev, n = lev - 1, n + 1
            anc = lambda bb: [int(v) * 3 ** (o.L - int(pidt["level"][bb])) for v in pidt["b"][bb]]
        lifts += n
        hist[min(n, oracle.STATS_LEVELS - 1)] += 1
        A0, A1 = anc(b0), anc(b1)
        d = max(min(abs(u - v), o.S - abs(u - v)) for u, v in zip(A0, A1))
        max_tunnel = max(max_tunnel, d)
    return {"particles": x0_sorted.shape[1], "movers": movers, "lifts": lifts, "max_tunnel": max_tunnel,
            "lift_hist": [int(v) for v in hist]}


def _moved(rng, n, dim, S, max_cells):
    x0 = rng.random((dim, n))
    d = rng.integers(-max_cells, max_cells + 1, (dim, n)) + rng.random((dim, n)) - 0.5
    x1 = (x0 + d / S) % 1.0
    x1[x1 >= 1.0] = 0.0
    return x0, x1


@pytest.mark.parametrize("spec_name", ["reg2d_L2", "reg3d_L2", "disc2d_1_3"])
@pytest.mark.parametrize("scheme", [oracle.PIT, oracle.PIDT])
@pytest.mark.parametrize("max_cells", [1, 4, 50])
def test_stats_match_the_lift_mechanism(spec_name, scheme, max_cells):
    spec = {"reg2d_L2": lambda: W.regular_tree(2, 2), "reg3d_L2": lambda: W.regular_tree(3, 2),
            "disc2d_1_3": lambda: W.disc_tree(2, 1, 3)}[spec_name]()
    if scheme == oracle.PIDT and not spec_name.startswith("reg"):
        pytest.skip("adaptive PIDT: see test_adaptive_pidt_stats_match_dual_cell_sets")
    o = oracle.OracleTree(spec)
    rng = np.random.default_rng(max_cells * 7 + scheme)
    x0, x1 = _moved(rng, 600, spec.dim, o.S, max_cells)
    xs, _, _, start, perm = oracle.initial_sort(o, x0, x0, None, scheme)
    x1s = x1[:, perm]
    got = o.rebin_stats(start, o.bin_of(x1s, scheme), scheme)
    want = _literal_stats(o, scheme, xs, start, x1s)
    assert got == want


def _dual_set(b, level, L, S):
    """Finest vertices covered by the dual cell of the level-`level` vertex b."""
    s = 3 ** (L - level)
    axes = [{(int(bk) * s + j) % S for j in range(-(s - 1) // 2, (s - 1) // 2 + 1)} for bk in b]
    out = {()}
    for ax in axes:
        out = {t + (j,) for t in out for j in ax}
    return out


def test_adaptive_pidt_stats_match_dual_cell_sets():
    """On an adaptive tree the old and new dual cells can sit on different
    levels; the lift count is the number of parents taken from the old dual
    cell until one holds the new dual cell, checked on explicit vertex sets."""
    spec = W.disc_tree(2, 1, 3)
    o = oracle.OracleTree(spec)
    pidt = o.pidt_bins()
    rng = np.random.default_rng(5)
    x0, x1 = _moved(rng, 400, 2, o.S, 6)
    xs, _, _, start, perm = oracle.initial_sort(o, x0, x0, None, oracle.PIDT)
    nb1 = o.bin_of(x1[:, perm], oracle.PIDT)
    got = o.rebin_stats(start, nb1, oracle.PIDT)
    old = np.repeat(np.arange(len(start) - 1), np.diff(start))
    hist = np.zeros(oracle.STATS_LEVELS, np.int64)
    lifts = 0
    for p in range(len(nb1)):
        b0, b1 = int(old[p]), int(nb1[p])
        if b0 == b1:
            hist[0] += 1
            continue
        target = _dual_set(pidt["b"][b1], int(pidt["level"][b1]), o.L, o.S)
        lev, b, n = int(pidt["level"][b0]), [int(v) for v in pidt["b"][b0]], 0
        while not target <= _dual_set(b, lev, o.L, o.S):
            b = [((v + 1) // 3) % 3 ** (lev - 1) for v in b]
            lev, n = lev - 1, n + 1
        lifts += n
        hist[n] += 1
    assert got["lifts"] == lifts and got["lift_hist"] == [int(v) for v in hist]
    assert got["movers"] == int((nb1 != old).sum())
