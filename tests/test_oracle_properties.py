"""Property tests of the oracle's location and re-bin on random spacetrees
(paper Sec. 5.1 Theorem 1, Sec. 5.2 Theorem 2, Sec. 6.1 lift counts).

Hypothesis draws the tree (dimension, depth, which cells are refined), the
particle positions and displacements of up to 50 finest cells per axis.
Every property is checked against plain geometry computed here: the unique
leaf box (PIT) or dual box (PIDT) holding the point, the stable
stayers-then-arrivals bucket order, and the lift loop of the paper's PIT
mechanism.  derandomize keeps the examples the same from run to run.
"""
import itertools

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import workloads as W
from test_oracle_pins import _check_rebin, _geometric_leaves
from test_oracle_stats import _literal_stats

SETTINGS = settings(max_examples=80, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def trees(draw):
    dim = draw(st.sampled_from([2, 3]))
    L = draw(st.integers(1, 3 if dim == 2 else 2))
    p = draw(st.floats(0.15, 0.9))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    masks = [(rng.random((3 ** l) ** dim) < p).astype(np.uint8) for l in range(L)]
    masks[0][:] = 1          # at least one level below the root
    return W.TreeSpec(dim, L, masks)


@st.composite
def moved_sets(draw, tree):
    n = draw(st.integers(0, 120))
    max_cells = draw(st.sampled_from([0, 1, 3, 12, 50]))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    S = 3 ** tree.max_level
    x0 = rng.random((tree.dim, n))
    # a few positions on cell faces of every level
    if n:
        lv = rng.integers(0, tree.max_level + 1, n)
        face = rng.integers(0, 3 ** lv) / 3.0 ** lv
        ax = rng.integers(0, tree.dim, n)
        pick = rng.random(n) < 0.3
        x0[ax[pick], np.nonzero(pick)[0]] = face[pick]
    d = rng.integers(-max_cells, max_cells + 1, (tree.dim, n)) + rng.random((tree.dim, n)) - 0.5
    x1 = (x0 + d / S) % 1.0
    x1[x1 >= 1.0] = 0.0
    return x0, x1


def _brute_leaf(geo, L, x):
    S = 3 ** L
    I = np.minimum(np.floor(x * S), S - 1).astype(np.int64)     # the cell of fl(x S)
    out = []
    for p in range(x.shape[1]):
        hits = [(l, a) for l, a in geo
                if all(a[k] * 3 ** (L - l) <= I[k, p] < (a[k] + 1) * 3 ** (L - l) for k in range(x.shape[0]))]
        assert len(hits) == 1
        out.append(hits[0])
    return out


@SETTINGS
@given(data=st.data())
def test_locate_finds_the_unique_leaf_and_dual_cell(data):
    spec = data.draw(trees())
    x, _ = data.draw(moved_sets(spec))
    t = oracle.OracleTree(spec)
    L, d, S = spec.max_level, spec.dim, 3 ** spec.max_level
    leaf, pidt, _ = t.locate(x)
    lv, pb = t.leaves(), t.pidt_bins()
    for p, (l, a) in enumerate(_brute_leaf(_geometric_leaves(spec), L, x)):
        r = int(leaf[p])
        assert int(lv["level"][r]) == l and tuple(map(int, lv["coord"][r])) == a
        # the leaf corner whose level-l dual box [b s - s/2, b s + s/2) holds x S
        s = 3 ** (L - l)
        y2 = 2.0 * x[:, p] * S            # exact: doubling a double
        own = [tuple(((a[k] + c[k]) % 3 ** l) for k in range(d)) for c in itertools.product((0, 1), repeat=d)
               if all((2 * (a[k] + c[k]) - 1) * s <= y2[k] < (2 * (a[k] + c[k]) + 1) * s for k in range(d))]
        assert len(own) == 1
        q = int(pidt[p])
        assert int(pb["level"][q]) == l and tuple(map(int, pb["b"][q])) == own[0]


@SETTINGS
@given(data=st.data(), scheme=st.sampled_from([oracle.PIT, oracle.PIDT]))
def test_rebin_keeps_the_theorems_and_the_stable_order(data, scheme):
    spec = data.draw(trees())
    x0, x1 = data.draw(moved_sets(spec))
    t = oracle.OracleTree(spec)
    xs, _, _, start, perm0 = oracle.initial_sort(t, x0, x0, None, scheme)
    _check_rebin(t, scheme, xs, start, perm0, None, t.bin_of(x0, scheme))
    x1s = x1[:, perm0]
    nb = t.bin_of(x1s, scheme)
    perm, start1 = oracle.rebin(nb, t.n_bins(scheme), start)
    _check_rebin(t, scheme, x1s[:, perm], start1, perm, start, nb)
    assert start1[-1] == x0.shape[1]


@SETTINGS
@given(data=st.data())
def test_pit_lift_counts_follow_the_lift_loop(data):
    spec = data.draw(trees())
    x0, x1 = data.draw(moved_sets(spec))
    t = oracle.OracleTree(spec)
    xs, _, _, start, perm = oracle.initial_sort(t, x0, x0, None, oracle.PIT)
    x1s = x1[:, perm]
    got = t.rebin_stats(start, t.bin_of(x1s, oracle.PIT), oracle.PIT)
    assert got == _literal_stats(t, oracle.PIT, xs, start, x1s)
