"""Pins of the oracle's particle-handling benchmark pieces (paper Sec. 6
setup): free streaming with periodic or reflecting walls, the artificial
flops, and the ppc-driven refinement and coarsening of the tree.

  - free streaming against closed forms: the unfolded straight line folded
    by the triangle wave (reflecting) or taken modulo 1 (periodic), exact
    for dyadic positions and steps that never land on a wall;
  - hand cases at both walls, including a landing exactly on 1;
  - the flops leave every result unchanged;
  - adaptation: hand-built refine and coarsen cases, and the fixed point of
    repeated adaptation checked by brute-force counting of particles in the
    leaf boxes of the geometry generator.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _dyadic_set(rng, dim, n):
    # positions odd/2^12 and steps odd/2^11 (dt = 1/8): the unfolded
    # position always has an odd numerator over 2^12, so it never sits on 0
    # or 1 and every sum is exact
    x = (2 * rng.integers(0, 2048, (dim, n)) + 1) / 4096.0
    dx = (2 * rng.integers(-300, 300, (dim, n)) + 1) / 2048.0
    return x, dx * 8.0, 0.125


def test_reflecting_stream_is_the_folded_straight_line():
    rng = np.random.default_rng(3)
    t = oracle.OracleTree(W.regular_tree(2, 2))
    x0, v0, dt = _dyadic_set(rng, 2, 300)
    x, v = x0.copy(), v0.copy()
    for k in range(1, 40):
        x, v, _ = t.free_stream(x, v, dt, oracle.REFLECT)
        u = x0 + k * (v0 * dt)                # exact: small dyadics
        r = np.mod(u, 2.0)
        want_x = np.where(r < 1.0, r, 2.0 - r)
        want_v = np.where(r < 1.0, v0, -v0)
        assert np.array_equal(x, want_x) and np.array_equal(v, want_v)


def test_periodic_stream_is_the_straight_line_modulo_one():
    rng = np.random.default_rng(4)
    t = oracle.OracleTree(W.regular_tree(2, 2))
    x0, v0, dt = _dyadic_set(rng, 2, 300)
    x, v = x0.copy(), v0.copy()
    for k in range(1, 40):
        x, v, _ = t.free_stream(x, v, dt, oracle.PERIODIC)
        assert np.array_equal(x, np.mod(x0 + k * (v0 * dt), 1.0)) and np.array_equal(v, v0)


def test_reflection_hand_cases():
    t = oracle.OracleTree(W.regular_tree(1 + 1, 1))
    # rows: x, v with dt = 1/4 on axis 0 (axis 1 stays at 0.5 with v = 0)
    cases = [(0.125, -1.0, 0.125, 1.0),            # mirrored at 0
             (0.875, 1.0, 0.875, -1.0),            # mirrored at 1
             (0.75, 1.0, np.nextafter(1.0, 0.0), -1.0),   # lands on 1: just below it
             (0.25, -1.0, 0.0, -1.0),              # lands on 0: inside, no reflection
             (0.5, 0.5, 0.625, 0.5)]               # no wall
    x = np.array([[c[0] for c in cases], [0.5] * len(cases)])
    v = np.array([[c[1] for c in cases], [0.0] * len(cases)])
    x1, v1, b = t.free_stream(x, v, 0.25, oracle.REFLECT)
    assert list(x1[0]) == [c[2] for c in cases] and list(v1[0]) == [c[3] for c in cases]
    assert np.array_equal(b, t.bin_of(x1, oracle.PIT))
    _, _, b2 = t.free_stream(x, v, 0.25, oracle.REFLECT, scheme=oracle.PIDT)
    assert np.array_equal(b2, t.bin_of(x1, oracle.PIDT))
    with pytest.raises(ValueError):
        t.free_stream(np.array([[0.5], [0.5]]), np.array([[-6.0], [0.0]]), 0.25, oracle.REFLECT)


def test_flops_change_nothing():
    rng = np.random.default_rng(5)
    t = oracle.OracleTree(W.disc_tree(2, 1, 3))
    x, v = rng.random((2, 500)), rng.uniform(-1, 1, (2, 500))
    a = t.free_stream(x, v, 0.01, oracle.REFLECT, flops=0)
    b = t.free_stream(x, v, 0.01, oracle.REFLECT, flops=4096)
    for u, w in zip(a, b):
        assert np.array_equal(u, w)


# ---------------------------------------------------------------------------
# ppc-driven adaptivity
# ---------------------------------------------------------------------------

def _at_cells(cells, S, rng=None):
    """Particles at the centres of finest cells (list of coordinate tuples)."""
    return ((np.asarray(cells, np.float64) + 0.5) / S).T.copy()


def _masks(spec):
    return [np.asarray(m, np.uint8).ravel().tolist() for m in spec.refine]


def test_overfull_leaf_is_refined_once(adapt=None):
    adapt = adapt or oracle.adapt
    spec = W.regular_tree(2, 1)
    # level-1 leaf (1, 1) holds 4 particles, leaf (2, 0) one; ppc 3
    x = _at_cells([(1, 1)] * 4 + [(2, 0)], 3)
    new = adapt(spec, x, 3, 5)
    assert new.max_level == 2
    assert _masks(new)[0] == [1]
    want = [0] * 9
    want[1 + 3 * 1] = 1
    assert _masks(new)[1] == want
    # the cap: nothing below max_level 1
    assert _masks(adapt(spec, x, 3, 1)) == [[1]]


def test_underfull_children_are_coarsened(adapt=None):
    adapt = adapt or oracle.adapt
    m1 = np.zeros(9, np.uint8)
    m1[0] = 1
    spec = W.TreeSpec(2, 2, [np.ones(1, np.uint8), m1])
    # two particles in the children of level-1 cell (0, 0), ppc 2: coarsened
    x = _at_cells([(0, 0), (2, 1), (5, 5)], 9)
    new = adapt(spec, x, 2, 4)
    assert new.max_level == 1 and _masks(new) == [[1]]
    # three particles there: kept
    x3 = _at_cells([(0, 0), (2, 1), (1, 1), (5, 5)], 9)
    assert _masks(adapt(spec, x3, 2, 4)) == _masks(spec)
    # the root is never coarsened
    assert _masks(adapt(W.regular_tree(2, 1), x[:, :1] * 0 + 0.5, 5, 4)) == [[1]]


def test_cell_with_a_refined_child_is_not_coarsened(adapt=None):
    adapt = adapt or oracle.adapt
    m1 = np.zeros(9, np.uint8)
    m1[0] = 1
    m2 = np.zeros(81, np.uint8)
    m2[0] = 1
    spec = W.TreeSpec(2, 3, [np.ones(1, np.uint8), m1, m2])
    x = _at_cells([(0, 0)], 27)
    new = adapt(spec, x, 4, 4)
    # level-2 cell (0,0) has leaf children holding 1 <= 4: coarsened; level-1
    # cell (0,0) had a refined child this time, so it stays refined
    assert new.max_level == 2 and _masks(new)[1] == m1.tolist()


def _brute_counts(spec, x):
    S = 3 ** spec.max_level
    I = np.minimum(np.floor(x * S), S - 1).astype(np.int64)
    out = {}
    for l, ids in enumerate(W.leaf_cells(spec)):
        n, s = 3 ** l, 3 ** (spec.max_level - l)
        for i in ids:
            a, r = [], int(i)
            for _ in range(spec.dim):
                a.append(r % n)
                r //= n
            inside = np.all([(I[k] // s) == a[k] for k in range(spec.dim)], axis=0)
            out[(l, tuple(a))] = int(inside.sum())
    return out


@pytest.mark.parametrize("dim,start", [(2, "homogeneous"), (2, "subbox"), (3, "subbox")])
def test_repeated_adaptation_reaches_the_ppc_fixed_point(dim, start, adapt=None):
    adapt = adapt or oracle.adapt
    rng = np.random.default_rng(11 + dim)
    n, ppc, cap = (3000, 40, 5) if dim == 2 else (1500, 30, 3)
    x = rng.random((dim, n)) * (0.1 if start == "subbox" else 1.0)
    spec = W.regular_tree(dim, 1)
    for _ in range(12):
        new = adapt(spec, x, ppc, cap)
        if new.max_level == spec.max_level and _masks(new) == _masks(spec):
            break
        spec = new
    else:
        pytest.fail("no fixed point")
    cnt = _brute_counts(spec, x)
    assert sum(cnt.values()) == n
    for (l, a), c in cnt.items():
        assert c <= ppc or l == cap
    # no refined non-root cell with all-leaf children holding <= ppc
    for (l, a), c in cnt.items():
        if l < 2:
            continue
        parent = tuple(v // 3 for v in a)
        sib = [(l, tuple(3 * parent[k] + o[k] for k in range(dim)))
               for o in np.ndindex(*(3,) * dim)]
        if all(sb in cnt for sb in sib):
            assert sum(cnt[sb] for sb in sib) > ppc
    if start == "subbox":
        assert spec.max_level > 1


# ---------------------------------------------------------------------------
# raPIDT's v_max (Sec. 5.4, Eq. (vmax))
# ---------------------------------------------------------------------------

def test_vmax_hand_case():
    spec = W.regular_tree(2, 2)
    # one particle with |v| = (0.25, -0.7) in finest cell (4, 4), one slow in
    # cell (0, 0); everything else empty
    x = np.array([[4.5 / 9, 0.5 / 9], [4.5 / 9, 0.5 / 9]])
    v = np.array([[0.25, 0.01], [-0.7, 0.0]])
    pit, q = oracle.vmax_cells(spec, x, v, oracle.PIT, dt=0.5)
    assert pit[0][0] == 0.7
    assert pit[1][1 + 3 * 1] == 0.7 and pit[1][0] == 0.01 and pit[1].sum() == 0.71
    assert pit[2][4 + 9 * 4] == 0.7 and pit[2][0] == 0.01 and np.count_nonzero(pit[2]) == 2
    # predicate: 0.7 * 0.5 <= 1/3 fails at level 1, holds at level 0
    assert q[0][0] == 1 and q[1][4] == 0 and q[1][0] == 1 and q[2][40] == 0
    # dt = 0.3: 0.21 <= h = 1/3 at level 1 (though above h/2), above 1/9 at level 2
    _, q3 = oracle.vmax_cells(spec, x, v, oracle.PIT, dt=0.3)
    assert q3[1][4] == 1 and q3[2][40] == 0
    # cells that do not exist are never quiet
    _, qa = oracle.vmax_cells(W.disc_tree(2, 1, 2), x, v, oracle.PIT, dt=0.3)
    assert qa[2].sum() == np.count_nonzero(W.disc_tree(2, 1, 2).refine[1]) * 9 - (1 if qa[2][40] == 0 else 0)
    # PIDT: the fast particle's dual cell is that of vertex (5, 5) (nearest
    # corner of cell (4, 4), ties up), shared by the four leaves around it
    pidt = oracle.vmax_cells(spec, x, v, oracle.PIDT)
    for c in [(4, 4), (5, 4), (4, 5), (5, 5)]:
        assert pidt[2][c[0] + 9 * c[1]] == 0.7
    assert pidt[2][3 + 9 * 3] == 0.0


@pytest.mark.parametrize("scheme", [oracle.PIT, oracle.PIDT])
def test_vmax_of_a_cell_is_the_max_over_its_subtree_particles(scheme):
    rng = np.random.default_rng(8)
    spec = W.disc_tree(2, 1, 3)
    x, v = rng.random((2, 700)), rng.uniform(-1, 1, (2, 700))
    out = oracle.vmax_cells(spec, x, v, scheme)
    S = 27
    I = np.minimum(np.floor(x * S), S - 1).astype(np.int64)
    sp = np.abs(v).max(axis=0)
    # the root holds every particle; for PIT a level-1 cell holds exactly
    # the particles inside it, for PIDT at least those
    assert out[0][0] == sp.max()
    for a0 in range(3):
        for a1 in range(3):
            inside = (I[0] // 9 == a0) & (I[1] // 9 == a1)
            val = out[1][a0 + 3 * a1]
            if scheme == oracle.PIT:
                assert val == (sp[inside].max() if inside.any() else 0.0)
            else:
                assert val >= (sp[inside].max() if inside.any() else 0.0)
