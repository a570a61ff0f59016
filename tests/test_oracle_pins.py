"""Pins that tie the oracle to the paper and to mathematics, not to itself.

Each group names what fixes the expected values: brute force on tiny inputs
in exact rational arithmetic, closed forms, invariants (Theorems 1 and 2 of
the paper, conservation), and textbook special cases.  A plausible slip in
the oracle (a dropped term, a flipped sign, a swapped index or operand)
fails at least one of these; ``test_oracle_mutants.py`` checks that claim by
compiling deliberately broken copies of the oracle.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lattice(dim, n):
    return [c for c in itertools.product(range(n), repeat=dim)]


# ---------------------------------------------------------------------------
# Peano index (paper Sec. 4.2, Peano ordering of cells and of their arrays)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim,L", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_peano_is_a_face_continuous_bijection(dim, L):
    n = 3 ** L
    pts = _lattice(dim, n)
    keys = [oracle.peano(dim, L, p[::-1]) for p in pts]      # p[::-1]: axis 0 first
    assert sorted(keys) == list(range(n ** dim))
    inv = {k: np.array(p[::-1]) for p, k in zip(pts, keys)}
    for k in range(n ** dim - 1):
        assert np.abs(inv[k] - inv[k + 1]).sum() == 1, (k, inv[k], inv[k + 1])
    # the curve runs from one corner of the box to the opposite one
    assert (inv[0] == 0).all() and (inv[n ** dim - 1] == n - 1).all()


@pytest.mark.parametrize("dim,L", [(2, 1), (2, 2), (3, 1)])
def test_peano_prefix_property(dim, L):
    """A child's index over 3^d is its parent's index: cells nest along the curve."""
    n = 3 ** (L + 1)
    for p in _lattice(dim, n):
        c = list(p)
        parent = [v // 3 for v in c]
        assert oracle.peano(dim, L + 1, c) // 3 ** dim == oracle.peano(dim, L, parent)


def test_peano_matches_textbook_level1_order():
    rows = [list(map(int, ln.split())) for ln in open(os.path.join(GOLDEN, "peano_2d_level1.txt"))
            if ln.strip() and not ln.startswith("#")]
    for key, i0, i1 in rows:
        assert oracle.peano(2, 1, [i0, i1]) == key


# ---------------------------------------------------------------------------
# Spacetree tables (paper Sec. 4)
# ---------------------------------------------------------------------------

def _geometric_leaves(spec):
    """Leaves from the generator's geometry: list of (level, coords)."""
    out = []
    for l, ids in enumerate(W.leaf_cells(spec)):
        n = 3 ** l
        for i in ids:
            c, r = [], int(i)
            for _ in range(spec.dim):
                c.append(r % n)
                r //= n
            out.append((l, tuple(c)))
    return out


@pytest.mark.parametrize("spec", [W.regular_tree(2, 3), W.regular_tree(3, 2), W.disc_tree(2, 2, 4),
                                  W.disc_tree(3, 1, 3), W.disc_tree(2, 1, 3, radius=(1, 3))])
def test_tree_tables_match_geometry(spec):
    t = oracle.OracleTree(spec)
    geo = _geometric_leaves(spec)
    lv = t.leaves()
    assert t.n_leaves == len(geo)
    got = sorted((int(l), tuple(int(v) for v in c)) for l, c in zip(lv["level"], lv["coord"]))
    assert got == sorted(geo)
    d, S, L = spec.dim, t.S, spec.max_level
    # leaves tile the finest-level curve: their index ranges are contiguous and exhaustive
    start = (lv["key"] // 64).astype(object)
    span = [3 ** (d * (L - int(l))) for l in lv["level"]]
    assert start[0] == 0
    for r in range(t.n_leaves - 1):
        assert start[r] + span[r] == start[r + 1]
    assert start[-1] + span[-1] == 3 ** (d * L)
    # vertices: brute-force distinct corner positions, lexicographic
    pos = set()
    for l, a in geo:
        s = 3 ** (L - l)
        for c in itertools.product((0, 1), repeat=d):
            pos.add(tuple(((a[k] + c[k]) * s) % S for k in range(d)))
    want = sorted(pos, key=lambda p: sum(p[k] * S ** k for k in range(d)))
    vp = t.vertex_positions()
    assert [tuple(map(int, p)) for p in vp] == want
    # leaf -> corner vertex table points at the right positions
    for r in range(t.n_leaves):
        l, a = int(lv["level"][r]), lv["coord"][r]
        s = 3 ** (L - l)
        for c in range(1 << d):
            bits = [(c >> k) & 1 for k in range(d)]
            p = tuple(int(((a[k] + bits[k]) * s) % S) for k in range(d))
            assert tuple(vp[lv["vtx"][r, c]]) == p
    # PIDT bins: one per (level, vertex of a leaf of that level)
    pb = t.pidt_bins()
    pairs = set()
    for l, a in geo:
        for c in itertools.product((0, 1), repeat=d):
            pairs.add((l, tuple((a[k] + c[k]) % 3 ** l for k in range(d))))
    assert t.n_pidt == len(pairs)
    assert np.all(pb["key"][1:] > pb["key"][:-1])
    assert sorted((int(l), tuple(map(int, b))) for l, b in zip(pb["level"], pb["b"])) == sorted(pairs)


def test_config3_tree_sizes():
    spec = W.disc_tree(2, 4, 6)
    t = oracle.OracleTree(spec)
    assert t.n_leaves == sum(x.size for x in W.leaf_cells(spec)) == 74609


@pytest.mark.parametrize("dim,L", [(2, 2), (2, 3), (3, 2)])
def test_regular_pidt_order_walks_neighbouring_vertices(dim, L):
    """On a regular tree consecutive PIDT bins are lattice neighbours (dual cells nest)."""
    t = oracle.OracleTree(W.regular_tree(dim, L))
    b = t.pidt_bins()["b"]
    S = t.S
    for i in range(t.n_pidt - 1):
        dlt = (b[i + 1] - b[i]) % S
        dlt = np.minimum(dlt, S - dlt)
        assert dlt.sum() == 1


# ---------------------------------------------------------------------------
# Location: Theorem 1 (PIT) and Theorem 2 (PIDT), brute force in exact arithmetic
# ---------------------------------------------------------------------------

def _adversarial_positions(rng, dim, L, n_rand):
    xs = [rng.random((dim, n_rand))]
    faces = []
    for lvl in range(L + 1):
        m = 3 ** lvl
        for i in rng.integers(0, m, 12):
            base = i / m
            mid = (2 * i + 1) / (2 * m)          # cell midpoint: a dual-cell face
            for cand in (base, np.nextafter(base, 2.0), np.nextafter(base, -1.0),
                         mid, np.nextafter(mid, 2.0), np.nextafter(mid, -1.0)):
                if 0.0 <= cand < 1.0:
                    faces.append(cand)
    faces += [0.0, np.nextafter(1.0, 0.0)]
    faces = np.array(faces)
    k = faces.size
    for ax in range(dim):
        arr = rng.random((dim, k))
        arr[ax] = faces
        xs.append(arr)
    # points on lattice corners in every axis
    arr = np.stack([faces[rng.permutation(k)] for _ in range(dim)])
    xs.append(arr)
    return np.concatenate(xs, axis=1)


@pytest.mark.parametrize("spec", [W.regular_tree(2, 2), W.disc_tree(2, 2, 4), W.disc_tree(3, 1, 3)])
def test_locate_matches_brute_force(spec):
    rng = np.random.default_rng(7)
    d, L = spec.dim, spec.max_level
    t = oracle.OracleTree(spec)
    S = t.S
    x = _adversarial_positions(rng, d, L, 300)
    leaf, pidt, cell = t.locate(x)
    lv = t.leaves()
    pb = t.pidt_bins()
    geo = _geometric_leaves(spec)
    for p in range(x.shape[1]):
        y = [Fraction(float(x[k, p]) * S) for k in range(d)]       # the single rounding y = fl(x S)
        yc = [min(v, Fraction(S) - Fraction(1, 2 ** 40)) if v == S else v for v in y]
        # brute force: the unique leaf whose closed-open box holds y (y == S is the last cell)
        hits = [(l, a) for l, a in geo
                if all(a[k] * 3 ** (L - l) <= yc[k] < (a[k] + 1) * 3 ** (L - l) for k in range(d))]
        assert len(hits) == 1
        l, a = hits[0]
        r = leaf[p]
        assert int(lv["level"][r]) == l and tuple(map(int, lv["coord"][r])) == a
        # brute force PIDT: the level-l vertex whose dual box [b s - s/2, b s + s/2) holds y
        s = 3 ** (L - l)
        own = []
        for c in itertools.product((0, 1), repeat=d):
            b = [a[k] + c[k] for k in range(d)]
            if all(Fraction(2 * b[k] - 1, 2) * s <= y[k] < Fraction(2 * b[k] + 1, 2) * s for k in range(d)):
                own.append(tuple(v % 3 ** l for v in b))
        assert len(own) == 1
        q = pidt[p]
        assert int(pb["level"][q]) == l and tuple(map(int, pb["b"][q])) == own[0]


def test_locate_rejects_positions_outside_the_box():
    t = oracle.OracleTree(W.regular_tree(2, 2))
    for bad in (1.0, -1e-300, np.nan, np.inf):
        with pytest.raises(ValueError):
            t.locate(np.array([[0.5], [bad]]))


# ---------------------------------------------------------------------------
# d-linear restriction and its transpose (paper Sec. 3, steps 1 and 3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("spec", [W.regular_tree(2, 3), W.disc_tree(2, 2, 4), W.disc_tree(3, 1, 3)])
def test_weights_exact_and_partition_of_unity(spec):
    rng = np.random.default_rng(3)
    t = oracle.OracleTree(spec)
    d, L, S = t.dim, t.L, t.S
    x = _adversarial_positions(rng, d, L, 200)
    w, vtx = t.weights(x)
    leaf, _, _ = t.locate(x)
    lv = t.leaves()
    assert np.all(np.abs(w.sum(axis=1) - 1.0) <= 4 * U)
    assert np.all(w >= 0.0)
    for p in range(x.shape[1]):
        l, a = int(lv["level"][leaf[p]]), lv["coord"][leaf[p]]
        s = 3 ** (L - l)
        f = [(Fraction(float(x[k, p]) * S) - int(a[k]) * s) / s for k in range(d)]
        for c in range(1 << d):
            we = Fraction(1)
            for k in range(d):
                we *= f[k] if (c >> k) & 1 else 1 - f[k]
            assert abs(float(we) - w[p, c]) <= 8 * U


def test_gather_reproduces_constant_and_linear_fields():
    spec = W.disc_tree(2, 2, 4)
    t = oracle.OracleTree(spec)
    rng = np.random.default_rng(11)
    n = 4000
    x = rng.random((2, n)) * 0.8              # keep away from the periodic seam
    pos = t.vertex_positions().T.astype(float)            # finest units
    E = np.stack([np.full(t.n_vertices, 2.5), 0.3 + 0.01 * pos[0] - 0.02 * pos[1]])
    _, _, ep, _ = t.gather_push(x, np.zeros((2, n)), E, 0.0, 0.0)
    assert np.all(np.abs(ep[0] - 2.5) <= 8 * U * 2.5)
    y = x * t.S
    want = 0.3 + 0.01 * y[0] - 0.02 * y[1]
    assert np.max(np.abs(ep[1] - want)) <= 1e-13


def test_particle_on_a_vertex_sits_entirely_there():
    t = oracle.OracleTree(W.regular_tree(2, 3))
    x = np.array([[0.0, 0.0], [0.0, 0.0]])
    w, vtx = t.weights(x[:, :1])
    assert w[0, 0] == 1.0 and w[0, 1:].sum() == 0.0 and vtx[0, 0] == 0
    rho = t.deposit(x[:, :1], None, -0.25)
    assert rho[0] == -0.25 and np.count_nonzero(rho) == 1


def test_deposit_exact_small_and_adjoint_to_gather():
    spec = W.disc_tree(2, 2, 4)
    t = oracle.OracleTree(spec)
    rng = np.random.default_rng(5)
    n = 300
    x = rng.random((2, n))
    q = -rng.random(n)
    rho = t.deposit(x, q)
    lv = t.leaves()
    leaf, _, _ = t.locate(x)
    exact = [Fraction(0)] * t.n_vertices
    for p in range(n):
        l, a = int(lv["level"][leaf[p]]), lv["coord"][leaf[p]]
        s = 3 ** (t.L - l)
        f = [(Fraction(float(x[k, p]) * t.S) - int(a[k]) * s) / s for k in range(2)]
        for c in range(4):
            we = (f[0] if c & 1 else 1 - f[0]) * (f[1] if c & 2 else 1 - f[1])
            exact[lv["vtx"][leaf[p], c]] += Fraction(float(q[p])) * we
    ex = np.array([float(e) for e in exact])
    assert np.max(np.abs(rho - ex)) <= 4 * U * np.abs(q).sum()
    # <rho, E> = sum_p q_p E_p: the deposit is the transpose of the gather
    E = rng.standard_normal((2, t.n_vertices))
    _, _, ep, _ = t.gather_push(x, np.zeros((2, n)), E, 0.0, 0.0)
    lhs = rho @ E[0]
    rhs = np.sum(q * ep[0])
    assert abs(lhs - rhs) <= 1e-12 * np.abs(q).sum() * np.abs(E).max()


@pytest.mark.parametrize("name", ["config1", "small_adaptive", "small_3d"])
def test_deposit_conserves_charge(name):
    wl = W.by_name(name)
    t = oracle.OracleTree(wl.tree)
    rho = t.deposit(wl.x, wl.q, wl.q_uniform)
    qsum = wl.q.sum() if wl.q is not None else wl.q_uniform * wl.n
    qabs = np.abs(wl.q).sum() if wl.q is not None else abs(wl.q_uniform) * wl.n
    assert abs(rho.sum() - qsum) <= (1 << wl.dim) * wl.n * U * qabs


# ---------------------------------------------------------------------------
# Push (paper Sec. 3 step 4): leapfrog, periodic wrap
# ---------------------------------------------------------------------------

def test_free_streaming_matches_closed_form():
    t = oracle.OracleTree(W.disc_tree(2, 2, 4))
    rng = np.random.default_rng(2)
    n, steps, dt = 500, 40, 0.37
    x0 = rng.random((2, n))
    v0 = rng.standard_normal((2, n)) * 0.3
    x, v = x0.copy(), v0.copy()
    E = np.zeros((2, t.n_vertices))
    for _ in range(steps):
        x, v, _, _ = t.gather_push(x, v, E, -1.0, dt)
    assert np.array_equal(v, v0)
    want = (x0 + steps * v0 * dt) % 1.0
    err = np.abs(x - want)
    err = np.minimum(err, 1.0 - err)
    assert err.max() <= 4 * steps * U * (1 + np.abs(v0 * dt).max())
    assert np.all((x >= 0.0) & (x < 1.0))


def test_push_kicks_against_the_field_for_negative_charge():
    t = oracle.OracleTree(W.regular_tree(2, 2))
    E = np.zeros((2, t.n_vertices))
    E[0] = 1.0
    x = np.array([[0.5], [0.5]])
    x1, v1, ep, _ = t.gather_push(x, np.zeros((2, 1)), E, -1.0 * 0.1, 0.1)
    assert ep[0, 0] == 1.0 and v1[0, 0] == -0.1 and v1[1, 0] == 0.0
    assert x1[0, 0] == 0.5 + (-0.1) * 0.1


def test_wrap_never_returns_one():
    t = oracle.OracleTree(W.regular_tree(2, 1))
    E = np.zeros((2, t.n_vertices))
    x = np.array([[0.0, 0.5], [0.0, 0.5]])
    v = np.array([[-1e-30, 0.5], [1e-30, -0.5]])
    x1, _, _, _ = t.gather_push(x, v, E, 0.0, 1.0)
    assert np.all((x1 >= 0.0) & (x1 < 1.0))
    assert x1[0, 0] == 0.0          # 0 - 1e-30 rounds to 1.0 after the wrap, taken as 0
    assert x1[0, 1] == 0.0 and x1[1, 1] == 0.0


# ---------------------------------------------------------------------------
# Re-bin (Theorems 1 and 2; stable bucket order)
# ---------------------------------------------------------------------------

def _check_rebin(t, scheme, x_out, start, perm, old_start, new_bin):
    n = perm.size
    assert np.array_equal(np.sort(perm), np.arange(n))
    nb_sorted = np.repeat(np.arange(t.n_bins(scheme)), np.diff(start))
    assert np.array_equal(nb_sorted, new_bin[perm])
    # Theorem 1 / 2: every particle sits in the box (dual box) of its bin
    d, L, S = t.dim, t.L, t.S
    y = x_out * S
    if scheme == oracle.PIT:
        lv = t.leaves()
        s = 3.0 ** (L - lv["level"][nb_sorted])
        a = lv["coord"][nb_sorted].T
        I = np.minimum(np.floor(y), S - 1)
        assert np.all((I >= a * s) & (I < (a + 1) * s))
    else:
        pb = t.pidt_bins()
        s = 3.0 ** (L - pb["level"][nb_sorted])
        b = pb["b"][nb_sorted].T * s
        off = (y - b + s / 2.0) % S           # position relative to the dual box's lower face
        assert np.all((off >= -1e-9) & (off < s + 1e-9))
    # order: inside each bin stayers first, each sub-sequence in old order
    if old_start is not None:
        old_bin = np.repeat(np.arange(t.n_bins(scheme)), np.diff(old_start))
        for b in range(t.n_bins(scheme)):
            seg = perm[start[b]:start[b + 1]]
            stay = old_bin[seg] == b
            k = stay.sum()
            assert stay[:k].all() and not stay[k:].any()
            assert np.all(np.diff(seg[:k]) > 0) and np.all(np.diff(seg[k:]) > 0)
    else:
        for b in range(t.n_bins(scheme)):
            assert np.all(np.diff(perm[start[b]:start[b + 1]]) > 0)


@pytest.mark.parametrize("name,scheme", [("config1", 0), ("config1", 1), ("small_adaptive", 0),
                                         ("small_adaptive", 1), ("small_3d", 0), ("small_3d", 1),
                                         ("small_3d_adaptive", 0), ("small_3d_adaptive", 1)])
def test_step_satisfies_theorems_and_order(name, scheme):
    wl = W.by_name(name)
    t = oracle.OracleTree(wl.tree)
    nb0 = t.bin_of(wl.x, scheme)
    perm0, start0 = oracle.rebin(nb0, t.n_bins(scheme), None)
    _check_rebin(t, scheme, wl.x[:, perm0], start0, perm0, None, nb0)
    x, v = wl.x[:, perm0], wl.v[:, perm0]
    q = None if wl.q is None else wl.q[perm0]
    E = wl.field(t.vertex_positions_unit())
    for _ in range(2):
        r = oracle.step(t, x, v, E, wl.qm * wl.dt, wl.dt, start0, scheme, q, wl.q_uniform)
        _check_rebin(t, scheme, r["x"], r["bin_start"], r["perm"], start0, r["new_bin"])
        x, v, q, start0 = r["x"], r["v"], r["q"], r["bin_start"]


def test_rebin_rejects_bad_bins():
    with pytest.raises(ValueError):
        oracle.rebin(np.array([0, 5]), 3, None)
    with pytest.raises(ValueError):
        oracle.rebin(np.array([0, 1]), 2, np.array([0, 1, 3]))


def test_rebin_empty_input():
    perm, start = oracle.rebin(np.zeros(0, np.int32), 4, None)
    assert perm.size == 0 and np.array_equal(start, np.zeros(5))


# ---------------------------------------------------------------------------
# Physics (paper App. A): momentum, cold oscillation, Bohm-Gross dispersion
# ---------------------------------------------------------------------------

def _mode_series(tree, x, v, qmdt, dt, steps, q_uniform):
    amp = []

    def rec(it, rho, V, E, xx, vv):
        n = 3 ** tree.L
        g = E[0].reshape((n,) * tree.dim)
        axes = tuple(range(tree.dim - 1))
        line = g.mean(axis=axes) if axes else g
        amp.append(np.imag(np.fft.fft(line)[1]))
    oracle.langmuir_run(tree, x, v, qmdt, dt, steps, q_uniform, rec)
    return np.array(amp)


def _frequency(series, dt):
    s = series - series.mean()
    idx = np.nonzero(np.sign(s[:-1]) * np.sign(s[1:]) < 0)[0]
    tz = idx + s[idx] / (s[idx] - s[idx + 1])
    assert tz.size >= 4
    half = np.diff(tz)
    return math.pi / (np.mean(half) * dt)


def test_total_momentum_conserved():
    tree = oracle.OracleTree(W.regular_tree(2, 3))
    wl = W.config1()
    p0 = wl.v.sum(axis=1)
    x, v = oracle.langmuir_run(tree, wl.x, wl.v, wl.qm * 0.2, 0.2, 10, wl.q_uniform)
    # the first half kick and ten full kicks must all cancel to rounding
    assert np.all(np.abs(v.sum(axis=1) - p0) <= 1e-12 * np.abs(wl.v).sum())


def _cold_setup(L, per_axis, delta):
    n = 3 ** L * per_axis
    g = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(g, g, indexing="xy")
    x = np.stack([X.ravel(), Y.ravel()])
    x[0] = (x[0] + delta * np.sin(2 * np.pi * x[0])) % 1.0
    return x, np.zeros_like(x)


@pytest.mark.slow
@pytest.mark.parametrize("wdt", [0.5, 1.0])
def test_cold_plasma_oscillates_at_leapfrog_plasma_frequency(wdt):
    L = 4
    tree = oracle.OracleTree(W.regular_tree(2, L))
    x, v = _cold_setup(L, 2, 1e-3)
    n = x.shape[1]
    steps = int(round(8 * 2 * math.pi / wdt))
    amp = _mode_series(tree, x, v, -wdt, wdt, steps, -1.0 / n)
    w = _frequency(amp, wdt)
    theta = 2 * math.pi / 3 ** L
    grid = math.sqrt((math.sin(theta / 2) / (theta / 2)) ** 3 * math.cos(theta / 2))
    want = 2.0 / wdt * math.asin(wdt * grid / 2.0)
    assert abs(w / want - 1.0) < 3e-3, (w, want)


def _golden(name):
    vals = {}
    for ln in open(os.path.join(GOLDEN, name)):
        if ln.strip() and not ln.startswith("#"):
            k, v = ln.split()
            vals[k] = float(v)
    return vals


@pytest.mark.slow
@pytest.mark.parametrize("klam,tol", [(0.1, 0.02), (0.2, 0.02), (0.3, 0.04)])
def test_bohm_gross_dispersion(klam, tol):
    g = _golden("langmuir_appendix.txt")
    assert g["charge_to_mass"] == -1 and g["electron_density"] == -1
    L = 4
    tree = oracle.OracleTree(W.regular_tree(2, L))
    rng = np.random.default_rng(100 + int(klam * 10))
    lam = klam / (2 * math.pi)                 # k = 2 pi (first box mode), omega_p = 1
    n = 3 ** (2 * L) * 12
    x = np.stack([rng.random(n), rng.random(n)])
    x[0] = (x[0] + 0.05 / (2 * math.pi) * np.sin(2 * math.pi * x[0])) % 1.0
    v = rng.standard_normal((2, n)) * lam       # v_th = lambda_D omega_p
    dt = 0.2
    steps = int(6 * 2 * math.pi / dt)
    amp = _mode_series(tree, x, v, g["charge_to_mass"] * dt, dt, steps, -1.0 / n)
    w = _frequency(amp, dt)
    w_leap = 2.0 / dt * math.sin(w * dt / 2.0)  # undo the leapfrog frequency shift
    want = math.sqrt(1.0 + 3.0 * klam ** 2)
    assert abs(w_leap / want - 1.0) < tol, (w_leap, want)


def test_fig16_ring_is_bohm_gross():
    """The fixed-frequency cut of Fig. 16 lies on |k| lambda_D = sqrt((w^2-1)/3)."""
    g = _golden("langmuir_appendix.txt")
    klam = math.sqrt((g["ring_frequency"] ** 2 - 1.0) / 3.0)
    assert 0.31 < klam < 0.32


@pytest.mark.parametrize("dim,L", [(2, 2), (2, 3), (3, 2)])
def test_dual_cells_nest_along_the_curve(dim, L):
    """Dual-grid consistency for odd k (Sec. 4.1, dual spacetree grid).

    The level-L vertices inside the dual cell of one level-(L-1) vertex B
    (that is b = 3B + {-1,0,1}^d) must occupy 3^d consecutive PIDT ranks.
    """
    fine = oracle.OracleTree(W.regular_tree(dim, L))
    b = fine.pidt_bins()["b"]
    S = fine.S
    rank = {tuple(map(int, bb)): r for r, bb in enumerate(b)}
    for B in itertools.product(range(3 ** (L - 1)), repeat=dim):
        ranks = sorted(rank[tuple((3 * B[k] + o[k]) % S for k in range(dim))]
                       for o in itertools.product((-1, 0, 1), repeat=dim))
        assert ranks[-1] - ranks[0] == 3 ** dim - 1, (B, ranks)


def test_scaled_position_never_reaches_the_box_size():
    """For S = 3^L the product fl(x*S) stays below S for every double x < 1.

    The largest double below one is 1 - 2^-53; x*S then lies S*2^-53 below S,
    which is more than half the spacing of doubles just below S (S is not a
    power of two).  So the clamp of the cell index to S-1 never acts on valid
    input; it only keeps malformed input in range.
    """
    x = np.nextafter(1.0, 0.0)
    for L in range(0, 19):
        S = float(3 ** L)
        assert x * S < S
