"""GPU parity of the HIP hot path against the oracle (FP64 form).

Bar: bins, order and bin offsets bit-exact; x, v and the gathered field
bit-exact (the kernels follow the same IEEE operation sequence without
contraction); vertex charge within 1e-12 relative per vertex (all terms of a
vertex share one sign, so any summation order stays within (n-1) u).
Every call goes through libpic.so's C ABI via the Python binding.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1508_02435_amd as pic  # noqa: E402

CASES = [("config1", 0), ("config1", 1), ("small_adaptive", 0), ("small_adaptive", 1),
         ("small_3d", 0), ("small_3d", 1), ("small_3d_adaptive", 0), ("small_3d_adaptive", 1)]
RHO_TOL = 1e-12


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda")


def _tree(spec):
    return pic.Tree(spec).upload()


def _field(o, wl, rng, kind):
    if kind == "random":
        # a few cells of displacement per step: tunnelling in every direction
        scale = 3.0 * wl.h / (wl.dt * wl.dt)
        return W.random_field(rng, wl.dim, o.n_vertices, scale)
    return wl.field(o.vertex_positions_unit())


def _check_rho(rho_gpu, rho_orc):
    err = np.abs(rho_gpu - rho_orc)
    ok = err <= RHO_TOL * np.abs(rho_orc) + 1e-300
    assert ok.all(), (err.max(), np.abs(rho_orc).max(), int((~ok).sum()))


@pytest.mark.parametrize("name,scheme", CASES)
def test_locate_matches_oracle(name, scheme):
    dev = _dev()
    wl = W.by_name(name)
    o = oracle.OracleTree(wl.tree)
    t = _tree(wl.tree)
    x = torch.tensor(wl.x, dtype=torch.float64, device=dev)
    b = torch.empty(wl.n, dtype=torch.int32, device=dev)
    pic.locate(t, scheme, x, b)
    torch.cuda.synchronize()
    assert np.array_equal(b.cpu().numpy(), o.bin_of(wl.x, scheme))
    assert t.status_sync() == 0


@pytest.mark.parametrize("kind", ["random", "physical"])
@pytest.mark.parametrize("name,scheme", CASES)
def test_step_matches_oracle(name, scheme, kind):
    """Initial sort, then three teacher-forced steps: every output compared."""
    dev = _dev()
    wl = W.by_name(name)
    o = oracle.OracleTree(wl.tree)
    t = _tree(wl.tree)
    rng = np.random.default_rng(99)
    ids = np.arange(wl.n, dtype=np.int64)
    st = pic.Stepper(t, scheme, wl.x, wl.v, q=wl.q, ids=ids, device=dev)
    st.initial_sort()
    # oracle initial sort
    nb0 = o.bin_of(wl.x, scheme)
    perm, start = oracle.rebin(nb0, o.n_bins(scheme), None)
    torch.cuda.synchronize()
    assert np.array_equal(st.ids.cpu().numpy(), perm)
    assert np.array_equal(st.start.cpu().numpy(), start)
    x, v = wl.x[:, perm], wl.v[:, perm]
    q = None if wl.q is None else wl.q[perm]
    for it in range(3):
        E = _field(o, wl, rng, kind)
        Ed = torch.tensor(E, dtype=torch.float64, device=dev)
        qmdt, dt = wl.qm * wl.dt, wl.dt
        # teacher forcing: the GPU starts every step from the oracle's state
        st.x.copy_(torch.from_numpy(x))
        st.v.copy_(torch.from_numpy(v))
        st.gather_push(Ed, qmdt, dt, want_Ep=True)
        x1, v1, ep, nb = o.gather_push(x, v, E, qmdt, dt, scheme)
        torch.cuda.synchronize()
        assert np.array_equal(st.x.cpu().numpy(), x1), f"x differs at step {it}"
        assert np.array_equal(st.v.cpu().numpy(), v1), f"v differs at step {it}"
        assert np.array_equal(st.Ep.cpu().numpy(), ep), f"E_p differs at step {it}"
        assert np.array_equal(st.bin.cpu().numpy(), nb), f"bins differ at step {it}"
        ids_before = st.ids.cpu().numpy()
        st.rebin()
        perm, start2 = oracle.rebin(nb, o.n_bins(scheme), start)
        torch.cuda.synchronize()
        assert np.array_equal(st.start.cpu().numpy(), start2), f"bin_start differs at step {it}"
        assert np.array_equal(st.ids.cpu().numpy(), ids_before[perm]), f"order differs at step {it}"
        x, v, start = x1[:, perm], v1[:, perm], start2
        q = None if q is None else q[perm]
        assert np.array_equal(st.x.cpu().numpy(), x)
        st.deposit(wl.q_uniform)
        rho = o.deposit(x, q, wl.q_uniform)
        torch.cuda.synchronize()
        _check_rho(st.rho.cpu().numpy(), rho)
    assert t.status_sync() == 0


@pytest.mark.parametrize("scheme", [0, 1])
def test_deposit_is_bitwise_deterministic(scheme):
    dev = _dev()
    wl = W.config1()
    t = _tree(wl.tree)
    outs = []
    for _ in range(2):
        st = pic.Stepper(t, scheme, wl.x, wl.v, device=dev)
        st.initial_sort()
        st.deposit(wl.q_uniform)
        outs.append(st.rho.cpu().numpy().copy())
    assert np.array_equal(outs[0].view(np.uint64), outs[1].view(np.uint64))


def _synthetic(n, dim, rng, kind):
    if kind == "one_cell":              # every particle in one cell: one segment over many tiles
        x = 0.4 + 0.001 * rng.random((dim, n))
    elif kind == "faces":               # on cell faces, half cells and the box edge
        g = np.array([0.0, np.nextafter(1.0, 0.0), 1 / 3, 2 / 9, 0.5, 1 / 6, np.nextafter(1 / 3, 0.0)])
        x = g[rng.integers(0, g.size, (dim, n))]
    else:
        x = rng.random((dim, n))
    return x, rng.standard_normal((dim, n)) * 0.05


@pytest.mark.parametrize("n", [0, 1, 63, 4095, 4096, 4097, 3 * 4096 + 17])
@pytest.mark.parametrize("kind", ["uniform", "one_cell", "faces"])
@pytest.mark.parametrize("scheme", [0, 1])
def test_edge_sizes_and_positions(n, kind, scheme):
    dev = _dev()
    rng = np.random.default_rng(n + 7)
    spec = W.disc_tree(2, 2, 4)
    o = oracle.OracleTree(spec)
    t = _tree(spec)
    x, v = _synthetic(n, 2, rng, kind)
    ids = np.arange(n, dtype=np.int64)
    st = pic.Stepper(t, scheme, x, v, ids=ids, device=dev)
    st.initial_sort()
    nb0 = o.bin_of(x, scheme) if n else np.zeros(0, np.int32)
    perm, start = oracle.rebin(nb0, o.n_bins(scheme), None)
    torch.cuda.synchronize()
    assert np.array_equal(st.ids.cpu().numpy(), perm)
    assert np.array_equal(st.start.cpu().numpy(), start)
    E = W.random_field(rng, 2, o.n_vertices, 0.3)
    Ed = torch.tensor(E, dtype=torch.float64, device=dev)
    xs, vs = x[:, perm], v[:, perm]
    st.step(Ed, -0.7, 0.7, q_uniform=-1.0)
    x1, v1, _, nb = o.gather_push(xs, vs, E, -0.7, 0.7, scheme)
    perm2, start2 = oracle.rebin(nb, o.n_bins(scheme), start)
    rho = o.deposit(x1[:, perm2], None, -1.0)
    torch.cuda.synchronize()
    assert np.array_equal(st.start.cpu().numpy(), start2)
    assert np.array_equal(st.x.cpu().numpy(), x1[:, perm2])
    assert np.array_equal(st.v.cpu().numpy(), v1[:, perm2])
    _check_rho(st.rho.cpu().numpy(), rho)
    assert t.status_sync() == 0


@pytest.mark.parametrize("n", [0, 1, 63, 4095, 4096, 4097, 3 * 4096 + 17])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("scheme", [0, 1])
def test_fused_step_edge_sizes_with_default_launch_shape(n, dim, scheme):
    """pic_step with the default knobs on regular trees, at empty, tiny and
    tile-boundary sizes: in 3D (few particles per bin) the 4096-particle
    tiles, in 2D the 2048-particle tiles and, for PIT, the writing-pass
    deposit.  Offsets, state and order bit for bit; charge within 1e-12."""
    dev = _dev()
    rng = np.random.default_rng(n + 11 * dim + scheme)
    spec = W.regular_tree(dim, 2 if dim == 3 else 3)
    o = oracle.OracleTree(spec)
    t = _tree(spec)
    x, v = _synthetic(n, dim, rng, "uniform")
    st = pic.Stepper(t, scheme, x, v, ids=np.arange(n, dtype=np.int64), device=dev)
    st.initial_sort()
    xs, vs, _, start, ids = oracle.initial_sort(o, x, v, None, scheme)
    E = W.random_field(rng, dim, o.n_vertices, 0.3)
    st.step_fused(torch.tensor(E, dtype=torch.float64, device=dev), -0.7, 0.7, q_uniform=-1.0)
    r = oracle.step(o, xs, vs, E, -0.7, 0.7, start, scheme, None, -1.0)
    torch.cuda.synchronize()
    assert np.array_equal(st.start.cpu().numpy(), r["bin_start"])
    assert np.array_equal(st.ids.cpu().numpy(), ids[r["perm"]])
    assert np.array_equal(st.x.cpu().numpy(), r["x"]) and np.array_equal(st.v.cpu().numpy(), r["v"])
    _check_rho(st.rho.cpu().numpy(), r["rho"])
    assert t.status_sync() == 0


def test_nonfinite_and_out_of_box_are_flagged_not_fatal():
    dev = _dev()
    spec = W.regular_tree(2, 3)
    t = _tree(spec)
    rng = np.random.default_rng(3)
    x = rng.random((2, 1000))
    v = np.zeros((2, 1000))
    v[0, 10] = np.nan
    st = pic.Stepper(t, 0, x, v, device=dev)
    st.initial_sort()
    E = torch.zeros((2, t.n_vertices), dtype=torch.float64, device=dev)
    st.step(E, -0.1, 0.1, q_uniform=-1.0)
    torch.cuda.synchronize()
    assert t.status_sync() == pic._capi.PIC_E_NONFINITE
    assert t.status_sync() == 0                       # cleared
    xb = torch.tensor(np.array([[0.5, 1.5], [0.5, 0.5]]), device=dev)
    b = torch.empty(2, dtype=torch.int32, device=dev)
    pic.locate(t, 0, xb, b)
    assert t.status_sync() == pic._capi.PIC_E_RANGE
    assert int(b.max()) < t.n_leaves


def test_forest_locate_and_step_match_oracle_per_instance():
    dev = _dev()
    insts = W.config5(n_inst=5, n_min=2e3, n_max=3e4)
    specs = [w.tree for w in insts]
    t = _tree(specs)
    counts = [w.n for w in insts]
    inst_start = torch.tensor(np.concatenate([[0], np.cumsum(counts)]), dtype=torch.int64, device=dev)
    x = np.concatenate([w.x for w in insts], axis=1)
    v = np.concatenate([w.v for w in insts], axis=1)
    for scheme in (0, 1):
        st = pic.Stepper(t, scheme, x, v, ids=np.arange(x.shape[1]), inst_start=inst_start, device=dev)
        st.initial_sort()
        rng = np.random.default_rng(5)
        Es, qmdt, dts = [], [], []
        for i, w in enumerate(insts):
            o = oracle.OracleTree(w.tree)
            Es.append(W.random_field(rng, 2, o.n_vertices, 2.0 * w.h / w.dt ** 2))
            qmdt.append(w.qm * w.dt)
            dts.append(w.dt)
        E = torch.tensor(np.concatenate(Es, axis=1), dtype=torch.float64, device=dev)
        qd = torch.tensor(qmdt, dtype=torch.float64, device=dev)
        dd = torch.tensor(dts, dtype=torch.float64, device=dev)
        xs0 = st.x.cpu().numpy().copy()
        vs0 = st.v.cpu().numpy().copy()
        st.gather_push(E, 0.0, 0.0, qmdt_dev=qd, dt_dev=dd)
        torch.cuda.synchronize()
        xg, vg, bg = st.x.cpu().numpy(), st.v.cpu().numpy(), st.bin.cpu().numpy()
        p0 = 0
        for i, w in enumerate(insts):
            o = oracle.OracleTree(w.tree)
            ii = t.instance(i)
            sl = slice(p0, p0 + w.n)
            x1, v1, _, nb = o.gather_push(xs0[:, sl], vs0[:, sl], Es[i], qmdt[i], dts[i], scheme)
            assert np.array_equal(xg[:, sl], x1) and np.array_equal(vg[:, sl], v1)
            off = ii.leaf_offset if scheme == 0 else ii.pidt_offset
            assert np.array_equal(bg[sl], nb + off)
            p0 += w.n
        st.rebin()
        st.deposit(-1.0)
        torch.cuda.synchronize()
        # instance by instance the forest result equals the single-tree oracle
        xs, starts = st.x.cpu().numpy(), st.start.cpu().numpy()
        rho = st.rho.cpu().numpy()
        p0 = 0
        for i, w in enumerate(insts):
            o = oracle.OracleTree(w.tree)
            ii = t.instance(i)
            off = ii.leaf_offset if scheme == 0 else ii.pidt_offset
            nbi = o.n_bins(scheme)
            assert np.array_equal(starts[off:off + nbi + 1] - p0, oracle.rebin(
                o.bin_of(xs[:, p0:p0 + w.n], scheme), nbi, None)[1])
            _check_rho(rho[ii.vertex_offset:ii.vertex_offset + ii.n_vertices],
                       o.deposit(xs[:, p0:p0 + w.n], None, -1.0))
            p0 += w.n
        assert t.status_sync() == 0


KNOB_SETS = ([dict(rebin_tile=t, rebin_radix=r, scatter_mode=m, scatter_nt=nt)
              for t in (2048, 4096) for r in (4, 5) for m in (0, 1) for nt in (0, 1)]
             + [dict(scatter_group=g, deposit_lanes=d) for g in (1, 2, 4) for d in (16, 32, 64)]
             + [dict(deposit_batch=b, deposit_lanes=d) for b in (64, 256) for d in (16, 32, 64)])


@pytest.mark.parametrize("knobs", KNOB_SETS, ids=lambda k: "-".join(f"{v}" for v in k.values()))
@pytest.mark.parametrize("name,scheme", [("config1", 0), ("small_adaptive", 1)])
def test_every_launch_shape_gives_the_same_step(name, scheme, knobs):
    dev = _dev()
    saved = pic.tuning()
    try:
        for k, v in knobs.items():
            pic.tune(k, v)
        wl = W.by_name(name)
        o = oracle.OracleTree(wl.tree)
        t = _tree(wl.tree)
        rng = np.random.default_rng(17)
        st = pic.Stepper(t, scheme, wl.x, wl.v, q=wl.q, ids=np.arange(wl.n), device=dev)
        st.initial_sort()
        xs, vs, qs, start, perm = oracle.initial_sort(o, wl.x, wl.v, wl.q, scheme)
        E = _field(o, wl, rng, "random")
        st.step(torch.tensor(E, device=dev), wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
        r = oracle.step(o, xs, vs, E, wl.qm * wl.dt, wl.dt, start, scheme, qs, wl.q_uniform)
        torch.cuda.synchronize()
        assert np.array_equal(st.start.cpu().numpy(), r["bin_start"])
        assert np.array_equal(st.ids.cpu().numpy(), perm[r["perm"]])
        assert np.array_equal(st.x.cpu().numpy(), r["x"])
        _check_rho(st.rho.cpu().numpy(), r["rho"])
        assert t.status_sync() == 0
    finally:
        for k, v in saved.items():
            pic.tune(k, v)


@pytest.mark.parametrize("kind", ["random", "physical"])
@pytest.mark.parametrize("name,scheme", CASES)
def test_fused_step_matches_oracle(name, scheme, kind):
    """pic_step (fused kernels) against the oracle over three teacher-forced steps."""
    dev = _dev()
    wl = W.by_name(name)
    o = oracle.OracleTree(wl.tree)
    t = _tree(wl.tree)
    rng = np.random.default_rng(98)
    st = pic.Stepper(t, scheme, wl.x, wl.v, q=wl.q, ids=np.arange(wl.n, dtype=np.int64), device=dev)
    st.initial_sort()
    xs, vs, qs, start, perm = oracle.initial_sort(o, wl.x, wl.v, wl.q, scheme)
    ids = perm
    for it in range(3):
        E = _field(o, wl, rng, kind)
        st.x.copy_(torch.from_numpy(xs))
        st.v.copy_(torch.from_numpy(vs))
        st.step_fused(torch.tensor(E, device=dev), wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
        r = oracle.step(o, xs, vs, E, wl.qm * wl.dt, wl.dt, start, scheme, qs, wl.q_uniform)
        torch.cuda.synchronize()
        assert np.array_equal(st.start.cpu().numpy(), r["bin_start"]), f"offsets differ at step {it}"
        ids = ids[r["perm"]]
        assert np.array_equal(st.ids.cpu().numpy(), ids), f"order differs at step {it}"
        assert np.array_equal(st.x.cpu().numpy(), r["x"]) and np.array_equal(st.v.cpu().numpy(), r["v"])
        if qs is not None:
            assert np.array_equal(st.q.cpu().numpy(), r["q"])
        _check_rho(st.rho.cpu().numpy(), r["rho"])
        xs, vs, qs, start = r["x"], r["v"], r["q"], r["bin_start"]
    assert t.status_sync() == 0


STEP_FORMS = [dict(step_fuse=f, group_match=gm, emit_threads=nt, xcd_tiles=x, step_tile=tl, emit_deposit=dep)
              for f, gm in ((1, 0), (0, 0), (0, 1)) for nt in (1024, 512) for x in (1, 0) for tl in (2048, 1024)
              for dep in (1, 0)]
STEP_FORMS += [dict(step_fuse=0, group_match=0, emit_threads=nt, xcd_tiles=1, step_tile=tl, emit_deposit=dep,
                    key_stores=1) for nt in (1024, 512) for tl in (2048, 1024) for dep in (1, 0)]
# 4096-particle tiles: one staged column at a time, whatever step_fuse and
# emit_deposit say
STEP_FORMS += [dict(step_fuse=f, group_match=gm, emit_threads=nt, xcd_tiles=x, step_tile=4096, emit_deposit=1,
                    key_stores=ks) for f, gm in ((1, 0), (0, 0), (0, 1)) for nt in (1024, 512) for x in (1, 0)
               for ks in (0, 1)]


@pytest.mark.parametrize("knobs", STEP_FORMS, ids=lambda k: "-".join(f"{v}" for v in k.values()))
@pytest.mark.parametrize("name,scheme", [("config1", 0), ("small_adaptive", 1), ("small_3d", 0)])
def test_fused_step_forms_match_oracle(name, scheme, knobs):
    """Every pass form and launch shape of pic_step: two teacher-forced steps
    against the oracle (bins, order, state bit-exact; charge within 1e-12)."""
    dev = _dev()
    saved = pic.tuning()
    try:
        for k, v in knobs.items():
            pic.tune(k, v)
        wl = W.by_name(name)
        o = oracle.OracleTree(wl.tree)
        t = _tree(wl.tree)
        rng = np.random.default_rng(5)
        st = pic.Stepper(t, scheme, wl.x, wl.v, q=wl.q, ids=np.arange(wl.n, dtype=np.int64), device=dev)
        st.initial_sort()
        xs, vs, qs, start, ids = oracle.initial_sort(o, wl.x, wl.v, wl.q, scheme)
        for it, kind in enumerate(("random", "physical")):
            E = _field(o, wl, rng, kind)
            st.step_fused(torch.tensor(E, device=dev), wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
            r = oracle.step(o, xs, vs, E, wl.qm * wl.dt, wl.dt, start, scheme, qs, wl.q_uniform)
            torch.cuda.synchronize()
            ids = ids[r["perm"]]
            assert np.array_equal(st.start.cpu().numpy(), r["bin_start"]), f"offsets differ at step {it}"
            assert np.array_equal(st.ids.cpu().numpy(), ids), f"order differs at step {it}"
            assert np.array_equal(st.x.cpu().numpy(), r["x"]) and np.array_equal(st.v.cpu().numpy(), r["v"])
            _check_rho(st.rho.cpu().numpy(), r["rho"])
            xs, vs, qs, start = r["x"], r["v"], r["q"], r["bin_start"]
        assert t.status_sync() == 0
    finally:
        for k, v in saved.items():
            pic.tune(k, v)


@pytest.mark.parametrize("tiles", [12, 80, 160])
@pytest.mark.parametrize("step_fuse,group_match", [(1, 0), (0, 1), (0, 0)])
@pytest.mark.parametrize("step_tile", [2048, 1024, 4096])
@pytest.mark.parametrize("scheme", [0, 1])
def test_fused_step_with_overfull_key_lists(step_tile, step_fuse, group_match, scheme, tiles):
    """Every tile sends particles to every bin of a 3x3 tree, so each key
    collects about as many runs as there are tiles: 12 are placed by 16-lane
    groups (more than the 8 lanes a key starts with; 2048-particle tiles),
    80 by counting (more than a wavefront sorts), 160 overflow the direct
    list into the linked rest.  The step still matches the oracle."""
    dev = _dev()
    saved = pic.tuning()
    try:
        pic.tune("step_tile", step_tile)
        pic.tune("step_fuse", step_fuse)
        pic.tune("group_match", group_match)
        rng = np.random.default_rng(31)
        spec = W.regular_tree(2, 1)
        n = tiles * 2048 + 77
        x, v = rng.random((2, n)), rng.standard_normal((2, n)) * 0.4
        o = oracle.OracleTree(spec)
        t = _tree(spec)
        E = W.random_field(rng, 2, o.n_vertices, 0.5)
        st = pic.Stepper(t, scheme, x, v, ids=np.arange(n, dtype=np.int64), device=dev)
        st.initial_sort()
        xs, vs, _, start, ids = oracle.initial_sort(o, x, v, None, scheme)
        st.step_fused(torch.tensor(E, device=dev), -0.9, 0.9, q_uniform=-1.0)
        r = oracle.step(o, xs, vs, E, -0.9, 0.9, start, scheme, None, -1.0)
        torch.cuda.synchronize()
        # the case is the one meant: the most runs a key collects
        old_bin = np.repeat(np.arange(len(start) - 1), np.diff(start))
        new_bin = np.asarray(r["new_bin"], dtype=np.int64)
        key = 2 * new_bin + (new_bin != old_bin)
        pairs = np.unique(key * (n // step_tile + 1) + np.arange(n) // step_tile)
        most = np.bincount(pairs // (n // step_tile + 1)).max()
        if tiles == 12 and step_tile == 2048:
            assert 8 < most <= 16
        assert most <= (n + step_tile - 1) // step_tile
        assert np.array_equal(st.start.cpu().numpy(), r["bin_start"])
        assert np.array_equal(st.ids.cpu().numpy(), ids[r["perm"]])
        assert np.array_equal(st.x.cpu().numpy(), r["x"]) and np.array_equal(st.v.cpu().numpy(), r["v"])
        _check_rho(st.rho.cpu().numpy(), r["rho"])
        assert t.status_sync() == 0
    finally:
        for k, v in saved.items():
            pic.tune(k, v)


MANY_RUN_FORMS = [dict(), dict(emit_threads=512), dict(step_tile=1024), dict(step_tile=1024, emit_threads=512),
                  dict(step_fuse=1), dict(step_fuse=1, step_tile=1024), dict(group_match=1),
                  dict(group_match=1, step_tile=1024), dict(step_tile=4096), dict(step_tile=4096, emit_threads=512),
                  dict(step_tile=4096, group_match=1)]


@pytest.mark.parametrize("knobs", MANY_RUN_FORMS, ids=lambda k: "-".join(f"{a}{b}" for a, b in k.items()) or "default")
@pytest.mark.parametrize("scheme", [0, 1])
def test_fused_step_with_many_runs_per_tile(scheme, knobs):
    """A thermal spread of half the box scatters each sorted tile over a 27x27
    tree, so tiles hold several hundred runs: more than the head of the run
    table that the writing pass loads with the state.  The step still
    matches the oracle."""
    dev = _dev()
    saved = pic.tuning()
    try:
        for k, v in knobs.items():
            pic.tune(k, v)
        tile = pic.tuning()["step_tile"] or 2048   # 0: by dimension, 2048 for 2D trees
        rng = np.random.default_rng(47)
        spec = W.regular_tree(2, 3)
        n = 5 * 2048 + 333
        x, v = rng.random((2, n)), rng.standard_normal((2, n)) * 0.5
        o = oracle.OracleTree(spec)
        t = _tree(spec)
        E = W.random_field(rng, 2, o.n_vertices, 0.5)
        st = pic.Stepper(t, scheme, x, v, ids=np.arange(n, dtype=np.int64), device=dev)
        st.initial_sort()
        xs, vs, _, start, ids = oracle.initial_sort(o, x, v, None, scheme)
        st.step_fused(torch.tensor(E, device=dev), -0.9, 0.9, q_uniform=-1.0)
        r = oracle.step(o, xs, vs, E, -0.9, 0.9, start, scheme, None, -1.0)
        torch.cuda.synchronize()
        # the case is the one meant: some tile has more than 256 (tile, key) runs
        old_bin = np.repeat(np.arange(len(start) - 1), np.diff(start))
        new_bin = np.asarray(r["new_bin"], dtype=np.int64)
        key = 2 * new_bin + (new_bin != old_bin)
        runs = [len(np.unique(key[a:a + tile])) for a in range(0, n, tile)]
        assert max(runs) > 256
        assert np.array_equal(st.start.cpu().numpy(), r["bin_start"])
        assert np.array_equal(st.ids.cpu().numpy(), ids[r["perm"]])
        assert np.array_equal(st.x.cpu().numpy(), r["x"]) and np.array_equal(st.v.cpu().numpy(), r["v"])
        _check_rho(st.rho.cpu().numpy(), r["rho"])
        assert t.status_sync() == 0
    finally:
        for k, v in saved.items():
            pic.tune(k, v)


@pytest.mark.parametrize("spread", [0.05, 0.5])
@pytest.mark.parametrize("step_tile", [2048, 1024, 4096])
@pytest.mark.parametrize("n", [1, 1023, 2047, 2048, 2049, 4097, 5 * 2048 + 3])
def test_fused_and_separate_calls_agree_bitwise(n, step_tile, spread):
    """spread 0.5 scatters a tile over most of the tree's bins, so tiles hold
    far more distinct keys than the fast rank path takes."""
    dev = _dev()
    before = pic.tuning()["step_tile"]
    pic.tune("step_tile", step_tile)
    try:
        _fused_vs_separate(n, dev, spread)
    finally:
        pic.tune("step_tile", before)


def _fused_vs_separate(n, dev, spread):
    rng = np.random.default_rng(n)
    spec = W.disc_tree(2, 2, 4)
    t = _tree(spec)
    x, v = rng.random((2, n)), rng.standard_normal((2, n)) * spread
    E = torch.tensor(W.random_field(rng, 2, t.n_vertices, 0.3), device=dev)
    outs = []
    for fused in (False, True):
        st = pic.Stepper(t, 1, x, v, ids=np.arange(n), device=dev)
        st.initial_sort()
        for _ in range(2):
            (st.step_fused if fused else st.step)(E, -0.7, 0.7, q_uniform=-1.0)
        torch.cuda.synchronize()
        outs.append([a.cpu().numpy().copy() for a in (st.x, st.v, st.ids, st.start, st.rho)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name,scheme", [("config1", 0), ("config1", 1), ("small_3d", 0), ("small_3d", 1)])
def test_regular_tree_without_tables_matches_oracle(name, scheme):
    """Regular trees too large for Peano tables take the descent kernels;
    tables switched off exercise that path on small trees."""
    dev = _dev()
    wl = W.by_name(name)
    before = pic.tuning()["regular_tables"]
    pic.tune("regular_tables", 0)
    try:
        t = _tree(wl.tree)
    finally:
        pic.tune("regular_tables", before)
    assert pic.scratch_bytes(t, wl.n, scheme, pic.F32_OFFSET) == 0      # no tables: no FP32 form either
    o = oracle.OracleTree(wl.tree)
    rng = np.random.default_rng(21)
    st = pic.Stepper(t, scheme, wl.x, wl.v, ids=np.arange(wl.n), device=dev)
    st.initial_sort()
    xs, vs, qs, start, perm = oracle.initial_sort(o, wl.x, wl.v, wl.q, scheme)
    ids = perm
    for it in range(2):
        E = _field(o, wl, rng, "random")
        st.step_fused(torch.tensor(E, device=dev), wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
        r = oracle.step(o, xs, vs, E, wl.qm * wl.dt, wl.dt, start, scheme, qs, wl.q_uniform)
        torch.cuda.synchronize()
        ids = ids[r["perm"]]
        assert np.array_equal(st.start.cpu().numpy(), r["bin_start"])
        assert np.array_equal(st.ids.cpu().numpy(), ids)
        assert np.array_equal(st.x.cpu().numpy(), r["x"]) and np.array_equal(st.v.cpu().numpy(), r["v"])
        _check_rho(st.rho.cpu().numpy(), r["rho"])
        xs, vs, qs, start = r["x"], r["v"], r["q"], r["bin_start"]
    assert t.status_sync() == 0


def _add_stats(acc, st):
    if acc is None:
        return dict(st, lift_hist=list(st["lift_hist"]))
    for k in ("particles", "movers", "lifts"):
        acc[k] += st[k]
    acc["max_tunnel"] = max(acc["max_tunnel"], st["max_tunnel"])
    acc["lift_hist"] = [a + b for a, b in zip(acc["lift_hist"], st["lift_hist"])]
    return acc


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("name,scheme", CASES)
def test_rebin_stats_match_oracle(name, scheme, fused):
    """Re-bin statistics (movers, lifts per particle, the lift-count
    histogram and the largest tunnel distance, paper Sec. 6.1) of pic_rebin
    and of pic_step, accumulated over three teacher-forced steps with
    tunnelling fields, equal the oracle's bit for bit."""
    dev = _dev()
    wl = W.by_name(name)
    o = oracle.OracleTree(wl.tree)
    t = _tree(wl.tree)
    rng = np.random.default_rng(61)
    st = pic.Stepper(t, scheme, wl.x, wl.v, q=wl.q, device=dev)
    st.initial_sort()
    xs, vs, qs, start, _ = oracle.initial_sort(o, wl.x, wl.v, wl.q, scheme)
    stats = pic.new_stats(dev)
    want = None
    for it in range(3):
        E = _field(o, wl, rng, "random")
        st.x.copy_(torch.from_numpy(xs))
        st.v.copy_(torch.from_numpy(vs))
        (st.step_fused if fused else st.step)(torch.tensor(E, device=dev), wl.qm * wl.dt, wl.dt,
                                              q_uniform=wl.q_uniform, stats=stats)
        r = oracle.step(o, xs, vs, E, wl.qm * wl.dt, wl.dt, start, scheme, qs, wl.q_uniform)
        want = _add_stats(want, o.rebin_stats(start, r["new_bin"], scheme))
        xs, vs, qs, start = r["x"], r["v"], r["q"], r["bin_start"]
    torch.cuda.synchronize()
    got = pic.read_stats(stats)
    assert want["movers"] > 0 and max(i for i, c in enumerate(want["lift_hist"]) if c) >= 2
    assert got == want
    assert t.status_sync() == 0


def test_forest_stats_match_oracle_per_instance_sum():
    """A forest's statistics are the sums (and the largest tunnel) of its
    instances' statistics taken one by one by the oracle."""
    dev = _dev()
    insts = W.config5(n_inst=6, n_min=2e3, n_max=3e4)
    t = _tree([w.tree for w in insts])
    counts = [w.n for w in insts]
    inst_start = torch.tensor(np.concatenate([[0], np.cumsum(counts)]), dtype=torch.int64, device=dev)
    orc = [oracle.OracleTree(w.tree) for w in insts]
    rng = np.random.default_rng(8)
    Es = [W.random_field(rng, 2, o.n_vertices, 2.0 * w.h / w.dt ** 2) for w, o in zip(insts, orc)]
    E = torch.tensor(np.concatenate(Es, axis=1), device=dev)
    qd = torch.tensor([w.qm * w.dt for w in insts], dtype=torch.float64, device=dev)
    dd = torch.tensor([w.dt for w in insts], dtype=torch.float64, device=dev)
    for scheme in (0, 1):
        x = np.concatenate([w.x for w in insts], axis=1)
        v = np.concatenate([w.v for w in insts], axis=1)
        st = pic.Stepper(t, scheme, x, v, inst_start=inst_start, device=dev)
        st.initial_sort()
        stats = pic.new_stats(dev)
        st.step_fused(E, 0.0, 0.0, q_uniform=-1.0, qmdt_dev=qd, dt_dev=dd, stats=stats)
        want = None
        for i, (w, o) in enumerate(zip(insts, orc)):
            xs, vs, _, start, _ = oracle.initial_sort(o, w.x, w.v, None, scheme)
            r = oracle.step(o, xs, vs, Es[i], w.qm * w.dt, w.dt, start, scheme, None, -1.0)
            want = _add_stats(want, o.rebin_stats(start, r["new_bin"], scheme))
        torch.cuda.synchronize()
        assert pic.read_stats(stats) == want
        assert t.status_sync() == 0


@pytest.mark.parametrize("emit_threads", [1024, 512])
@pytest.mark.parametrize("step_tile", [2048, 1024])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 1023, 2048, 2049, 9000])
@pytest.mark.parametrize("scheme", [0, 1])
def test_writing_pass_deposit_with_long_runs_and_ragged_tiles(scheme, n, step_tile, emit_threads):
    """The writing pass's deposit on a regular 2D tree: half the particles
    sit in one cell with slow velocities, so each tile holds a run of stayers
    that spans several wavefronts (and whole tiles), the rest are spread over
    the tree; ragged last tiles and sets smaller than a wavefront.  The
    charge equals the oracle's within 1e-12 per vertex, the state bit for
    bit, and the separate deposit gives the same charge to rounding."""
    dev = _dev()
    saved = pic.tuning()
    try:
        pic.tune("step_tile", step_tile)
        pic.tune("emit_threads", emit_threads)
        rng = np.random.default_rng(n * 3 + scheme)
        spec = W.regular_tree(2, 2)
        o = oracle.OracleTree(spec)
        half = n // 2
        x = np.concatenate([0.40 + 0.02 * rng.random((2, half)), rng.random((2, n - half))], axis=1)
        v = np.concatenate([0.001 * rng.standard_normal((2, half)), 0.3 * rng.standard_normal((2, n - half))], axis=1)
        E = W.random_field(rng, 2, o.n_vertices, 0.02)
        rhos = []
        for dep in (1, 0):
            pic.tune("emit_deposit", dep)
            t = _tree(spec)
            st = pic.Stepper(t, scheme, x, v, ids=np.arange(n, dtype=np.int64), device=dev)
            st.initial_sort()
            xs, vs, _, start, ids = oracle.initial_sort(o, x, v, None, scheme)
            for it in range(2):
                st.step_fused(torch.tensor(E, device=dev), -0.5, 0.5, q_uniform=-1.0 / n)
                r = oracle.step(o, xs, vs, E, -0.5, 0.5, start, scheme, None, -1.0 / n)
                torch.cuda.synchronize()
                ids = ids[r["perm"]]
                assert np.array_equal(st.start.cpu().numpy(), r["bin_start"])
                assert np.array_equal(st.ids.cpu().numpy(), ids)
                assert np.array_equal(st.x.cpu().numpy(), r["x"]) and np.array_equal(st.v.cpu().numpy(), r["v"])
                _check_rho(st.rho.cpu().numpy(), r["rho"])
                xs, vs, start = r["x"], r["v"], r["bin_start"]
            rhos.append(st.rho.cpu().numpy())
            assert t.status_sync() == 0
        assert np.allclose(rhos[0], rhos[1], rtol=1e-13, atol=0.0)
    finally:
        for k, val in saved.items():
            pic.tune(k, val)


@pytest.mark.parametrize("clusters,spread,most", [(4, 0.0005, 16), (1, 0.0001, 64)])
@pytest.mark.parametrize("scheme", [0, 1])
def test_fused_step_with_short_direct_run_lists(scheme, clusters, spread, most):
    """A sparse set on a large tree (200k particles, 59,049 leaves) gets
    direct run lists of 16 per key; the particles sit in a few cells, so
    their keys collect runs from many tiles and spill into the linked
    overflow (from 17 runs on; past 64 with one cluster).  The step still
    matches the oracle."""
    dev = _dev()
    rng = np.random.default_rng(71 + scheme)
    spec = W.regular_tree(2, 5)
    n = 200_000
    centres = rng.random((2, clusters))
    x = (centres[:, rng.integers(0, clusters, n)] + spread * rng.standard_normal((2, n))) % 1.0
    x[x >= 1.0] = 0.0
    v = 0.002 * rng.standard_normal((2, n))
    o = oracle.OracleTree(spec)
    t = _tree(spec)
    E = W.random_field(rng, 2, o.n_vertices, 0.01)
    st = pic.Stepper(t, scheme, x, v, ids=np.arange(n, dtype=np.int64), device=dev)
    st.initial_sort()
    xs, vs, _, start, ids = oracle.initial_sort(o, x, v, None, scheme)
    # the case is the one meant: in the first step some key (a stayer key of
    # the sorted input) has more runs than the direct list holds
    tile = pic.tuning()["step_tile"] or 2048   # 0: by dimension, 2048 for 2D trees
    old_bin = np.repeat(np.arange(len(start) - 1), np.diff(start))
    runs = {}
    for a in range(0, n, tile):
        for k in np.unique(old_bin[a:a + tile]):
            runs[k] = runs.get(k, 0) + 1
    assert max(runs.values()) > most
    for _ in range(2):
        st.step_fused(torch.tensor(E, device=dev), -0.5, 0.5, q_uniform=-1.0 / n)
        r = oracle.step(o, xs, vs, E, -0.5, 0.5, start, scheme, None, -1.0 / n)
        torch.cuda.synchronize()
        ids = ids[r["perm"]]
        assert np.array_equal(st.start.cpu().numpy(), r["bin_start"])
        assert np.array_equal(st.ids.cpu().numpy(), ids)
        assert np.array_equal(st.x.cpu().numpy(), r["x"]) and np.array_equal(st.v.cpu().numpy(), r["v"])
        _check_rho(st.rho.cpu().numpy(), r["rho"])
        xs, vs, start = r["x"], r["v"], r["bin_start"]
    assert t.status_sync() == 0
