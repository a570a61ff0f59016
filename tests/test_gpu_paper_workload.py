"""The particle-handling benchmark of the paper's results section on the
GPU against the oracle: free streaming (periodic and reflecting walls,
artificial flops), particles per leaf, and whole runs with the ppc-driven
adaptation of the tree (paper Sec. 6 setup, Sec. 6.1 lift counts).  Bins,
order and state are compared bit for bit, the statistics and the refine
masks exactly."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1508_02435_amd as pic

pytestmark = pytest.mark.gpu

TREES = {"reg2d": lambda: W.regular_tree(2, 3), "disc2d": lambda: W.disc_tree(2, 2, 4),
         "reg3d": lambda: W.regular_tree(3, 2), "disc3d": lambda: W.disc_tree(3, 1, 3)}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda")


def _paper_particles(rng, dim, n, box=1.0):
    """Uniform positions in (0, box)^d; velocity of uniform length in [0, 1]
    and uniform direction."""
    x = rng.random((dim, n)) * box
    d = rng.standard_normal((dim, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return x, d * rng.random(n)


@pytest.mark.parametrize("flops", [0, 250])
@pytest.mark.parametrize("boundary", [pic._capi.PERIODIC, pic._capi.REFLECTING])
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("name", sorted(TREES))
def test_free_stream_matches_oracle(name, scheme, boundary, flops):
    dev = _dev()
    spec = TREES[name]()
    o = oracle.OracleTree(spec)
    t = pic.Tree(spec).upload()
    rng = np.random.default_rng(len(name) * 10 + scheme + 2 * boundary)
    n = 5 * 256 + 77
    x, v = _paper_particles(rng, spec.dim, n)
    # walls at every distance: some particles land exactly on 1 or 0
    x[0, :8] = [0.75, 0.25, 0.5, 0.875, 0.125, np.nextafter(1.0, 0.0), 0.0, 0.5]
    v[0, :8] = [1.0, -1.0, 2.0, 1.0, -1.0, 1e-300, -1e-300, -2.0]
    xd, vd = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
    b = torch.empty(n, dtype=torch.int32, device=dev)
    for dt in (0.25, 0.01, 0.3):
        pic.free_stream(t, scheme, xd, vd, dt, boundary, flops, b)
        x, v, nb = o.free_stream(x, v, dt, boundary, flops, scheme)
        torch.cuda.synchronize()
        assert np.array_equal(xd.cpu().numpy(), x) and np.array_equal(vd.cpu().numpy(), v)
        assert np.array_equal(b.cpu().numpy(), nb)
    assert t.status_sync() == 0


def test_free_stream_flags_a_move_longer_than_the_box():
    dev = _dev()
    t = pic.Tree(W.regular_tree(2, 2)).upload()
    x = torch.tensor([[0.5, 0.5], [0.5, 0.5]], dtype=torch.float64, device=dev)
    v = torch.tensor([[-9.0, 0.1], [0.0, 0.0]], dtype=torch.float64, device=dev)
    b = torch.empty(2, dtype=torch.int32, device=dev)
    pic.free_stream(t, 0, x, v, 0.25, pic._capi.REFLECTING, 0, b)
    assert t.status_sync() == pic._capi.PIC_E_RANGE
    xs = x.cpu().numpy()
    assert np.all((xs >= 0.0) & (xs < 1.0))
    assert 0 <= int(b.max()) < t.n_leaves


@pytest.mark.parametrize("name", sorted(TREES))
def test_leaf_counts_match_oracle(name):
    dev = _dev()
    spec = TREES[name]()
    o = oracle.OracleTree(spec)
    t = pic.Tree(spec).upload()
    rng = np.random.default_rng(9)
    for n in (0, 1, 1000, 20011):
        x = rng.random((spec.dim, n))
        c = torch.full((t.n_leaves,), 7, dtype=torch.int64, device=dev)
        pic.leaf_counts(t, torch.tensor(x, device=dev), c)
        want = np.bincount(o.bin_of(x, oracle.PIT), minlength=o.n_leaves) if n else np.zeros(o.n_leaves)
        assert np.array_equal(c.cpu().numpy(), want)


def _oracle_run(spec, scheme, x, v, steps, dt, boundary, ppc, cap, flops):
    """The same run on the oracle: per step free streaming, stable re-bin,
    statistics, then one adaptation and a re-sort into a changed tree."""
    o = oracle.OracleTree(spec)
    ids = np.arange(x.shape[1])
    nb = o.bin_of(x, scheme)
    perm, start = oracle.rebin(nb, o.n_bins(scheme), None)
    x, v, ids = x[:, perm], v[:, perm], ids[perm]
    rec = []
    for _ in range(steps):
        x, v, nb = o.free_stream(x, v, dt, boundary, flops, scheme)
        st = o.rebin_stats(start, nb, scheme)
        perm, start = oracle.rebin(nb, o.n_bins(scheme), start)
        x, v, ids = x[:, perm], v[:, perm], ids[perm]
        new = oracle.adapt(spec, x, ppc, cap)
        changed = not (new.max_level == spec.max_level and np.array_equal(new.masks_concat(), spec.masks_concat()))
        if changed:
            spec, o = new, oracle.OracleTree(new)
            nb = o.bin_of(x, scheme)
            perm, start = oracle.rebin(nb, o.n_bins(scheme), None)
            x, v, ids = x[:, perm], v[:, perm], ids[perm]
        rec.append(dict(x=x, v=v, ids=ids, start=start, stats=st, masks=spec.masks_concat(), L=spec.max_level))
    return rec


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("dim,box,scheme", [(2, 0.1, 0), (2, 0.1, 1), (2, 1.0, 0), (3, 0.1, 0), (3, 0.1, 1)])
def test_adaptive_runs_match_oracle(dim, box, scheme, fused):
    """Sub-box or homogeneous start, reflecting walls, ppc-driven tree: every
    step's state, order, offsets, lift statistics and tree equal the
    oracle's."""
    dev = _dev()
    rng = np.random.default_rng(dim * 100 + scheme + int(box * 10))
    n, ppc, cap, steps, dt = (6000, 60, 5, 8, 0.02) if dim == 2 else (3000, 40, 3, 6, 0.03)
    x, v = _paper_particles(rng, dim, n, box)
    spec = W.regular_tree(dim, 1)
    for _ in range(10):          # the initial ppc-driven grid: adapt to a fixed point
        new = oracle.adapt(spec, x, ppc, cap)
        if new.max_level == spec.max_level and np.array_equal(new.masks_concat(), spec.masks_concat()):
            break
        spec = new
    run = pic.FreeStreamRun(pic.Tree(spec).upload(), scheme, x, v, ids=np.arange(n, dtype=np.int64), device=dev)
    run.initial_sort()
    want = _oracle_run(spec, scheme, x, v, steps, dt, pic._capi.REFLECTING, ppc, cap, 128)
    changes = 0
    for k in range(steps):
        s = pic.new_stats(dev)
        (run.step_free_fused if fused else run.step_free)(dt, pic._capi.REFLECTING, 128, stats=s)
        got_stats = pic.read_stats(s)
        changes += run.adapt(ppc, cap)
        w = want[k]
        assert got_stats == w["stats"], k
        assert run.tree.specs[0].max_level == w["L"] and np.array_equal(run.tree.specs[0].masks_concat(), w["masks"])
        assert np.array_equal(run.start.cpu().numpy(), w["start"]), k
        assert np.array_equal(run.ids.cpu().numpy(), w["ids"]), k
        assert np.array_equal(run.x.cpu().numpy(), w["x"]) and np.array_equal(run.v.cpu().numpy(), w["v"]), k
        assert run.tree.status_sync() == 0
    if box < 1.0:
        assert changes > 0           # the particles leave the sub-box: the tree follows


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("name", sorted(TREES))
def test_vmax_matches_oracle(name, scheme):
    """raPIDT's v_max per cell and its predicate (Sec. 5.4, Eq. (vmax)):
    bit for bit against the oracle's definition, for several time steps."""
    dev = _dev()
    spec = TREES[name]()
    rng = np.random.default_rng(17 + scheme)
    n = 4000 + 33
    x, v = _paper_particles(rng, spec.dim, n)
    v[:, :5] *= 3.0                          # a few fast particles
    run = pic.FreeStreamRun(pic.Tree(spec).upload(), scheme, x, v, device=dev)
    run.initial_sort()
    xs, vs = run.x.cpu().numpy(), run.v.cpu().numpy()
    for dt in (1e-3, 0.05, 0.3):
        got, quiet = run.vmax(dt)
        want, wq = oracle.vmax_cells(spec, xs, vs, scheme, dt=dt)
        assert np.array_equal(got.cpu().numpy(), np.concatenate(want))
        assert np.array_equal(quiet.cpu().numpy(), np.concatenate(wq))
    assert run.tree.status_sync() == 0


@pytest.mark.parametrize("tile", [2048, 1024, 4096])
@pytest.mark.parametrize("flops", [0, 46])
@pytest.mark.parametrize("boundary", [pic._capi.PERIODIC, pic._capi.REFLECTING])
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("name", sorted(TREES))
def test_stream_step_matches_oracle(name, scheme, boundary, flops, tile):
    """pic_stream_step (free streaming in the passes of the fused step) against
    the oracle's free streaming and stable re-bin: state, order, offsets and
    statistics bit for bit, over three steps of uneven length (ragged last
    tiles, particles several cells away)."""
    dev = _dev()
    spec = TREES[name]()
    o = oracle.OracleTree(spec)
    t = pic.Tree(spec).upload()
    pic.tune("step_tile", tile, t)
    rng = np.random.default_rng(len(name) + 10 * scheme + 3 * boundary)
    n = 3 * 2048 + 517
    x, v = _paper_particles(rng, spec.dim, n)
    run = pic.FreeStreamRun(t, scheme, x, v, ids=np.arange(n, dtype=np.int64), device=dev)
    run.initial_sort()
    xs, vs, _, start, ids = oracle.initial_sort(o, x, v, None, scheme)
    for dt in (0.01, 0.2, 0.05):
        st = pic.new_stats(dev)
        run.step_free_fused(dt, boundary, flops, stats=st)
        x1, v1, nb = o.free_stream(xs, vs, dt, boundary, flops, scheme)
        want = o.rebin_stats(start, nb, scheme)
        perm, start = oracle.rebin(nb, o.n_bins(scheme), start)
        xs, vs, ids = x1[:, perm], v1[:, perm], ids[perm]
        torch.cuda.synchronize()
        assert np.array_equal(run.start.cpu().numpy(), start)
        assert np.array_equal(run.ids.cpu().numpy(), ids)
        assert np.array_equal(run.x.cpu().numpy(), xs) and np.array_equal(run.v.cpu().numpy(), vs)
        assert pic.read_stats(st) == want
    assert t.status_sync() == 0
