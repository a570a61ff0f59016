"""GPU checks of the FP32 offset form against the FP64 oracle.

The FP32 form cannot match FP64 bit for bit; its error is stated and bounded
per quantity, for one teacher-forced step from the oracle's sorted FP64 state
(converted to offsets o = fl32(x 3^L - I), u = fl32(v dt 3^L)):
  position   max |x32 - x64| * 3^L <= 1e-5 cells;
  velocity   max |v32 - v64| / max |v64| <= 1e-6;
  bins       every particle whose FP32 bin differs from the FP64 one lies
             within the position bound of a cell face (PIT) or of a dual-cell
             face (PIDT); all others keep the FP64 order inside their bin;
  charge     per vertex: |rho32 - rho64| / |rho64| <= 1e-6 on every populated
             vertex (charge >= 1% of the largest; in these uniform plasmas
             that is every vertex), and on every vertex an error <= 1e-6 times
             the total |charge| of the particles whose leaf has it as a corner
             (a vertex reached only by the tip of a weight holds a tiny charge
             whose relative error says nothing); the norm-wise figure
             max_v |rho32 - rho64| / max_v |rho64| stays below 1e-6 too.
The FP32 fused call and the three FP32 calls must agree bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from f32_bounds import check_rho_f32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1508_02435_amd as pic  # noqa: E402

POS_TOL = 1e-5      # cells
VEL_TOL = 1e-6      # relative to max |v|
RHO_TOL = 1e-6      # relative to max |rho|
CASES = [("config1", 0), ("config1", 1), ("small_3d", 0), ("small_3d", 1)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda")


def _face_distance(y, scheme):
    """Distance (in cells) of scaled positions y to the nearest face of the
    scheme's cells: integer lattice (PIT) or half-integer lattice (PIDT)."""
    frac = y - np.floor(y) if scheme == 0 else (y + 0.5) - np.floor(y + 0.5)
    return np.minimum(frac, 1.0 - frac).min(axis=0)


def _setup(name, scheme, dev, rng):
    wl = W.by_name(name)
    o = oracle.OracleTree(wl.tree)
    t = pic.Tree(wl.tree).upload()
    xs, vs, qs, start, perm = oracle.initial_sort(o, wl.x, wl.v, wl.q, scheme)
    scale = 3.0 * wl.h / (wl.dt * wl.dt)
    E = W.random_field(rng, wl.dim, o.n_vertices, scale)
    return wl, o, t, xs, vs, qs, start, E


@pytest.mark.parametrize("name,scheme", CASES)
def test_f32_step_error_against_oracle(name, scheme):
    dev = _dev()
    rng = np.random.default_rng(11)
    wl, o, t, xs, vs, qs, start, E = _setup(name, scheme, dev, rng)
    S = float(3 ** wl.tree.max_level)
    st = pic.Stepper32(t, scheme, xs, vs, dt=wl.dt, q=qs, ids=np.arange(wl.n), device=dev)
    # the conversion to offsets can round a particle on a face into the next
    # cell; such particles start in another bin than in FP64
    b64_0 = np.repeat(np.arange(len(start) - 1), np.diff(start))
    b32_0 = np.repeat(np.arange(len(st.start) - 1), np.diff(st.start.cpu().numpy()))
    ids0 = st.ids.cpu().numpy()
    moved0 = ids0[b32_0 != b64_0[ids0]]
    st.step(torch.tensor(E, device=dev), wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
    r = oracle.step(o, xs, vs, E, wl.qm * wl.dt, wl.dt, start, scheme, qs, wl.q_uniform)
    torch.cuda.synchronize()
    assert t.status_sync() == 0
    x32, v32 = (a.cpu().numpy() for a in st.to_f64())
    ids = st.ids.cpu().numpy()
    # oracle results indexed by the original particle index
    x64 = np.empty_like(r["x"]); v64 = np.empty_like(r["v"])
    x64[:, r["perm"]] = r["x"]; v64[:, r["perm"]] = r["v"]
    dx = np.abs(x32 - x64[:, ids])
    dx = np.minimum(dx, 1.0 - dx) * S                       # periodic distance in cells
    assert dx.max() <= POS_TOL, dx.max()
    assert np.abs(v32 - v64[:, ids]).max() <= VEL_TOL * np.abs(v64).max()
    # bins: where they differ the particle sits on a face to within the bound
    b32 = np.repeat(np.arange(len(st.start) - 1), np.diff(st.start.cpu().numpy()))
    b64 = np.empty(wl.n, dtype=np.int64)
    b64[r["perm"]] = np.repeat(np.arange(len(r["bin_start"]) - 1), np.diff(r["bin_start"]))
    diff = b32 != b64[ids]
    if diff.any():
        d = _face_distance(x64[:, ids[diff]] * S, scheme)
        assert d.max() <= POS_TOL, (int(diff.sum()), d.max())
    assert diff.mean() < 1e-3
    # order: the particles whose old and new bins agree with FP64 have the same
    # keys (bin, stayed) in both forms, so they keep the FP64 relative order
    diff |= np.isin(ids, moved0)
    rank64 = np.empty(wl.n, dtype=np.int64)
    rank64[r["perm"]] = np.arange(wl.n)
    keep = ~diff
    rk = rank64[ids[keep]]
    same_bin = b32[keep][1:] == b32[keep][:-1]
    assert (np.diff(rk)[same_bin] > 0).all()
    rho32, rho64 = st.rho.cpu().numpy(), r["rho"]
    assert np.abs(rho32 - rho64).max() <= RHO_TOL * np.abs(rho64).max()
    check_rho_f32(o, r["x"], r["q"], wl.q_uniform, rho32, rho64, name)


@pytest.mark.parametrize("key_stores,step_tile", [(0, 0), (1, 0), (0, 2048), (1, 2048), (0, 4096), (1, 4096)])
@pytest.mark.parametrize("name,scheme", CASES)
def test_f32_fused_equals_three_calls(name, scheme, key_stores, step_tile):
    """The single call (pushing twice, or storing the pushed state in the key
    pass; tiles of 2048 or 4096 particles) gives the three calls' state,
    order and charge bit for bit."""
    dev = _dev()
    rng = np.random.default_rng(12)
    wl, o, t, xs, vs, qs, start, E = _setup(name, scheme, dev, rng)
    pic.tune("key_stores", key_stores, t)
    pic.tune("step_tile", step_tile, t)
    Ed = torch.tensor(E, device=dev)
    outs = []
    for fused in (False, True):
        st = pic.Stepper32(t, scheme, xs, vs, dt=wl.dt, q=qs, ids=np.arange(wl.n), device=dev)
        for _ in range(3):
            (st.step_fused if fused else st.step)(Ed, wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
        torch.cuda.synchronize()
        outs.append([a.cpu().numpy().copy() for a in (st.off, st.u, st.ids, st.start, st.rho)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("scheme", [0, 1])
def test_f32_conversion_round_trip(scheme):
    dev = _dev()
    wl = W.config1()
    o = oracle.OracleTree(wl.tree)
    t = pic.Tree(wl.tree).upload()
    xs, vs, _, start, _ = oracle.initial_sort(o, wl.x, wl.v, None, scheme)
    st = pic.Stepper32(t, scheme, xs, vs, dt=wl.dt, ids=np.arange(wl.n), device=dev)
    x32, v32 = (a.cpu().numpy() for a in st.to_f64())
    ids = st.ids.cpu().numpy()
    S = float(3 ** wl.tree.max_level)
    dx = np.abs(x32 - xs[:, ids])
    assert (np.minimum(dx, 1 - dx) * S).max() <= 2.0 ** -23
    assert np.abs(v32 - vs[:, ids]).max() <= 2.0 ** -23 * np.abs(vs).max()
    assert t.status_sync() == 0


def test_f32_forest_matches_single_trees():
    """A forest of regular instances steps each instance as its own tree."""
    dev = _dev()
    insts = W.config5(n_inst=4, n_min=2e3, n_max=2e4)
    t = pic.Tree([w.tree for w in insts]).upload()
    counts = [w.n for w in insts]
    inst_start = torch.tensor(np.concatenate([[0], np.cumsum(counts)]), dtype=torch.int64, device=dev)
    rng = np.random.default_rng(3)
    Es = [W.random_field(rng, 2, oracle.OracleTree(w.tree).n_vertices, 2.0 * w.h / w.dt ** 2) for w in insts]
    qd = torch.tensor([w.qm * w.dt for w in insts], dtype=torch.float64, device=dev)
    dd = torch.tensor([w.dt for w in insts], dtype=torch.float64, device=dev)
    for scheme in (0, 1):
        x = np.concatenate([w.x for w in insts], axis=1)
        v = np.concatenate([w.v for w in insts], axis=1)
        st = pic.Stepper32(t, scheme, x, v, ids=np.arange(x.shape[1]), inst_start=inst_start, dt_dev=dd,
                           device=dev)
        st.step_fused(torch.tensor(np.concatenate(Es, axis=1), device=dev), 0.0, 0.0, q_uniform=-1.0,
                      qmdt_dev=qd, dt_dev=dd)
        torch.cuda.synchronize()
        assert t.status_sync() == 0
        off, u, ids, starts = (a.cpu().numpy() for a in (st.off, st.u, st.ids, st.start))
        rho = st.rho.cpu().numpy()
        p0 = 0
        for i, w in enumerate(insts):
            ti = pic.Tree(w.tree).upload()
            si = pic.Stepper32(ti, scheme, w.x, w.v, dt=w.dt, ids=np.arange(w.n) + p0, device=dev)
            si.step_fused(torch.tensor(Es[i], device=dev), w.qm * w.dt, w.dt, q_uniform=-1.0)
            torch.cuda.synchronize()
            ii = t.instance(i)
            b0 = ii.leaf_offset if scheme == 0 else ii.pidt_offset
            nb = ii.n_leaves if scheme == 0 else ii.n_pidt
            s_i = si.start.cpu().numpy()
            assert np.array_equal(starts[b0:b0 + nb + 1] - starts[b0], s_i)
            sl = slice(int(starts[b0]), int(starts[b0 + nb]))
            assert np.array_equal(ids[sl], si.ids.cpu().numpy())
            assert np.array_equal(off[:, sl], si.off.cpu().numpy())
            assert np.array_equal(u[:, sl], si.u.cpu().numpy())
            rv = rho[ii.vertex_offset:ii.vertex_offset + ii.n_vertices]
            assert np.array_equal(rv, si.rho.cpu().numpy())
            p0 += w.n


def test_f32_charge_is_conserved_over_steps():
    dev = _dev()
    wl = W.config1()
    o = oracle.OracleTree(wl.tree)
    t = pic.Tree(wl.tree).upload()
    st = pic.Stepper32(t, 0, wl.x, wl.v, dt=wl.dt, device=dev)
    E = torch.tensor(wl.field(o.vertex_positions_unit()), device=dev)
    for _ in range(10):
        st.step_fused(E, wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
        torch.cuda.synchronize()
        total = st.rho.sum().item()
        assert abs(total - wl.q_uniform * wl.n) <= 1e-6 * abs(wl.q_uniform * wl.n)
    assert int(st.start[-1].item()) == wl.n
    assert t.status_sync() == 0


@pytest.mark.parametrize("name,scheme", CASES)
def test_f32_rebin_stats(name, scheme):
    """The FP32 fused call and the three FP32 calls count the same movers and
    lifts; against the FP64 oracle they differ only by particles whose FP32
    bin differs (particles within the position bound of a face)."""
    dev = _dev()
    rng = np.random.default_rng(13)
    wl, o, t, xs, vs, qs, start, E = _setup(name, scheme, dev, rng)
    Ed = torch.tensor(E, device=dev)
    got = []
    for fused in (False, True):
        st = pic.Stepper32(t, scheme, xs, vs, dt=wl.dt, q=qs, device=dev)
        stats = pic.new_stats(dev)
        (st.step_fused if fused else st.step)(Ed, wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform, stats=stats)
        torch.cuda.synchronize()
        got.append(pic.read_stats(stats))
    assert got[0] == got[1]
    r = oracle.step(o, xs, vs, E, wl.qm * wl.dt, wl.dt, start, scheme, qs, wl.q_uniform)
    want = o.rebin_stats(start, r["new_bin"], scheme)
    assert got[0]["particles"] == want["particles"]
    assert abs(got[0]["movers"] - want["movers"]) <= 1e-3 * wl.n
    assert abs(got[0]["lifts"] - want["lifts"]) <= 1e-3 * wl.n * wl.tree.max_level
    assert t.status_sync() == 0
