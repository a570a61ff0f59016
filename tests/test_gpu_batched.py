"""GPU checks of the batched form: a forest of independent instances stepped
by one launch sequence, captured in a HIP graph and autotuned.

A replayed graph must give exactly the eager result after every replay (with
eager work and synchronisations between replays), and the autotuner's
launch shape must not change any result.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1508_02435_amd as pic  # noqa: E402
from paper_1508_02435_amd import autotune  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda")


def _forest(dev, n_inst=6, n_min=2e3, n_max=4e4):
    insts = W.config5(n_inst=n_inst, n_min=n_min, n_max=n_max)
    t = pic.Tree([w.tree for w in insts]).upload()
    counts = [w.n for w in insts]
    inst_start = torch.tensor(np.concatenate([[0], np.cumsum(counts)]), dtype=torch.int64, device=dev)
    x = np.concatenate([w.x for w in insts], axis=1)
    v = np.concatenate([w.v for w in insts], axis=1)
    Es = [w.field(oracle.OracleTree(w.tree).vertex_positions_unit()) for w in insts]
    E = torch.tensor(np.concatenate(Es, axis=1), device=dev)
    qd = torch.tensor([w.qm * w.dt for w in insts], dtype=torch.float64, device=dev)
    dd = torch.tensor([w.dt for w in insts], dtype=torch.float64, device=dev)
    return insts, t, inst_start, x, v, E, qd, dd


def _state(st):
    names = ("off", "u", "ids", "start", "rho") if isinstance(st, pic.Stepper32) else ("x", "v", "ids", "start", "rho")
    return [getattr(st, k).cpu().numpy().copy() for k in names]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("scheme", [0, 1])
def test_graph_replays_match_eager_steps(precision, scheme):
    dev = _dev()
    insts, t, inst_start, x, v, E, qd, dd = _forest(dev)
    ids = np.arange(x.shape[1])

    def make():
        if precision == "f32":
            return pic.Stepper32(t, scheme, x, v, ids=ids, inst_start=inst_start, dt_dev=dd, device=dev)
        st = pic.Stepper(t, scheme, x, v, ids=ids, inst_start=inst_start, device=dev)
        st.initial_sort()
        return st

    eager, cap = make(), make()
    kw = dict(q_uniform=-1.0, qmdt_dev=qd, dt_dev=dd)
    g = pic.StepGraph(cap, E, 0.0, 0.0, **kw)            # capture advances `cap` by two eager steps
    for _ in range(2):
        eager.step_fused(E, 0.0, 0.0, **kw)
    torch.cuda.synchronize()
    for a, b in zip(_state(eager), _state(cap)):
        assert np.array_equal(a, b)
    for rep in range(4):
        g.replay()
        for _ in range(2):
            eager.step_fused(E, 0.0, 0.0, **kw)
        junk = torch.ones(1000, device=dev).sum()         # eager work between replays
        torch.cuda.synchronize()
        assert junk.item() == 1000.0
        for a, b in zip(_state(eager), _state(cap)):
            assert np.array_equal(a, b), f"replay {rep}"
    assert t.status_sync() == 0


@pytest.mark.parametrize("fused", [True, False])
def test_autotune_changes_speed_not_results(fused, tmp_path):
    dev = _dev()
    insts, t, inst_start, x, v, E, qd, dd = _forest(dev, n_inst=4)
    before = pic.tuning()
    kw = dict(q_uniform=-1.0, qmdt_dev=qd, dt_dev=dd)
    try:
        ref = pic.Stepper(t, 0, x, v, ids=np.arange(x.shape[1]), inst_start=inst_start, device=dev)
        ref.initial_sort()
        (ref.step_fused if fused else ref.step)(E, 0.0, 0.0, **kw)
        torch.cuda.synchronize()
        want = _state(ref)
        st = pic.Stepper(t, 0, x, v, ids=np.arange(x.shape[1]), inst_start=inst_start, device=dev)
        st.initial_sort()
        cache = str(tmp_path / "tune.json")
        best = autotune.autotune(st, E, 0.0, 0.0, fused=fused, steps=1, cache=cache, **kw)
        assert set(best) == set(autotune.SPACES["fused_f64" if fused else "calls_f64"])
        assert all(pic.tuning(t)[k] == v for k, v in best.items())
        # the tuner restored the state it timed on; one step now equals the reference
        (st.step_fused if fused else st.step)(E, 0.0, 0.0, **kw)
        torch.cuda.synchronize()
        for a, b in zip(want, _state(st)):
            assert np.array_equal(a, b)
        # a cached signature applies without timing
        for k, val in before.items():
            if k not in pic.PROCESS_ONLY:
                pic.tune(k, val, t)
        assert autotune.autotune(st, E, 0.0, 0.0, fused=fused, cache=cache, **kw) == best
        assert all(pic.tuning(t)[k] == v for k, v in best.items())
    finally:
        for k, val in before.items():
            pic.tune(k, val)
