#!/usr/bin/env python3
"""Benchmark of the spacetree PIC hot path on one MI355X.

One step = gather + push + rebin + deposit over the whole particle set, inputs
resident in HBM.  By default the step is the fused entry point pic_step; with
--path calls it is pic_gather_push + pic_rebin + pic_deposit.

Workloads (--config):
  2  2D periodic regular depth-5 spacetree (243 x 243 leaves), 15,116,544
     electrons (256 per cell, Maxwellian v_th = 1 cell/step plus 1% beam
     particles at 8-20 cells/step, 1% density perturbation on modes 1..4).
  3  2D adaptive spacetree, depth 4 refined to 6 inside a disc of radius 0.2
     (74,609 leaves), 9,549,952 electrons (128 per leaf) with per-particle
     charges, v_th = 1 coarse cell/step.
  4  3D periodic regular depth-4 spacetree (81^3 leaves), 34,012,224 electrons
     (64 per cell, v_th = 1 cell/step plus 5% isotropic tunnelers at 1-10
     cells/step).

Configs 2 and 4 are Langmuir plasmas: before the timed region the run is
stepped self-consistently (deposit, FP64 periodic Poisson solve, field on
the vertices, then the hot path), and the field of every step is kept in HBM.
The timed region replays the hot-path steps from the state at its start with
those fields; the hot path is deterministic, so the replay is the same
trajectory with the Poisson solve (which is not part of the hot path) left
out of the timing.  Config 3 uses its prescribed field.

Prints one JSON line (the benchmark contract) with the whole-step throughput,
a roofline entry for the dominant kernel (algorithmic bytes over its average
HIP-event duration in the timed region) and the serial FP64 oracle timed on
the host as a CPU baseline.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle updates/s (gather+push+rebin+deposit), HBM GB/s vs peak; FP32/batched vs FP64"
HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes_f32(dim: int, per_particle_q: bool, stored: bool = False):
    """Bytes each kernel must move per particle (FP32 offset form); `stored`:
    the key pass writes the pushed state back (knob key_stores)."""
    s_push = 2 * 4 * dim                   # off, u
    q = 8 if per_particle_q else 0
    s_rec = s_push + q
    s_dep = 4 * dim + q
    key = s_push + 4 + (s_push if stored else 0)   # off, u read, key (and the pushed state) written
    return {
        "gather_push_f32": 2 * s_push + 4,
        "rebin_tiles": 4,
        "rebin_scatter": 2 * s_rec,
        "deposit_bins_f32": s_dep,
        "step_key_f32": key,
        "step_group": 4 + 4,
        "step_emit_f32": s_push + 4 + s_rec + q,
        "fused": key + 8 + (s_push + 4 + s_rec + q) + s_dep,
        "calls": 2 * s_push + 2 * s_rec + s_dep + 8,
    }


def algorithmic_bytes(dim: int, per_particle_q: bool, stored: bool = False, emit_deposit: bool = False,
                      fused_rank: bool = False):
    """Bytes each kernel must move per particle (FP64 form).  "calls" is the
    three-call path (gather_push, rebin, deposit); "fused" is pic_step (key,
    group and emit passes, then the deposit); `stored`: the key pass writes
    the pushed state back (knob key_stores); `emit_deposit`: the writing pass
    deposits while the positions are in LDS, so the deposit reads no
    positions (its per-run partials, a few per tile, are not counted);
    `fused_rank`: the key pass and the ranking are one kernel (knob
    step_fuse), which writes no keys."""
    s_push = 2 * 8 * dim                   # x, v
    q = 8 if per_particle_q else 0
    s_rec = s_push + q                     # a full record moved by a rebin
    s_dep = 8 * dim + q                    # positions (and charges) read by the deposit
    ab = {
        "gather_push": 2 * s_push + 4,     # x, v read and written, new bin written
        "rebin_tiles": 4,                  # new bins read
        "rebin_scatter": 2 * s_rec,        # every record read and written once
        "deposit_bins": s_dep,
        "step_key": s_push + 4 + (s_push if stored else 0),   # x, v read, key (and the pushed state) written
        "step_group": 4 + 4,               # key read, run index | rank written
        "step_emit": s_push + 4 + s_rec + q,   # x, v, run index | rank (and q) read, the record written
        "calls": 2 * s_push + 2 * s_rec + s_dep + 8,
    }
    ab["step_keyrank"] = s_push + 4                 # x, v read, run index | rank written
    first = ab["step_keyrank"] if fused_rank else ab["step_key"] + ab["step_group"]
    ab["fused"] = first + ab["step_emit"] + (0 if emit_deposit else s_dep)
    return ab


def kernel_times(lib):
    arr = (pic_capi.KernelTime * 64)()
    n = min(lib.pic_profile_read(arr, 64), 64)
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n)}


def cpu_baseline(wl, scheme, sample, E_np, min_seconds=10.0, max_steps=8):
    """The oracle as it stands, single-threaded: whole steps over the first `sample`
    particles, repeated (each step continues from the previous one) until
    `min_seconds` of oracle time have passed."""
    import numpy as np
    import oracle
    o = oracle.OracleTree(wl.tree)
    x = np.ascontiguousarray(wl.x[:, :sample])
    v = np.ascontiguousarray(wl.v[:, :sample])
    q = None if wl.q is None else np.ascontiguousarray(wl.q[:sample])
    xs, vs, qs, start, _ = oracle.initial_sort(o, x, v, q, scheme)
    steps, spent = 0, 0.0
    while spent < min_seconds and steps < max_steps:
        t0 = time.perf_counter()
        r = oracle.step(o, xs, vs, E_np, wl.qm * wl.dt, wl.dt, start, scheme, qs, wl.q_uniform)
        spent += time.perf_counter() - t0
        xs, vs, qs, start = r["x"], r["v"], r["q"], r["bin_start"]
        steps += 1
    model = platform.processor() or ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": sample * steps / spent, "unit": "particle updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps (gather+push, rebin, deposit) of the first {sample} particles of the same "
                      f"workload on the same tree, serial C oracle, {spent:.1f} s; host {model}, "
                      f"{os.cpu_count()} logical CPUs visible"}


def source_digest() -> str:
    """sha256 over every kernel source and the ABI header, in name order: the
    stored counter figures hold only for the sources they were taken with."""
    import glob
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1508_02435_amd", "csrc", "*"))) + \
        [os.path.join(ROOT, "include", "pic.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if still
    valid (taken with the current kernel sources)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("source_digest") != source_digest():
        return None                       # a kernel changed since the counters were taken
    return ent["bytes_per_launch"]


def poisson_field(rho_charge, dim: int, level: int, background: float = 1.0):
    """Field of a periodic plasma on a regular tree's vertices (support for
    the benchmark, outside the hot path; paper Sec. 3 steps 2-3, App. A):
    -Lap_h V = rho / h^d + background with the (2d+1)-point Laplacian on the
    periodic vertex grid, solved by the DFT (eigenvalues sum_k (2 - 2 cos(2 pi
    m_k / n)) / h^2, mean of V zero), then E = -grad V by central differences.
    rho_charge: vertex charge (what the deposit returns), vertices numbered
    lexicographically with axis 0 fastest.  FP64 throughout."""
    import numpy as np
    n = 3 ** level
    h = 1.0 / n
    dens = np.asarray(rho_charge, np.float64).reshape((n,) * dim) / h ** dim + background
    m = np.arange(n)
    eig = (2.0 - 2.0 * np.cos(2.0 * np.pi * m / n)) / (h * h)
    lam = np.zeros((n,) * dim)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = n
        lam = lam + eig.reshape(shape)
    lam.flat[0] = 1.0
    vh = np.fft.fftn(dens) / lam
    vh.flat[0] = 0.0
    V = np.real(np.fft.ifftn(vh))
    E = np.zeros((dim, n ** dim))
    for k in range(dim):
        ax = dim - 1 - k                      # axis k of the domain is array axis d-1-k
        E[k] = (-(np.roll(V, -1, axis=ax) - np.roll(V, 1, axis=ax)) / (2.0 * h)).ravel()
    return E


def langmuir_sequence(torch, st, wl, steps, dev, first=False):
    """Steps `st` (an FP64 stepper) `steps` times self-consistently and returns
    the field of every step on the device.  With `first`, the leapfrog is
    started: v^(-1/2) = v^0 - (q/m) (dt/2) E(x^0) (a zero-length push)."""
    qmdt, dt = wl.qm * wl.dt, wl.dt
    fields = []
    st.deposit(wl.q_uniform)
    for k in range(steps):
        E = torch.tensor(poisson_field(st.rho.cpu().numpy(), wl.dim, wl.tree.max_level), device=dev)
        if first and k == 0:
            st.gather_push(E, -0.5 * qmdt, 0.0)
        fields.append(E)
        st.step_fused(E, qmdt, dt, q_uniform=wl.q_uniform)
    torch.cuda.synchronize()
    return fields


WORKLOADS = {
    2: ("2D periodic regular depth-5 spacetree (243x243 leaves), {n} electrons (256/cell, v_th 1 cell/step, "
        "1% beam 8-20 cells/step)"),
    3: ("2D periodic adaptive spacetree, depth 4 refined to 6 in a disc of radius 0.2 ({leaves} leaves), {n} "
        "electrons (128/leaf, per-particle charge, v_th 1 coarse cell/step)"),
    4: ("3D periodic regular depth-4 spacetree (81^3 leaves), {n} electrons (64/cell, v_th 1 cell/step, "
        "5% isotropic 1-10 cells/step)"),
}


def fp32_accuracy(pic, torch, tree, scheme, wl, x, v, E, dev):
    """One step of the FP32 form against the FP64 form (which equals the
    serial oracle bit for bit) from the same sorted state, error per quantity;
    the charge per vertex over vertices touched by at least 64 particles, and
    norm-wise."""
    import numpy as np
    assert wl.q is None, "the FP32 form runs on regular trees with uniform charge"
    s64 = pic.Stepper(tree, scheme, x, v, ids=np.arange(wl.n), device=dev)
    s64.initial_sort()
    s32 = pic.Stepper32(tree, scheme, s64.x, s64.v, dt=wl.dt, q=s64.q, ids=s64.ids, device=dev)
    S = float(3 ** wl.tree.max_level)
    s64.step_fused(E, wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
    s32.step_fused(E, wl.qm * wl.dt, wl.dt, q_uniform=wl.q_uniform)
    x32, v32 = s32.to_f64()
    torch.cuda.synchronize()
    inv = torch.empty_like(s64.ids)
    inv[s64.ids] = torch.arange(wl.n, device=dev, dtype=s64.ids.dtype)
    j = inv[s32.ids]
    dx = (x32 - s64.x[:, j]).abs()
    dx = torch.minimum(dx, 1.0 - dx) * S
    b32 = torch.repeat_interleave(torch.arange(len(s32.start) - 1, device=dev), s32.start.diff())
    b64 = torch.repeat_interleave(torch.arange(len(s64.start) - 1, device=dev), s64.start.diff())
    moved = (b32 != b64[j]).sum().item()
    # particles touching each vertex (leaf corners; regular trees: the finest cells)
    cnt = torch.zeros(tree.n_vertices, dtype=torch.float64, device=dev)
    Sn = int(S)
    cell = torch.clamp((s64.x * S).floor().long(), 0, Sn - 1)
    for c in range(1 << wl.dim):
        vid = torch.zeros(wl.n, dtype=torch.long, device=dev)
        stride = 1
        for k in range(wl.dim):
            vid += ((cell[k] + ((c >> k) & 1)) % Sn) * stride
            stride *= Sn
        cnt.index_add_(0, vid, torch.ones(wl.n, dtype=torch.float64, device=dev))
    pop = (cnt >= 64) & (s64.rho != 0)
    rel = ((s32.rho - s64.rho).abs()[pop] / s64.rho.abs()[pop]).max().item() if pop.any() else 0.0
    out = {"position_max_abs_cells": dx.max().item(),
           "velocity_max_rel": ((v32 - s64.v[:, j]).abs().max() / s64.v.abs().max()).item(),
           "rho_max_rel_per_vertex": rel,
           "rho_vertices_compared": int(pop.sum().item()),
           "rho_max_rel_normwise": ((s32.rho - s64.rho).abs().max() / s64.rho.abs().max()).item(),
           "bins_differing_fraction": moved / wl.n,
           "reference": "FP64 form of the same step (bit-exact to the serial oracle in the parity tests)"}
    del s64, s32
    torch.cuda.empty_cache()
    return out


def run_batched(args, scheme):
    """Config 5: 64 independent 2D Langmuir instances (depths 3-5, 0.1M-4M
    particles each) as one forest, one launch sequence per step, autotuned
    and replayed from a HIP graph; FP64 and FP32, against the same 64
    instances stepped one after another as plain single trees (FP64)."""
    import numpy as np
    import torch
    import workloads as W
    import paper_1508_02435_amd as pic
    from paper_1508_02435_amd import autotune

    dev = torch.device("cuda:0")
    _log("[bench] generating config 5")
    insts = W.config5()
    n = sum(w.n for w in insts)
    t = pic.Tree([w.tree for w in insts]).upload(dev)
    inst_start = torch.tensor(np.concatenate([[0], np.cumsum([w.n for w in insts])]), dtype=torch.int64, device=dev)
    Es = [w.field(pic.Tree(w.tree).vertex_table().T.astype(np.float64) / w.tree.finest) for w in insts]
    E = torch.tensor(np.concatenate(Es, axis=1), dtype=torch.float64, device=dev)
    qd = torch.tensor([w.qm * w.dt for w in insts], dtype=torch.float64, device=dev)
    dd = torch.tensor([w.dt for w in insts], dtype=torch.float64, device=dev)
    q_uniform = -1.0 / n
    kw = dict(q_uniform=q_uniform, qmdt_dev=qd, dt_dev=dd)
    steps = max(2, args.steps - args.steps % 2)
    lib = pic.lib()
    results = {}

    def timed_graph(st, label):
        if args.knob:   # the given launch shape instead of the autotuned one
            for kv in args.knob:
                name, value = kv.split("=")
                pic.tune(name, int(value), t)
            knobs = pic.tuning(t)
        else:
            knobs = autotune.autotune(st, E, 0.0, 0.0, fused=True, steps=2, **kw)
        g = pic.StepGraph(st, E, 0.0, 0.0, **kw)
        for _ in range(max(1, args.warmup // 2)):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // 2):
            g.replay()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if t.status_sync() != 0:
            raise RuntimeError(f"device status error in the {label} run")
        results[label] = {"updates_per_s": n * steps / el, "ms_per_step": 1e3 * el / steps, "knobs": knobs}
        _log(f"[bench] {label}: {1e3 * el / steps:.3f} ms/step, {n * steps / el:.4g} updates/s, knobs {knobs}")

    _log(f"[bench] forest: {len(insts)} instances, {n} particles")
    x = np.concatenate([w.x for w in insts], axis=1)
    v = np.concatenate([w.v for w in insts], axis=1)
    st = pic.Stepper(t, scheme, x, v, inst_start=inst_start, device=dev)
    st.initial_sort()
    timed_graph(st, "batched_f64")
    # per-kernel table and roofline of the batched FP64 step (profiled eager steps)
    lib.pic_profile_enable(1)
    kernel_times(lib)
    for _ in range(steps):
        st.step_fused(E, 0.0, 0.0, **kw)
    torch.cuda.synchronize()
    kt = kernel_times(lib)
    lib.pic_profile_enable(0)
    per_kernel = {k: {"launches": a, "avg_ms": tot / a} for k, (a, tot) in kt.items()}
    ab = algorithmic_bytes(2, False)
    dominant = max((k for k in per_kernel if k in ab), key=lambda k: per_kernel[k]["avg_ms"])
    achieved = ab[dominant] * n / (per_kernel[dominant]["avg_ms"] * 1e-3) / 1e9
    del st
    torch.cuda.empty_cache()

    st = pic.Stepper32(t, scheme, x, v, inst_start=inst_start, dt_dev=dd, device=dev)
    timed_graph(st, "batched_f32")
    lib.pic_profile_enable(1)
    kernel_times(lib)
    for _ in range(steps):
        st.step_fused(E, 0.0, 0.0, **kw)
    torch.cuda.synchronize()
    kt32 = kernel_times(lib)
    lib.pic_profile_enable(0)
    results["batched_f32"]["kernels_ms"] = {k: round(tot / a, 4) for k, (a, tot) in
                                            sorted(kt32.items(), key=lambda kv: -kv[1][1])}
    del st
    torch.cuda.empty_cache()

    # the same instances as 64 plain single-tree FP64 runs, one after another
    plain = []
    for w in insts:
        ti = pic.Tree(w.tree).upload(dev)
        si = pic.Stepper(ti, scheme, w.x, w.v, device=dev)
        si.initial_sort()
        Ei = torch.tensor(w.field(ti.vertex_table().T.astype(np.float64) / w.tree.finest), device=dev)
        plain.append((ti, si, Ei, w))
    for _ in range(args.warmup):
        for ti, si, Ei, w in plain:
            si.step_fused(Ei, w.qm * w.dt, w.dt, q_uniform=q_uniform)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for ti, si, Ei, w in plain:
            si.step_fused(Ei, w.qm * w.dt, w.dt, q_uniform=q_uniform)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    results["plain_f64"] = {"updates_per_s": n * steps / el, "ms_per_step": 1e3 * el / steps}
    _log(f"[bench] plain_f64: {1e3 * el / steps:.3f} ms/step")
    del plain
    torch.cuda.empty_cache()

    b = results["batched_f64"]
    out = {
        "metric": METRIC, "value": b["updates_per_s"], "unit": "particle updates/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": b["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"64 independent 2D Langmuir instances (regular depths 3-5, 0.1M-4M electrons "
                               f"each, {n} in total) as one forest, {args.scheme.upper()}, FP64, fused step "
                               f"replayed from a HIP graph, autotuned launch shape",
                   "particles": n, "instances": len(insts), "scheme": args.scheme, "path": "fused"},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "step_algorithmic_GBps": round(ab["fused"] * b["updates_per_s"] / 1e9, 1),
                     "step_frac": round(ab["fused"] * b["updates_per_s"] / 1e9 / HBM_PEAK_GBS, 4)},
        "cpu_baseline": None,
        "kernels_ms": {k: round(vv["avg_ms"], 4) for k, vv in sorted(per_kernel.items(), key=lambda kv: -kv[1]["avg_ms"])},
        "batched": results,
    }
    print(json.dumps(out), flush=True)


def paper_particles(rng, dim, n, box):
    """The paper's start (Sec. 6 setup): positions uniform in (0, box)^d,
    velocity of uniform length in [0, 1] along a uniform direction."""
    import numpy as np
    x = rng.random((dim, n)) * box
    d = rng.standard_normal((dim, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return x, d * rng.random(n)


def run_paper(args, scheme):
    """The paper's particle-handling benchmark: free streaming with reflecting
    walls and re-binning on a tree that follows a ppc threshold (refined and
    coarsened every step), no field; lifts per particle per step."""
    import numpy as np
    import torch
    import paper_1508_02435_amd as pic
    import workloads as W
    lib = pic_capi.lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(args.seed)
    n, dim = args.particles, args.dim
    box = 0.1 if args.start == "subbox" else 1.0
    cap = args.max_level or (8 if dim == 2 else 5)
    _log(f"[bench] paper workload: {dim}D, {n} particles, {args.start}, dt {args.dt}, ppc {args.ppc}")
    x, v = paper_particles(rng, dim, n, box)
    run = pic.FreeStreamRun(pic.Tree(W.regular_tree(dim, 1)).upload(dev), scheme, x, v, device=dev)
    del x, v
    run.initial_sort()
    for _ in range(3 * cap):                 # the initial ppc-driven grid
        if not run.adapt(args.ppc, cap):
            break
    for kv in args.knob:
        name, value = kv.split("=")
        pic.tune(name, int(value), run.tree)
    step = run.step_free_fused if args.path == "fused" else run.step_free
    for _ in range(max(args.warmup, 1)):
        step(args.dt, pic_capi.REFLECTING, args.flops)
        run.adapt(args.ppc, cap)
    torch.cuda.synchronize()
    steps = args.steps
    # the hot path: steps back to back on the stream (no host round trip in
    # between)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step(args.dt, pic_capi.REFLECTING, args.flops)
    b.record()
    b.synchronize()
    hot_ms = [a.elapsed_time(b) / steps]
    # the same number of further steps with the re-bin statistics (their
    # kernel is not part of the timed path)
    stats = pic.new_stats(dev)
    for _ in range(steps):
        step(args.dt, pic_capi.REFLECTING, args.flops, stats=stats)
    acc = pic.read_stats(stats)
    # steps with an adaptation check after each (counts to the host, the
    # rule, a rebuild and re-sort when the tree changes), on the wall clock
    changes = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        step(args.dt, pic_capi.REFLECTING, args.flops)
        changes += run.adapt(args.ppc, cap)
    torch.cuda.synchronize()
    with_adapt_ms = (time.perf_counter() - t0) * 1e3 / steps
    # per-kernel times of the hot path (profiled steps)
    lib.pic_profile_enable(1)
    kernel_times(lib)
    for _ in range(min(steps, 5)):
        step(args.dt, pic_capi.REFLECTING, args.flops)
    torch.cuda.synchronize()
    kt = kernel_times(lib)
    lib.pic_profile_enable(0)
    if run.tree.status_sync() != 0:
        raise RuntimeError("device status error in the paper workload")
    hot = float(np.mean(hot_ms))
    value = n / (hot * 1e-3)
    # the paper's grid-free stream benchmark on the same arrays (Table 1)
    xs = (C.c_void_p * 3)(*[run.x2[k].data_ptr() if k < dim else None for k in range(3)])
    vs = (C.c_void_p * 3)(*[run.v2[k].data_ptr() if k < dim else None for k in range(3)])
    run.x2.copy_(run.x)
    run.v2.copy_(run.v)
    sp = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    lib.pic_stream_push(dim, n, xs, vs, args.dt, sp)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for _ in range(steps):
        lib.pic_stream_push(dim, n, xs, vs, args.dt, sp)
    torch.cuda.synchronize()
    stream_s = (time.perf_counter() - s0) / steps
    # raPIDT's predicate on the final state: cells whose particles cannot
    # move by the cell's width in one step (Sec. 5.4)
    vm, quiet = run.vmax(args.dt)
    quiet = quiet.cpu().numpy().astype(bool)
    spec = run.tree.specs[0]
    refined = np.concatenate([np.asarray(m, np.uint8).ravel() for m in spec.refine] +
                             [np.zeros(3 ** (dim * spec.max_level), np.uint8)]).astype(bool)
    n_leaf = int(run.tree.n_leaves)
    rapidt = {"root_quiet": bool(quiet[0]), "vmax_root": float(vm[0]),
              "quiet_refined_cells": int((quiet & refined).sum()), "refined_cells": int(refined.sum()),
              "quiet_leaves": int((quiet & ~refined).sum()), "leaves": n_leaf}
    tot = acc["particles"]
    out = {
        "metric": "particle updates/s (free streaming + re-bin: the paper's particle-handling benchmark)",
        "value": value, "unit": "particle updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(hot, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"paper Sec. 6 setup: {dim}D, {n} particles, {args.start} start, |v| <= 1 uniform, "
                               f"reflecting walls, dt {args.dt}, ppc {args.ppc} (dynamic refine/coarsen, level cap "
                               f"{cap}), {args.flops} artificial flops per move, {args.scheme.upper()}, "
                               f"{'one call (pic_stream_step)' if args.path == 'fused' else 'pic_free_stream + pic_rebin'}",
                   "particles": n, "leaves": int(run.tree.n_leaves), "max_level": int(run.tree.specs[0].max_level),
                   "scheme": args.scheme, "dt": args.dt, "ppc": args.ppc, "flops": args.flops, "start": args.start,
                   "path": args.path,
                   "knobs": pic.tuning(run.tree)},
        "with_adaptation": {"ms_per_step": round(with_adapt_ms, 4), "tree_changes": changes,
                            "updates_per_s": n / (with_adapt_ms * 1e-3)},
        "rebin_stats": {"mover_fraction": acc["movers"] / tot, "lifts_per_particle_step": acc["lifts"] / tot,
                        "max_tunnel_cells": acc["max_tunnel"], "lift_histogram": acc["lift_hist"][:8],
                        "steps": steps},
        "kernels_ms": {k: round(t_ / a_, 4) for k, (a_, t_) in sorted(kt.items(), key=lambda kv: -kv[1][1])},
        "stream_benchmark": {"updates_per_s": n / stream_s, "GBps": 4 * 8 * dim * n / stream_s / 1e9},
        "hot_path_vs_stream": round((n / stream_s) / value, 3),
        "rapidt": rapidt,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", choices=["2", "3", "4", "5", "paper"], default="2")
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--scheme", choices=["pit", "pidt"], default="pit")
    ap.add_argument("--path", choices=["fused", "calls"], default="fused")
    ap.add_argument("--cpu-sample", type=int, default=16_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--knob", action="append", default=[], metavar="NAME=VALUE",
                    help="launch-shape knob of the tree (results do not depend on it)")
    # the paper's particle-handling benchmark (--config paper)
    ap.add_argument("--dim", type=int, choices=[2, 3], default=2)
    ap.add_argument("--particles", type=int, default=10_000_000)
    ap.add_argument("--start", choices=["homogeneous", "subbox"], default="homogeneous")
    ap.add_argument("--dt", type=float, default=1e-4)
    ap.add_argument("--ppc", type=int, default=1000)
    ap.add_argument("--flops", type=int, default=0)
    ap.add_argument("--max-level", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    if args.config != "paper":
        args.config = int(args.config)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (how it would shard is a design note); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    import paper_1508_02435_amd as pic
    global pic_capi
    from paper_1508_02435_amd import _capi as pic_capi

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    scheme = pic.PIT if args.scheme == "pit" else pic.PIDT
    if args.config == 5:
        return run_batched(args, scheme)
    if args.config == "paper":
        return run_paper(args, scheme)
    _log(f"[bench] generating config {args.config}")
    wl = {2: W.config2, 3: W.config3, 4: W.config4}[args.config]()
    tree = pic.Tree(wl.tree).upload(dev)
    for kv in args.knob:
        name, value = kv.split("=")
        pic.tune(name, int(value), tree)
    f32 = args.precision == "f32"
    qmdt, dt = wl.qm * wl.dt, wl.dt
    langmuir = args.config in (2, 4)
    warm, steps = max(args.warmup, 1), args.steps

    # The state at the start of the timed region and the field of every timed
    # step: configs 2 and 4 run the Langmuir plasma self-consistently (the
    # warmup steps included), config 3 keeps its prescribed field.
    gen = pic.Stepper(tree, scheme, wl.x, wl.v, q=wl.q, device=dev)
    gen.initial_sort()
    if langmuir:
        _log(f"[bench] self-consistent Langmuir run: {warm} warmup + {steps} timed steps (Poisson FP64 on the host)")
        langmuir_sequence(torch, gen, wl, warm, dev, first=True)
    else:
        pos = tree.vertex_table().T.astype(np.float64) / wl.tree.finest
        E0 = torch.tensor(wl.field(pos), dtype=torch.float64, device=dev)
        for _ in range(warm):
            gen.step_fused(E0, qmdt, dt, q_uniform=wl.q_uniform)
    torch.cuda.synchronize()
    snap = {k: getattr(gen, k).clone() for k in ("x", "v", "q", "start") if getattr(gen, k) is not None}
    fields = langmuir_sequence(torch, gen, wl, steps, dev) if langmuir else [E0] * steps
    x0_host, v0_host = snap["x"].cpu().numpy(), snap["v"].cpu().numpy()
    del gen
    torch.cuda.empty_cache()

    def fresh():
        """A stepper holding the state at the start of the timed region."""
        if f32:
            return pic.Stepper32(tree, scheme, snap["x"], snap["v"], dt=wl.dt, q=snap.get("q"), device=dev)
        st = pic.Stepper(tree, scheme, snap["x"], snap["v"], q=snap.get("q"), device=dev)
        st.start.copy_(snap["start"])
        return st

    accuracy = fp32_accuracy(pic, torch, tree, scheme, wl, x0_host, v0_host, fields[0], dev) if f32 else None
    knobs = pic.tuning(tree)
    ks, ed = knobs["key_stores"], knobs["emit_deposit"]
    stored = args.path == "fused" and (ks == 1 or (ks == 2 and f32 and wl.dim == 3))
    # the writing pass deposits (the library's rule: FP64 fused step, 2D
    # regular single tree, uniform charge, tiles of at most 2048)
    emit_dep = (args.path == "fused" and not f32 and wl.dim == 2 and tree.regular and tree.n_inst == 1 and
                wl.q is None and knobs["step_tile"] in (0, 1024, 2048) and
                (ed == 1 or (ed == 2 and scheme == pic.PIT)))
    # the key pass and the ranking as one kernel (the library's rule)
    sf = knobs["step_fuse"]
    fuse_auto = wl.dim == 2 and tree.regular and tree.n_inst == 1 and scheme == pic.PIT and ks != 1
    fused_rank = (args.path == "fused" and not f32 and knobs["step_tile"] in (0, 1024, 2048) and
                  (sf == 1 or (sf == 2 and fuse_auto)))
    ab = algorithmic_bytes_f32(wl.dim, wl.q is not None, stored) if f32 else \
        algorithmic_bytes(wl.dim, wl.q is not None, stored, emit_dep, fused_rank)
    lib = pic.lib()
    st = fresh()
    step = st.step_fused if args.path == "fused" else st.step
    _log(f"[bench] n={wl.n} leaves={tree.n_leaves} path={args.path} warmup={warm} steps={steps}")

    # one profiled step (every launch bracketed by events) names the dominant kernel
    lib.pic_profile_enable(1)
    kernel_times(lib)
    step(fields[0], qmdt, dt, q_uniform=wl.q_uniform)
    torch.cuda.synchronize()
    warm_k = kernel_times(lib)
    lib.pic_profile_enable(0)
    if tree.status_sync() != 0:
        raise RuntimeError("device status error during warmup")
    dominant = max((k for k in warm_k if k in ab), key=lambda k: warm_k[k][1] / warm_k[k][0])

    # timed region: the steps from the snapshot, events only around the dominant
    # kernel (on the library's stream)
    del st, step
    torch.cuda.empty_cache()
    st = fresh()
    step = st.step_fused if args.path == "fused" else st.step
    lib.pic_profile_enable(1)
    lib.pic_profile_only(dominant.encode())
    kernel_times(lib)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for k in range(steps):
        step(fields[k], qmdt, dt, q_uniform=wl.q_uniform)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gpu_ms_step = ev0.elapsed_time(ev1) / steps
    launches, total = kernel_times(lib)[dominant]
    lib.pic_profile_only(None)
    lib.pic_profile_enable(0)
    if tree.status_sync() != 0:
        raise RuntimeError("device status error in the timed region")

    # the same steps again: per-kernel table (every launch bracketed by events)
    # and the re-bin statistics (movers, lifts per particle, paper Sec. 6.1)
    del st, step
    torch.cuda.empty_cache()
    st = fresh()
    step = st.step_fused if args.path == "fused" else st.step
    stats = pic.new_stats(dev)
    lib.pic_profile_enable(1)
    kernel_times(lib)
    for k in range(steps):
        step(fields[k], qmdt, dt, q_uniform=wl.q_uniform, stats=stats)
    torch.cuda.synchronize()
    per_kernel = {}
    for name, (nl, tot) in sorted(kernel_times(lib).items(), key=lambda kv: -kv[1][1]):
        per_kernel[name] = {"launches": nl, "avg_ms": tot / nl}
    lib.pic_profile_enable(0)
    if tree.status_sync() != 0:
        raise RuntimeError("device status error in the profiled steps")
    rs = pic.read_stats(stats)
    rebin_stats = {"mover_fraction": rs["movers"] / rs["particles"],
                   "lifts_per_particle_step": rs["lifts"] / rs["particles"],
                   "max_tunnel_cells": rs["max_tunnel"],
                   "lift_histogram": rs["lift_hist"][:max(i for i, c in enumerate(rs["lift_hist"]) if c) + 1],
                   "steps": steps}

    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / steps
    value = wl.n * steps / elapsed
    _log(f"[bench] {ms_step:.3f} ms/step, {value:.4g} updates/s, mover fraction {rebin_stats['mover_fraction']:.3f}, "
         f"lifts/particle/step {rebin_stats['lifts_per_particle_step']:.3f}")

    avg_s = total / launches * 1e-3
    bytes_launch = ab[dominant] * wl.n
    achieved = bytes_launch / avg_s / 1e9
    workload = f"config{args.config}_{args.scheme}_{args.precision}_{args.path}"
    traffic = stored_traffic(dominant, workload)
    step_bytes = ab[args.path]
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "bytes_per_launch_algorithmic": bytes_launch,
                "step_bytes_per_particle": step_bytes,
                "step_algorithmic_GBps": round(step_bytes * value / 1e9, 1),
                "step_frac": round(step_bytes * value / 1e9 / HBM_PEAK_GBS, 4),
                # the same step priced at the three-call ABI's bytes (each call streams its own
                # inputs and outputs once), the yardstick of the 60%-of-HBM target
                "three_call_bytes_per_particle": ab["calls"],
                "three_call_frac": round(ab["calls"] * value / 1e9 / HBM_PEAK_GBS, 4)}

    stream = None
    if not args.no_stream and not f32:
        # the paper's stream benchmark on the same arrays: explicit Euler + reflecting walls, no grid
        xs = (C.c_void_p * 3)(*[st.x2[k].data_ptr() if k < wl.dim else None for k in range(3)])
        vs = (C.c_void_p * 3)(*[st.v2[k].data_ptr() if k < wl.dim else None for k in range(3)])
        st.x2.copy_(st.x)
        st.v2.copy_(st.v)
        stream_ptr = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        for _ in range(3):
            lib.pic_stream_push(wl.dim, wl.n, xs, vs, 1e-3, stream_ptr)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(steps):
            lib.pic_stream_push(wl.dim, wl.n, xs, vs, 1e-3, stream_ptr)
        torch.cuda.synchronize()
        s_el = (time.perf_counter() - s0) / steps
        stream = {"updates_per_s": wl.n / s_el, "GBps": 4 * 8 * wl.dim * wl.n / s_el / 1e9}

    cpu = None
    if not args.no_cpu_baseline and not f32:
        _log(f"[bench] cpu baseline on up to {args.cpu_sample} particles")
        wl.x, wl.v = x0_host, v0_host      # the state at the start of the timed region
        wl.q = snap["q"].cpu().numpy() if "q" in snap else None
        cpu = cpu_baseline(wl, scheme, min(args.cpu_sample, wl.n), fields[0].cpu().numpy())

    out = {
        "metric": METRIC, "value": value, "unit": "particle updates/s", "n_gpus": 1,
        "steps": steps, "warmup": warm, "ms_per_step": ms_step, "higher_is_better": True,
        # stream time of the same timed steps (first launch to last completion), beside the wall clock
        "gpu_ms_per_step": round(gpu_ms_step, 4),
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if f32 else "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config].format(n=wl.n, leaves=int(tree.n_leaves)) +
                               f", {args.scheme.upper()}, {'FP32 offsets' if f32 else 'FP64'}, {args.path} path" +
                               (", self-consistent Langmuir field (Poisson FP64 outside the timed hot path)"
                                if langmuir else ", prescribed field"),
                   "particles": wl.n, "leaves": int(tree.n_leaves), "scheme": args.scheme, "path": args.path,
                   "knobs": pic.tuning(tree)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        # per-launch averages from a second run of the same steps with every
        # launch bracketed by events and the re-bin statistics on (rebin_stats
        # is that run's statistics kernel, not part of the timed step)
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in per_kernel.items()},
        "rebin_stats": rebin_stats,
        "stream_benchmark": stream,
    }
    if accuracy is not None:
        out["fp32_vs_fp64"] = accuracy
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
