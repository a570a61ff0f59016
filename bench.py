#!/usr/bin/env python3
"""Benchmark of the spacetree PIC hot path on one MI355X.

One step = pic_gather_push + pic_rebin + pic_deposit over the whole particle
set, inputs resident in HBM.  Default workload: 2D periodic regular depth-5
spacetree (243 x 243 leaves), 15,116,544 electrons (256 per cell, Maxwellian
v_th = 1 cell/step plus 1% beam particles at 8-20 cells/step, 1% density
perturbation on modes 1..4), PIT, FP64.  The field is the linear-theory
Langmuir field of the perturbation, fixed over the run (the Poisson solve is
not part of the step).

Prints one JSON line (the benchmark contract) with the whole-step throughput,
a roofline entry for the dominant kernel (algorithmic bytes over its average
HIP-event duration in the timed region) and the serial FP64 oracle timed on a
bounded sample on the host as a CPU baseline.
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


def algorithmic_bytes(dim: int, per_particle_q: bool):
    """Bytes each kernel must move per particle (FP64 form)."""
    s_push = 2 * 8 * dim                   # x, v read and written by gather_push
    s_rec = s_push + (8 if per_particle_q else 0)
    s_dep = 8 * dim + (8 if per_particle_q else 0)
    return {
        "gather_push": 2 * s_push + 4,     # + the new bin written
        "rebin_tiles": 4,                  # bins read
        "rebin_scatter": 2 * s_rec,        # every record read and written once
        "deposit_bins": s_dep,
        "step": 2 * s_push + 2 * s_rec + s_dep + 8,
    }


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
    xs, vs, _, start, _ = oracle.initial_sort(o, x, v, None, scheme)
    steps, spent = 0, 0.0
    while spent < min_seconds and steps < max_steps:
        t0 = time.perf_counter()
        r = oracle.step(o, xs, vs, E_np, wl.qm * wl.dt, wl.dt, start, scheme, None, wl.q_uniform)
        spent += time.perf_counter() - t0
        xs, vs, start = r["x"], r["v"], r["bin_start"]
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


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if still valid."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel)
    if not ent:
        return None
    src = os.path.join(ROOT, ent["source"])
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if digest != ent.get("source_sha256"):
        return None                       # the kernel changed since the counters were taken
    return ent["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scheme", choices=["pit", "pidt"], default="pit")
    ap.add_argument("--ppc", type=int, default=256)
    ap.add_argument("--cpu-sample", type=int, default=16_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (sharding is a design note); "
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
    _log(f"[bench] generating config2 (ppc={args.ppc})")
    wl = W.config2(ppc=args.ppc)
    tree = pic.Tree(wl.tree).upload(dev)
    pos = tree.vertex_table().T.astype(np.float64) / wl.tree.finest
    E_np = wl.field(pos)
    E = torch.tensor(E_np, dtype=torch.float64, device=dev)
    st = pic.Stepper(tree, scheme, wl.x, wl.v, device=dev)
    st.initial_sort()
    torch.cuda.synchronize()
    qmdt, dt = wl.qm * wl.dt, wl.dt
    _log(f"[bench] n={wl.n} leaves={tree.n_leaves} warmup={args.warmup} steps={args.steps}")
    for _ in range(args.warmup):
        st.step(E, qmdt, dt, q_uniform=wl.q_uniform)
    torch.cuda.synchronize()
    if tree.status_sync() != 0:
        raise RuntimeError("device status error during warmup")

    lib = pic.lib()
    lib.pic_profile_enable(1)
    kernel_times(lib)                       # drop anything recorded so far
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st.step(E, qmdt, dt, q_uniform=wl.q_uniform)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = kernel_times(lib)
    lib.pic_profile_enable(0)
    if tree.status_sync() != 0:
        raise RuntimeError("device status error in the timed region")
    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps
    value = wl.n * args.steps / elapsed
    _log(f"[bench] {ms_step:.3f} ms/step, {value:.4g} updates/s")

    ab = algorithmic_bytes(wl.dim, False)
    per_kernel = {}
    for name, (launches, total) in sorted(kt.items(), key=lambda kv: -kv[1][1]):
        per_kernel[name] = {"launches": launches, "avg_ms": total / launches}
    dominant = max((k for k in per_kernel if k in ab), key=lambda k: per_kernel[k]["avg_ms"])
    avg_s = per_kernel[dominant]["avg_ms"] * 1e-3
    bytes_launch = ab[dominant] * wl.n
    achieved = bytes_launch / avg_s / 1e9
    workload = f"config2_{args.scheme}_f64_ppc{args.ppc}"
    traffic = stored_traffic(dominant, workload)
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "bytes_per_launch_algorithmic": bytes_launch,
                "step_algorithmic_GBps": round(ab["step"] * value / 1e9, 1),
                "step_frac": round(ab["step"] * value / 1e9 / HBM_PEAK_GBS, 4)}

    # paper's stream benchmark on the same arrays: explicit Euler + reflecting walls, no grid
    xs = (C.c_void_p * 3)(*[st.x2[k].data_ptr() if k < wl.dim else None for k in range(3)])
    vs = (C.c_void_p * 3)(*[st.v2[k].data_ptr() if k < wl.dim else None for k in range(3)])
    st.x2.copy_(st.x)
    st.v2.copy_(st.v)
    stream_ptr = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(3):
        lib.pic_stream_push(wl.dim, wl.n, xs, vs, 1e-3, stream_ptr)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for _ in range(args.steps):
        lib.pic_stream_push(wl.dim, wl.n, xs, vs, 1e-3, stream_ptr)
    torch.cuda.synchronize()
    s_el = (time.perf_counter() - s0) / args.steps
    stream = {"updates_per_s": wl.n / s_el, "GBps": 4 * 8 * wl.dim * wl.n / s_el / 1e9}

    cpu = None
    if not args.no_cpu_baseline:
        _log(f"[bench] cpu baseline on {args.cpu_sample} particles")
        cpu = cpu_baseline(wl, scheme, min(args.cpu_sample, wl.n), E_np)

    out = {
        "metric": METRIC, "value": value, "unit": "particle updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2D periodic regular depth-5 spacetree (243x243 leaves), {wl.n} electrons "
                               f"({args.ppc}/cell, v_th 1 cell/step, 1% beam 8-20 cells/step), "
                               f"{args.scheme.upper()}, FP64",
                   "particles": wl.n, "leaves": int(tree.n_leaves), "scheme": args.scheme},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in per_kernel.items()},
        "stream_benchmark": stream,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
