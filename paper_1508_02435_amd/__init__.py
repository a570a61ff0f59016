"""MI355X spacetree particle-in-cell hot path: Python binding of libpic.so.

The arithmetic runs in the HIP kernels of ``libpic.so`` (see ``include/pic.h``
for the C ABI).  This module only marshals arguments: PyTorch provides device
memory and the current HIP stream.  There is no CPU fallback; if the library
or a GPU is missing the calls raise.

Paper: "Two Particle-in-Grid Realisations on Spacetrees" (Sec. 3 PIC cycle,
Sec. 4 spacetree and dual grid, Sec. 5.1 PIT, Sec. 5.2 PIDT).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _capi
from ._capi import F32_OFFSET, F64, PIDT, PIT, PicError, check, lib

__all__ = ["Tree", "PIT", "PIDT", "F64", "F32_OFFSET", "PicError", "locate", "gather_push", "rebin",
           "deposit", "scratch_bytes", "Stepper", "Stepper32", "lib", "tune", "tuning", "TUNING_KNOBS", "step",
           "new_stats", "read_stats"]


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _need(cond: bool, what: str):
    if not cond:
        raise ValueError(what)


def _check_soa(t, dim: int, n: int, dtype_name: str, what: str):
    import torch
    _need(t is not None and t.is_cuda and t.is_contiguous(), f"{what}: contiguous device tensor expected")
    _need(t.dim() == 2 and t.shape[0] >= dim and t.shape[1] == n, f"{what}: shape (dim, n) expected")
    _need(t.dtype == getattr(torch, dtype_name), f"{what}: {dtype_name} expected")


def _check_vec(t, n: int, what: str):
    _need(t is not None and t.is_cuda and t.is_contiguous() and t.numel() >= n, f"{what}: >= {n} elements on device")


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class RefineMasks:
    """A tree description as pic_tree_create takes it: refine flags per
    level (``refine[l]``, (3^l)^dim bytes, lexicographic, axis 0 fastest)."""

    def __init__(self, dim: int, max_level: int, refine):
        self.dim, self.max_level, self.refine = dim, max_level, list(refine)

    def masks_concat(self):
        if not self.refine:
            return np.zeros(0, np.uint8)
        return np.ascontiguousarray(np.concatenate([np.asarray(m, np.uint8).ravel() for m in self.refine]))


class Tree:
    """A forest of spacetrees (one or more instances of the same dimension).

    ``specs``: objects with ``dim``, ``max_level`` and ``masks_concat()``
    (refine flags per level, lexicographic, axis 0 fastest).
    """

    def __init__(self, specs):
        if not isinstance(specs, (list, tuple)):
            specs = [specs]
        dim = specs[0].dim
        assert all(s.dim == dim for s in specs)
        levels = np.array([s.max_level for s in specs], np.int32)
        masks = np.concatenate([s.masks_concat() for s in specs] + [np.zeros(1, np.uint8)])
        self._masks = np.ascontiguousarray(masks)
        self.specs = list(specs)
        h = C.c_void_p()
        check(lib().pic_tree_create(dim, len(specs), levels.ctypes.data_as(C.c_void_p),
                                    self._masks.ctypes.data_as(C.c_void_p), C.byref(h)), "pic_tree_create")
        self._h = h
        self._lib = lib()
        info = _capi.TreeInfo()
        check(lib().pic_tree_get_info(self._h, C.byref(info)), "pic_tree_get_info")
        self.info = info
        self.dim = info.dim
        self.n_inst = info.n_inst
        self.n_leaves = info.n_leaves
        self.n_vertices = info.n_vertices
        self.n_pidt = info.n_pidt
        self.regular = bool(info.regular)
        self.buffer = None

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(self, "_lib", None)
        if h is not None and h.value and L is not None:
            L.pic_tree_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def n_bins(self, scheme: int) -> int:
        return self.n_leaves if scheme == PIT else self.n_pidt

    def instance(self, i: int) -> _capi.InstanceInfo:
        ii = _capi.InstanceInfo()
        check(lib().pic_tree_get_instance(self._h, i, C.byref(ii)), "pic_tree_get_instance")
        return ii

    # host tables -------------------------------------------------------------
    def leaf_table(self):
        nl, d, nc = self.n_leaves, self.dim, 1 << self.dim
        key = np.zeros(nl, np.uint64)
        level = np.zeros(nl, np.int32)
        coord = np.zeros((nl, d), np.int64)
        vtx = np.zeros((nl, nc), np.int32)
        pidt = np.zeros((nl, nc), np.int32)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        check(lib().pic_tree_leaf_table(self._h, p(key), p(level), p(coord), p(vtx), p(pidt)), "leaf_table")
        return {"key": key, "level": level, "coord": coord, "vtx": vtx, "pidt": pidt}

    def vertex_table(self):
        pos = np.zeros((self.n_vertices, self.dim), np.int64)
        check(lib().pic_tree_vertex_table(self._h, pos.ctypes.data_as(C.c_void_p)), "vertex_table")
        return pos

    def pidt_table(self):
        n, d = self.n_pidt, self.dim
        key = np.zeros(n, np.uint64)
        level = np.zeros(n, np.int32)
        b = np.zeros((n, d), np.int64)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        check(lib().pic_tree_pidt_table(self._h, p(key), p(level), p(b)), "pidt_table")
        return {"key": key, "level": level, "b": b}

    # device ------------------------------------------------------------------
    def upload(self, device="cuda", stream=None):
        import torch
        nbytes = int(self.info.device_bytes)
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        self.buffer = buf
        check(lib().pic_tree_upload(self._h, C.c_void_p(buf.data_ptr() + off), nbytes, C.c_void_p(_stream(stream))),
              "pic_tree_upload")
        return self

    def status_sync(self, stream=None) -> int:
        return lib().pic_status_sync(self._h, C.c_void_p(_stream(stream)))


def _particles(n, x=None, v=None, off=None, u=None, inst_start=None) -> _capi.Particles:
    P = _capi.Particles()
    P.n = int(n)
    for k in range(3):
        P.x[k] = _ptr(x[k]) if x is not None and k < x.shape[0] else None
        P.v[k] = _ptr(v[k]) if v is not None and k < v.shape[0] else None
        P.off[k] = _ptr(off[k]) if off is not None and k < off.shape[0] else None
        P.u[k] = _ptr(u[k]) if u is not None and k < u.shape[0] else None
    P.inst_start_dev = _ptr(inst_start)
    return P


def _to_dev(a, dtype, dev):
    """A contiguous device copy of a NumPy array or tensor (None stays None)."""
    import torch
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=dev, dtype=dtype if dtype is not None else a.dtype, copy=True).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev).contiguous()


def _check_inst(tree, inst_start):
    if tree.n_inst > 1:
        _check_vec(inst_start, tree.n_inst + 1, "inst_start")


TUNING_KNOBS = {"rebin_tile": (2048, 4096), "rebin_radix": (4, 5), "scatter_mode": (0, 1), "scatter_nt": (0, 1),
                "scatter_group": (1, 2, 4), "deposit_lanes": (0, 16, 32, 64), "step_tile": (0, 2048, 1024, 4096),
                "xcd_tiles": (1, 0), "emit_threads": (1024, 512), "deposit_bpw": (1, 2), "deposit_batch": (64, 256), "step_fuse": (2, 0, 1), "emit_deposit": (2, 0, 1),
                "group_match": (0, 1), "key_stores": (2, 0, 1),
                "regular_tables": (1, 0)}
PROCESS_ONLY = ("regular_tables",)   # read when a tree is created; not a knob of a tree


def tune(name: str, value: int, tree: Optional["Tree"] = None):
    """Set a launch-shape knob (results do not depend on it): of one tree, or
    the process default that trees created afterwards copy."""
    if tree is None:
        check(lib().pic_tune_set(name.encode(), int(value)), f"pic_tune_set({name}={value})")
    else:
        check(lib().pic_tree_tune_set(tree.handle, name.encode(), int(value)), f"pic_tree_tune_set({name}={value})")


def tuning(tree: Optional["Tree"] = None) -> dict:
    """Knob values of one tree, or the process defaults."""
    if tree is None:
        return {k: int(lib().pic_tune_get(k.encode())) for k in TUNING_KNOBS}
    return {k: int(lib().pic_tree_tune_get(tree.handle, k.encode())) for k in TUNING_KNOBS if k not in PROCESS_ONLY}


def new_stats(device="cuda"):
    """A zeroed device record for the re-bin statistics (int64 words)."""
    import torch
    return torch.zeros(_capi.STATS_WORDS, dtype=torch.int64, device=device)


def read_stats(stats) -> dict:
    """The re-bin statistics record as a dict (particles, movers, lifts,
    max_tunnel, lift_hist)."""
    a = stats.cpu().numpy()
    return {"particles": int(a[0]), "movers": int(a[1]), "lifts": int(a[2]), "max_tunnel": int(a[3]),
            "lift_hist": [int(x) for x in a[4:4 + _capi.STATS_LEVELS]]}


def scratch_bytes(tree: Tree, n: int, scheme: int, precision: int = F64) -> int:
    return int(lib().pic_scratch_bytes(tree.handle, int(n), scheme, precision))


def locate(tree: Tree, scheme: int, x, bin_out, inst_start=None, stream=None):
    """Bins of an (unsorted) FP64 set: x is a (dim, n) float64 device tensor."""
    _check_soa(x, tree.dim, x.shape[1], "float64", "x")
    _check_vec(bin_out, x.shape[1], "bin_out")
    _check_inst(tree, inst_start)
    P = _particles(x.shape[1], x=x, inst_start=inst_start)
    check(lib().pic_locate(tree.handle, scheme, F64, C.byref(P), None, C.c_void_p(_ptr(bin_out)),
                           C.c_void_p(_stream(stream))), "pic_locate")


def gather_push(tree: Tree, scheme: int, x, v, E, qmdt: float, dt: float, bin_out, Ep=None,
                inst_start=None, qmdt_dev=None, dt_dev=None, stream=None):
    """In-place leapfrog step of an FP64 set; writes new bins to bin_out."""
    n = x.shape[1]
    _check_soa(x, tree.dim, n, "float64", "x")
    _check_soa(v, tree.dim, n, "float64", "v")
    _check_vec(bin_out, n, "bin_out")
    for k in range(tree.dim):
        _check_vec(E[k], tree.n_vertices, f"E[{k}]")
    if Ep is not None:
        _check_soa(Ep, tree.dim, n, "float64", "Ep")
    _check_inst(tree, inst_start)
    for a in (qmdt_dev, dt_dev):
        if a is not None:
            _check_vec(a, tree.n_inst, "per-instance parameter")
    P = _particles(x.shape[1], x=x, v=v, inst_start=inst_start)
    Eptr = (C.c_void_p * 3)(*[_ptr(E[k]) if k < tree.dim else None for k in range(3)])
    pp = _capi.PushParams(_ptr(qmdt_dev), _ptr(dt_dev))
    check(lib().pic_gather_push(tree.handle, scheme, F64, C.byref(P), Eptr, float(qmdt), float(dt),
                                C.byref(pp), None, C.c_void_p(_ptr(bin_out)),
                                C.c_void_p(_ptr(Ep)) if Ep is not None else None,
                                C.c_void_p(_stream(stream))), "pic_gather_push")


def free_stream(tree: Tree, scheme: int, x, v, dt: float, boundary: int, flops: int, bin_out, inst_start=None,
                dt_dev=None, stream=None):
    """In-place free-streaming move of an FP64 set (no field), periodic or
    reflecting walls, ``flops`` artificial operations per move; writes the
    new bins to bin_out."""
    n = x.shape[1]
    _check_soa(x, tree.dim, n, "float64", "x")
    _check_soa(v, tree.dim, n, "float64", "v")
    _check_vec(bin_out, n, "bin_out")
    _check_inst(tree, inst_start)
    if dt_dev is not None:
        _check_vec(dt_dev, tree.n_inst, "per-instance dt")
    P = _particles(n, x=x, v=v, inst_start=inst_start)
    pp = _capi.PushParams(None, _ptr(dt_dev))
    check(lib().pic_free_stream(tree.handle, scheme, F64, C.byref(P), float(dt), C.byref(pp), int(boundary),
                                int(flops), C.c_void_p(_ptr(bin_out)), C.c_void_p(_stream(stream))),
          "pic_free_stream")


def stream_step(tree: Tree, scheme: int, x, v, dt: float, boundary: int, flops: int, bin_start, x_out, v_out,
                new_start, scratch, extra_in=(), extra_out=(), stats=None, stream=None):
    """Free streaming and the stable re-bin in one call (the passes of
    pic_step, no deposit); x, v are the sorted input, x_out/v_out receive
    the re-binned set."""
    n = x.shape[1]
    for a, nm in ((x, "x"), (v, "v"), (x_out, "x_out"), (v_out, "v_out")):
        _check_soa(a, tree.dim, n, "float64", nm)
    nb = tree.n_bins(scheme)
    _check_vec(bin_start, nb + 1, "bin_start")
    _check_vec(new_start, nb + 1, "new_start")
    _need(len(extra_in) == len(extra_out), "extra column lists differ in length")
    for a, b in zip(extra_in, extra_out):
        _check_vec(a, n, "extra in")
        _check_vec(b, n, "extra out")
    P = _particles(n, x=x, v=v)
    Q = _particles(n, x=x_out, v=v_out)
    ne = len(extra_in)
    ins = (C.c_void_p * max(ne, 1))(*[_ptr(c) for c in extra_in])
    outs = (C.c_void_p * max(ne, 1))(*[_ptr(c) for c in extra_out])
    sizes = (C.c_int32 * max(ne, 1))(*[c.element_size() for c in extra_in])
    check(lib().pic_stream_step(tree.handle, scheme, C.byref(P), C.c_void_p(_ptr(bin_start)), float(dt),
                                int(boundary), int(flops), ne, ins, outs, sizes, C.byref(Q),
                                C.c_void_p(_ptr(new_start)), C.c_void_p(_ptr(scratch)),
                                scratch.numel() * scratch.element_size(), _stats_ptr(stats),
                                C.c_void_p(_stream(stream))), "pic_stream_step")


def leaf_counts(tree: Tree, x, count_out, inst_start=None, stream=None):
    """Particles per leaf of an FP64 set (any order) into count_out (int64
    device tensor, one entry per leaf)."""
    n = x.shape[1]
    _check_soa(x, tree.dim, n, "float64", "x")
    _check_vec(count_out, tree.n_leaves, "count_out")
    _need(count_out.element_size() == 8, "count_out must hold 64-bit integers")
    _check_inst(tree, inst_start)
    P = _particles(n, x=x, inst_start=inst_start)
    check(lib().pic_leaf_counts(tree.handle, C.byref(P), C.c_void_p(_ptr(count_out)), C.c_void_p(_stream(stream))),
          "pic_leaf_counts")


def vmax(tree: Tree, scheme: int, x, v, bin_start, dt: float, scratch, stream=None):
    """raPIDT's per-cell v_max and the predicate v_max dt <= h of a sorted
    single-tree set: returns two device tensors (float64, uint8), one entry
    per cell position of levels 0..L in the refine-mask layout."""
    import torch
    n = x.shape[1]
    _check_soa(x, tree.dim, n, "float64", "x")
    _check_soa(v, tree.dim, n, "float64", "v")
    _check_vec(bin_start, tree.n_bins(scheme) + 1, "bin_start")
    L, d = tree.specs[0].max_level, tree.dim
    cells = (3 ** (d * (L + 1)) - 1) // (3 ** d - 1)
    out = torch.empty(cells, dtype=torch.float64, device=x.device)
    quiet = torch.empty(cells, dtype=torch.uint8, device=x.device)
    P = _particles(n, x=x, v=v)
    check(lib().pic_vmax(tree.handle, scheme, C.byref(P), C.c_void_p(_ptr(bin_start)), float(dt),
                         C.c_void_p(_ptr(out)), C.c_void_p(_ptr(quiet)), C.c_void_p(_ptr(scratch)),
                         scratch.numel() * scratch.element_size(), C.c_void_p(_stream(stream))), "pic_vmax")
    return out, quiet


def adapt(tree: Tree, leaf_count, ppc: int, max_level: int):
    """One ppc-driven adaptation of a single tree (host): returns the new
    tree's TreeSpec (refine masks), or None when nothing changes."""
    cnt = np.ascontiguousarray(np.asarray(leaf_count, dtype=np.int64))
    _need(cnt.shape == (tree.n_leaves,), "leaf_count needs one entry per leaf")
    ln, nl = C.c_size_t(0), C.c_int32(0)
    L0, d = tree.specs[0].max_level, tree.dim
    deepest = max(L0, min(L0 + 1, int(max_level)))
    masks = np.zeros(max(sum(3 ** (d * lev) for lev in range(deepest)), 1), np.uint8)
    check(lib().pic_tree_adapt(tree.handle, cnt.ctypes.data, int(ppc), int(max_level), masks.ctypes.data,
                               masks.size, C.byref(ln), C.byref(nl)), "pic_tree_adapt")
    L = nl.value
    levels, off = [], 0
    for lev in range(L):
        k = 3 ** (d * lev)
        levels.append(masks[off:off + k].copy())
        off += k
    old = tree.specs[0]
    if old.max_level == L and np.array_equal(np.asarray(old.masks_concat(), np.uint8).ravel(),
                                             np.concatenate(levels) if levels else np.zeros(0, np.uint8)):
        return None
    return RefineMasks(d, L, levels)


def rebin(tree: Tree, scheme: int, new_bin, old_start, cols_in: Sequence, cols_out: Sequence, new_start,
          scratch, stats=None, stream=None):
    """Stable re-bin; permutes every column of cols_in into cols_out."""
    n = new_bin.numel()
    _check_vec(new_bin, n, "new_bin")
    nb = tree.n_bins(scheme)
    if old_start is not None:
        _check_vec(old_start, nb + 1, "old_start")
    _check_vec(new_start, nb + 1, "new_start")
    _need(len(cols_in) == len(cols_out), "column lists differ in length")
    for a, b in zip(cols_in, cols_out):
        _check_vec(a, n, "column in")
        _check_vec(b, n, "column out")
        _need(a.element_size() == b.element_size(), "column widths differ")
    nc = len(cols_in)
    ins = (C.c_void_p * max(nc, 1))(*[_ptr(c) for c in cols_in])
    outs = (C.c_void_p * max(nc, 1))(*[_ptr(c) for c in cols_out])
    sizes = (C.c_int32 * max(nc, 1))(*[c.element_size() for c in cols_in])
    check(lib().pic_rebin(tree.handle, scheme, n, C.c_void_p(_ptr(new_bin)),
                          C.c_void_p(_ptr(old_start)) if old_start is not None else None,
                          nc, ins, outs, sizes, C.c_void_p(_ptr(new_start)), C.c_void_p(_ptr(scratch)),
                          scratch.numel() * scratch.element_size(), _stats_ptr(stats),
                          C.c_void_p(_stream(stream))), "pic_rebin")


def _stats_ptr(stats):
    if stats is None:
        return None
    _check_vec(stats, _capi.STATS_WORDS, "stats")
    _need(stats.element_size() == 8, "stats: 64-bit words expected")
    return C.c_void_p(_ptr(stats))


def deposit(tree: Tree, scheme: int, x, bin_start, rho, scratch, q=None, q_uniform: float = 0.0,
            inst_start=None, stream=None):
    """Vertex charge of a sorted FP64 set."""
    n = x.shape[1]
    _check_soa(x, tree.dim, n, "float64", "x")
    _check_vec(bin_start, tree.n_bins(scheme) + 1, "bin_start")
    _check_vec(rho, tree.n_vertices, "rho")
    if q is not None:
        _check_vec(q, n, "q")
    _check_inst(tree, inst_start)
    P = _particles(x.shape[1], x=x, inst_start=inst_start)
    check(lib().pic_deposit(tree.handle, scheme, F64, C.byref(P), C.c_void_p(_ptr(bin_start)),
                            C.c_void_p(_ptr(q)) if q is not None else None, float(q_uniform),
                            C.c_void_p(_ptr(rho)), C.c_void_p(_ptr(scratch)),
                            scratch.numel() * scratch.element_size(), C.c_void_p(_stream(stream))),
          "pic_deposit")


def step(tree: Tree, scheme: int, x, v, E, qmdt: float, dt: float, bin_start, x_out, v_out, new_start, rho,
         scratch, extra_in=(), extra_out=(), q_column: int = -1, q_uniform: float = 0.0, inst_start=None,
         qmdt_dev=None, dt_dev=None, stats=None, stream=None):
    """Fused whole step (gather+push, re-bin into x_out/v_out, deposit); x, v are consumed."""
    n = x.shape[1]
    for a, nm in ((x, "x"), (v, "v"), (x_out, "x_out"), (v_out, "v_out")):
        _check_soa(a, tree.dim, n, "float64", nm)
    for k in range(tree.dim):
        _check_vec(E[k], tree.n_vertices, f"E[{k}]")
    nb = tree.n_bins(scheme)
    _check_vec(bin_start, nb + 1, "bin_start")
    _check_vec(new_start, nb + 1, "new_start")
    _check_vec(rho, tree.n_vertices, "rho")
    _check_inst(tree, inst_start)
    _need(len(extra_in) == len(extra_out), "extra column lists differ in length")
    for a, b in zip(extra_in, extra_out):
        _check_vec(a, n, "extra in")
        _check_vec(b, n, "extra out")
    for a in (qmdt_dev, dt_dev):
        if a is not None:
            _check_vec(a, tree.n_inst, "per-instance parameter")
    P = _particles(n, x=x, v=v, inst_start=inst_start)
    Q = _particles(n, x=x_out, v=v_out, inst_start=inst_start)
    Eptr = (C.c_void_p * 3)(*[_ptr(E[k]) if k < tree.dim else None for k in range(3)])
    pp = _capi.PushParams(_ptr(qmdt_dev), _ptr(dt_dev))
    ne = len(extra_in)
    ins = (C.c_void_p * max(ne, 1))(*[_ptr(c) for c in extra_in])
    outs = (C.c_void_p * max(ne, 1))(*[_ptr(c) for c in extra_out])
    sizes = (C.c_int32 * max(ne, 1))(*[c.element_size() for c in extra_in])
    check(lib().pic_step(tree.handle, scheme, F64, C.byref(P), C.c_void_p(_ptr(bin_start)), Eptr, float(qmdt),
                         float(dt), C.byref(pp), ne, ins, outs, sizes, int(q_column), float(q_uniform), C.byref(Q),
                         C.c_void_p(_ptr(new_start)), C.c_void_p(_ptr(rho)), C.c_void_p(_ptr(scratch)),
                         scratch.numel() * scratch.element_size(), _stats_ptr(stats), C.c_void_p(_stream(stream))),
          "pic_step")


class Stepper:
    """Device state of one particle set and the three calls of a time step.

    Holds two SoA buffers (the re-bin writes into the other one), the bin
    array, the segment offsets and one scratch buffer.  Optional per-particle
    charge ``q`` and integer tags ``ids`` travel with the particles.
    """

    def __init__(self, tree: Tree, scheme: int, x, v, q=None, ids=None, inst_start=None, device="cuda"):
        import torch
        self.tree, self.scheme = tree, scheme
        self.n = int(x.shape[1])
        dev = torch.device(device)
        self.x = _to_dev(x, torch.float64, dev)
        self.v = _to_dev(v, torch.float64, dev)
        self.q = _to_dev(q, torch.float64, dev)
        self.ids = _to_dev(ids, None, dev)
        self.x2 = torch.empty_like(self.x)
        self.v2 = torch.empty_like(self.v)
        self.q2 = None if self.q is None else torch.empty_like(self.q)
        self.ids2 = None if self.ids is None else torch.empty_like(self.ids)
        self.bin = torch.empty(self.n, dtype=torch.int32, device=dev)
        nb = tree.n_bins(scheme)
        self.start = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        self.start2 = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        self.scratch = torch.empty(scratch_bytes(tree, self.n, scheme) // 8 + 1, dtype=torch.int64, device=dev)
        self.rho = torch.zeros(tree.n_vertices, dtype=torch.float64, device=dev)
        self.Ep = None
        self.inst_start = inst_start

    def _cols(self, a, b):
        ins = [a[0][k] for k in range(self.tree.dim)] + [a[1][k] for k in range(self.tree.dim)]
        outs = [b[0][k] for k in range(self.tree.dim)] + [b[1][k] for k in range(self.tree.dim)]
        if self.q is not None:
            ins.append(a[2]); outs.append(b[2])
        if self.ids is not None:
            ins.append(a[3]); outs.append(b[3])
        return ins, outs

    def _swap(self):
        self.x, self.x2 = self.x2, self.x
        self.v, self.v2 = self.v2, self.v
        self.q, self.q2 = self.q2, self.q
        self.ids, self.ids2 = self.ids2, self.ids
        self.start, self.start2 = self.start2, self.start

    def initial_sort(self):
        locate(self.tree, self.scheme, self.x, self.bin, inst_start=self.inst_start)
        ins, outs = self._cols((self.x, self.v, self.q, self.ids), (self.x2, self.v2, self.q2, self.ids2))
        rebin(self.tree, self.scheme, self.bin, None, ins, outs, self.start2, self.scratch)
        self._swap()

    def gather_push(self, E, qmdt, dt, want_Ep=False, **kw):
        import torch
        if want_Ep and self.Ep is None:
            self.Ep = torch.empty_like(self.x)
        gather_push(self.tree, self.scheme, self.x, self.v, E, qmdt, dt, self.bin,
                    Ep=self.Ep if want_Ep else None, inst_start=self.inst_start, **kw)

    def rebin(self, stats=None):
        ins, outs = self._cols((self.x, self.v, self.q, self.ids), (self.x2, self.v2, self.q2, self.ids2))
        rebin(self.tree, self.scheme, self.bin, self.start, ins, outs, self.start2, self.scratch, stats=stats)
        self._swap()

    def deposit(self, q_uniform=0.0):
        deposit(self.tree, self.scheme, self.x, self.start, self.rho, self.scratch, q=self.q,
                q_uniform=q_uniform, inst_start=self.inst_start)

    def step(self, E, qmdt, dt, q_uniform=0.0, stats=None, **kw):
        """Three separate calls: gather_push, rebin, deposit."""
        self.gather_push(E, qmdt, dt, **kw)
        self.rebin(stats)
        self.deposit(q_uniform)

    def step_fused(self, E, qmdt, dt, q_uniform=0.0, qmdt_dev=None, dt_dev=None, stats=None):
        """The same step through the single fused call."""
        extra_in, extra_out = [], []
        q_col = -1
        if self.q is not None:
            q_col = len(extra_in)
            extra_in.append(self.q); extra_out.append(self.q2)
        if self.ids is not None:
            extra_in.append(self.ids); extra_out.append(self.ids2)
        step(self.tree, self.scheme, self.x, self.v, E, qmdt, dt, self.start, self.x2, self.v2, self.start2,
             self.rho, self.scratch, extra_in, extra_out, q_col, q_uniform, inst_start=self.inst_start,
             qmdt_dev=qmdt_dev, dt_dev=dt_dev, stats=stats)
        self._swap()


class FreeStreamRun(Stepper):
    """The particle-handling benchmark of the paper's results section on one
    tree: free streaming (pic_free_stream), the stable re-bin (pic_rebin),
    and the ppc-driven adaptation of the tree (pic_leaf_counts,
    pic_tree_adapt, a new tree, pic_locate and pic_rebin against it)."""

    def __init__(self, tree: Tree, scheme: int, x, v, ids=None, device="cuda"):
        super().__init__(tree, scheme, x, v, ids=ids, device=device)
        self.device = device

    def move(self, dt: float, boundary: int = _capi.REFLECTING, flops: int = 0):
        free_stream(self.tree, self.scheme, self.x, self.v, dt, boundary, flops, self.bin)

    def step_free(self, dt: float, boundary: int = _capi.REFLECTING, flops: int = 0, stats=None):
        """Free streaming, then the re-bin (two calls)."""
        self.move(dt, boundary, flops)
        self.rebin(stats)

    def step_free_fused(self, dt: float, boundary: int = _capi.REFLECTING, flops: int = 0, stats=None):
        """The same step in one call (pic_stream_step)."""
        extra_in = [self.ids] if self.ids is not None else []
        extra_out = [self.ids2] if self.ids is not None else []
        stream_step(self.tree, self.scheme, self.x, self.v, dt, boundary, flops, self.start, self.x2, self.v2,
                    self.start2, self.scratch, extra_in, extra_out, stats=stats)
        self._swap()

    def leaf_counts(self):
        """Particles per leaf (host int64 array): the PIT bin offsets, or the
        counting kernel for PIDT."""
        import torch
        if self.scheme == PIT:
            return np.diff(self.start.cpu().numpy())
        c = torch.empty(self.tree.n_leaves, dtype=torch.int64, device=self.x.device)
        leaf_counts(self.tree, self.x, c)
        return c.cpu().numpy()

    def vmax(self, dt: float):
        """raPIDT's per-cell v_max and predicate for this set (see vmax)."""
        return vmax(self.tree, self.scheme, self.x, self.v, self.start, dt, self.scratch)

    def adapt(self, ppc: int, max_level: int) -> bool:
        """One adaptation; on a change the particles are re-sorted into the
        new tree (stable: old order within each new bin).  Returns whether
        the tree changed."""
        import torch
        spec = adapt(self.tree, self.leaf_counts(), ppc, max_level)
        if spec is None:
            return False
        tree = Tree(spec).upload(self.device)
        nb = tree.n_bins(self.scheme)
        dev = self.x.device
        self.tree = tree
        self.start = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        self.start2 = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        self.scratch = torch.empty(scratch_bytes(tree, self.n, self.scheme) // 8 + 1, dtype=torch.int64, device=dev)
        self.rho = torch.zeros(tree.n_vertices, dtype=torch.float64, device=dev)
        self.initial_sort()
        return True


class Stepper32:
    """Device state of one particle set in the FP32 offset form.

    ``off`` (dim, n) float32 offsets inside the finest cell, ``u`` (dim, n)
    float32 velocities in finest cells per step; the cell is implicit in the
    bin.  Built from an FP64 set (any order) for a step ``dt`` (or per
    instance ``dt_dev``), sorted once, then stepped with the three calls or
    the single fused call.  Trees whose instances are all regular only.
    """

    def __init__(self, tree: Tree, scheme: int, x, v, dt: float = 0.0, q=None, ids=None, inst_start=None,
                 dt_dev=None, device="cuda"):
        import torch
        self.tree, self.scheme = tree, scheme
        self.n = int(x.shape[1])
        self.dt, self.dt_dev = float(dt), dt_dev
        dev = torch.device(device)
        d = tree.dim
        self.off = torch.empty((d, self.n), dtype=torch.float32, device=dev)
        self.u = torch.empty_like(self.off)
        self.off2 = torch.empty_like(self.off)
        self.u2 = torch.empty_like(self.off)
        self.q = _to_dev(q, torch.float64, dev)
        self.ids = _to_dev(ids, None, dev)
        self.q2 = None if self.q is None else torch.empty_like(self.q)
        self.ids2 = None if self.ids is None else torch.empty_like(self.ids)
        self.bin = torch.empty(self.n, dtype=torch.int32, device=dev)
        nb = tree.n_bins(scheme)
        self.start = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        self.start2 = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        sb = scratch_bytes(tree, self.n, scheme, F32_OFFSET)
        _need(sb > 0, "the FP32 form needs a tree whose instances are all regular (with Peano tables)")
        self.scratch = torch.empty(sb // 8 + 1, dtype=torch.int64, device=dev)
        self.rho = torch.zeros(tree.n_vertices, dtype=torch.float64, device=dev)
        self.inst_start = inst_start
        _check_inst(tree, inst_start)
        xd = _to_dev(x, torch.float64, dev)
        vd = _to_dev(v, torch.float64, dev)
        self._convert(F32_OFFSET, xd, vd, None)
        self._rebin(None)

    def _pp(self, qmdt_dev=None, dt_dev=None):
        return _capi.PushParams(_ptr(qmdt_dev), _ptr(dt_dev if dt_dev is not None else self.dt_dev))

    def _convert(self, to, xd, vd, bin_start):
        P = _particles(self.n, x=xd, v=vd, off=self.off, u=self.u, inst_start=self.inst_start)
        pp = self._pp()
        check(lib().pic_convert(self.tree.handle, self.scheme, to, C.byref(P), self.dt, C.byref(pp),
                                C.c_void_p(_ptr(bin_start)) if bin_start is not None else None,
                                C.c_void_p(_ptr(self.bin)), C.c_void_p(_stream(None))), "pic_convert")

    def _cols(self):
        d = self.tree.dim
        ins = [self.off[k] for k in range(d)] + [self.u[k] for k in range(d)]
        outs = [self.off2[k] for k in range(d)] + [self.u2[k] for k in range(d)]
        for a, b in ((self.q, self.q2), (self.ids, self.ids2)):
            if a is not None:
                ins.append(a); outs.append(b)
        return ins, outs

    def _swap(self):
        self.off, self.off2 = self.off2, self.off
        self.u, self.u2 = self.u2, self.u
        self.q, self.q2 = self.q2, self.q
        self.ids, self.ids2 = self.ids2, self.ids
        self.start, self.start2 = self.start2, self.start

    def _rebin(self, old_start, stats=None):
        ins, outs = self._cols()
        rebin(self.tree, self.scheme, self.bin, old_start, ins, outs, self.start2, self.scratch, stats=stats)
        self._swap()

    def to_f64(self):
        """(x, v) FP64 device tensors of the current (sorted) set."""
        import torch
        xd = torch.empty((self.tree.dim, self.n), dtype=torch.float64, device=self.off.device)
        vd = torch.empty_like(xd)
        self._convert(F64, xd, vd, self.start)
        return xd, vd

    def step(self, E, qmdt, dt, q_uniform=0.0, qmdt_dev=None, dt_dev=None, stats=None):
        """Three separate calls: gather_push (in place), rebin, deposit."""
        for k in range(self.tree.dim):
            _check_vec(E[k], self.tree.n_vertices, f"E[{k}]")
        P = _particles(self.n, off=self.off, u=self.u, inst_start=self.inst_start)
        Eptr = (C.c_void_p * 3)(*[_ptr(E[k]) if k < self.tree.dim else None for k in range(3)])
        pp = self._pp(qmdt_dev, dt_dev)
        check(lib().pic_gather_push(self.tree.handle, self.scheme, F32_OFFSET, C.byref(P), Eptr, float(qmdt),
                                    float(dt), C.byref(pp), C.c_void_p(_ptr(self.start)),
                                    C.c_void_p(_ptr(self.bin)), None, C.c_void_p(_stream(None))),
              "pic_gather_push")
        self._rebin(self.start, stats)
        self.deposit(q_uniform)

    def deposit(self, q_uniform=0.0):
        P = _particles(self.n, off=self.off, u=self.u, inst_start=self.inst_start)
        check(lib().pic_deposit(self.tree.handle, self.scheme, F32_OFFSET, C.byref(P),
                                C.c_void_p(_ptr(self.start)),
                                C.c_void_p(_ptr(self.q)) if self.q is not None else None, float(q_uniform),
                                C.c_void_p(_ptr(self.rho)), C.c_void_p(_ptr(self.scratch)),
                                self.scratch.numel() * self.scratch.element_size(), C.c_void_p(_stream(None))),
              "pic_deposit")

    def step_fused(self, E, qmdt, dt, q_uniform=0.0, qmdt_dev=None, dt_dev=None, stats=None):
        """The same step through the single call pic_step (FP32 form)."""
        for k in range(self.tree.dim):
            _check_vec(E[k], self.tree.n_vertices, f"E[{k}]")
        P = _particles(self.n, off=self.off, u=self.u, inst_start=self.inst_start)
        Q = _particles(self.n, off=self.off2, u=self.u2, inst_start=self.inst_start)
        Eptr = (C.c_void_p * 3)(*[_ptr(E[k]) if k < self.tree.dim else None for k in range(3)])
        pp = self._pp(qmdt_dev, dt_dev)
        extra_in, extra_out, q_col = [], [], -1
        if self.q is not None:
            q_col = 0
            extra_in.append(self.q); extra_out.append(self.q2)
        if self.ids is not None:
            extra_in.append(self.ids); extra_out.append(self.ids2)
        ne = len(extra_in)
        ins = (C.c_void_p * max(ne, 1))(*[_ptr(c) for c in extra_in])
        outs = (C.c_void_p * max(ne, 1))(*[_ptr(c) for c in extra_out])
        sizes = (C.c_int32 * max(ne, 1))(*[c.element_size() for c in extra_in])
        check(lib().pic_step(self.tree.handle, self.scheme, F32_OFFSET, C.byref(P), C.c_void_p(_ptr(self.start)),
                             Eptr, float(qmdt), float(dt), C.byref(pp), ne, ins, outs, sizes, q_col,
                             float(q_uniform), C.byref(Q), C.c_void_p(_ptr(self.start2)),
                             C.c_void_p(_ptr(self.rho)), C.c_void_p(_ptr(self.scratch)),
                             self.scratch.numel() * self.scratch.element_size(), _stats_ptr(stats),
                             C.c_void_p(_stream(None))),
              "pic_step")
        self._swap()


class StepGraph:
    """Two consecutive steps of a stepper captured in one HIP graph.

    Every launch of a step goes to the current stream and nothing in it
    allocates, synchronises or writes through memset nodes (counters are
    cleared by kernels), so the step sequence can be captured and replayed.
    Two steps are captured so that the double buffers return to their places;
    each replay advances the state by two steps.  The field, the step
    parameters and all buffers are fixed at capture.
    """

    def __init__(self, stepper, E, qmdt, dt, q_uniform=0.0, fused=True, **kw):
        import torch
        self.stepper = stepper
        f = stepper.step_fused if fused else stepper.step
        args = (E, qmdt, dt)
        kw = dict(kw, q_uniform=q_uniform)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):              # warm-up outside the capture
            f(*args, **kw)
            f(*args, **kw)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            f(*args, **kw)
            f(*args, **kw)

    def replay(self):
        self.graph.replay()
