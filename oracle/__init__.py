"""Plain serial FP64 oracle for the spacetree PIC hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product library.  It
shares no code with the GPU path.  The arithmetic lives in ``pic_oracle.c``
(serial C, ``-O2 -ffp-contract=off``); this module marshals numpy arrays and
adds the FP64 support pieces that sit outside the hot path (periodic Poisson
solve and the vertex field), which the physics pins need.

Paper sections followed (see the C file header for the readings):
  Sec. 3   PIC cycle: deposit rho = sum R(x_i), solve, E = -grad V,
           gather E_i = R^T(x_i) E, push.
  Sec. 4   k=3 spacetree, dual grid, Peano ordering of the storage.
  Sec. 5.1 PIT: each particle held by the leaf covering it (Theorem 1).
  Sec. 5.2 PIDT: each particle held by the vertex whose dual cell covers it
           (Theorem 2).
  Sec. 6   the particle-handling benchmark: free streaming with periodic or
           reflecting walls and artificial flops; the ppc-driven dynamic
           refinement and coarsening of the tree.
  Sec. 6.1 lifts per particle and step (re-bin statistics).
  App. A   Langmuir-wave units and the Bohm-Gross relation.
"""
from __future__ import annotations

import ctypes as C
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "_pic_oracle.so")

PIT, PIDT = 0, 1
PERIODIC, REFLECT = 0, 1
STATS_LEVELS = 20   # entries of the lift-count histogram


# A prebuilt library to load instead (the sanitized build of the CPU test run).
_LIB_OVERRIDE = os.environ.get("PIC_ORACLE_LIB")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out: str) -> str:
    """Compile the oracle with clang under AddressSanitizer and
    UndefinedBehaviorSanitizer (same arithmetic flags), for a process that
    preloads clang's ASan runtime."""
    clang = os.environ.get("CLANG", "/opt/rocm/llvm/bin/clang")
    subprocess.check_call([clang, "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                           "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-shared-libsan", "-fPIC", "-shared", "-o", out, _SRC,
                           "-lm"])
    return out


_lib = None


def load(path: str):
    """Load a compiled oracle library and declare its signatures."""
    L = C.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load(_LIB_OVERRIDE or _LIB)
    return _lib


def _declare(L):
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
    L.orc_tree_new.restype = vp
    L.orc_tree_new.argtypes = [i32, i32, vp]
    L.orc_tree_free.argtypes = [vp]
    L.orc_tree_sizes.argtypes = [vp, vp]
    L.orc_tree_leaves.argtypes = [vp, vp, vp, vp, vp, vp]
    L.orc_tree_vertices.argtypes = [vp, vp]
    L.orc_tree_pidt.argtypes = [vp, vp, vp, vp, vp]
    L.orc_peano.restype = C.c_uint64
    L.orc_peano.argtypes = [i32, i32, vp]
    L.orc_locate.restype = i32
    L.orc_locate.argtypes = [vp, i64, vp, vp, vp, vp]
    L.orc_weights.restype = i32
    L.orc_weights.argtypes = [vp, i64, vp, vp, vp]
    L.orc_gather_push.restype = i32
    L.orc_gather_push.argtypes = [vp, i64, vp, vp, vp, dbl, dbl, vp, vp, i32]
    L.orc_free_stream.restype = i32
    L.orc_free_stream.argtypes = [vp, i64, vp, vp, dbl, i32, i32, vp, i32]
    L.orc_rebin.restype = i32
    L.orc_rebin.argtypes = [i64, i64, vp, vp, vp, vp]
    L.orc_deposit.restype = i32
    L.orc_deposit.argtypes = [vp, i64, vp, vp, dbl, vp]
    L.orc_rebin_stats.restype = i32
    L.orc_rebin_stats.argtypes = [vp, i32, i64, vp, vp, i32, vp]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def peano(dim: int, level: int, coords) -> int:
    """Peano index of the level-``level`` cell with integer ``coords``."""
    c = np.zeros(3, np.int64)
    c[:dim] = coords
    return int(lib().orc_peano(dim, level, _p(c)))


class OracleTree:
    """The oracle's own spacetree, rebuilt from the refine masks."""

    def __init__(self, spec):
        self.spec = spec
        self.dim = spec.dim
        self.L = spec.max_level
        masks = spec.masks_concat()
        if masks.size == 0:
            masks = np.zeros(1, np.uint8)
        self._masks = masks
        self._L = lib()
        self._h = self._L.orc_tree_new(self.dim, self.L, _p(masks))
        if not self._h:
            raise ValueError("oracle: unsupported tree")
        s = np.zeros(8, np.int64)
        self._L.orc_tree_sizes(self._h, _p(s))
        self.n_nodes, self.n_leaves, self.n_vertices, self.n_pidt, self.S = (int(v) for v in s[:5])
        self.n_corners = 1 << self.dim

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_tree_free(h)
            self._h = None

    def n_bins(self, scheme: int) -> int:
        return self.n_leaves if scheme == PIT else self.n_pidt

    def leaves(self):
        nl, d, nc = self.n_leaves, self.dim, self.n_corners
        key = np.zeros(nl, np.uint64)
        level = np.zeros(nl, np.int32)
        coord = np.zeros((nl, d), np.int64)
        vtx = np.zeros((nl, nc), np.int32)
        pidt = np.zeros((nl, nc), np.int32)
        self._L.orc_tree_leaves(self._h, _p(key), _p(level), _p(coord), _p(vtx), _p(pidt))
        return {"key": key, "level": level, "coord": coord, "vtx": vtx, "pidt": pidt}

    def vertex_positions(self) -> np.ndarray:
        """(n_vertices, dim) int64 positions in finest-cell units (periodic)."""
        pos = np.zeros((self.n_vertices, self.dim), np.int64)
        self._L.orc_tree_vertices(self._h, _p(pos))
        return pos

    def vertex_positions_unit(self) -> np.ndarray:
        """(dim, n_vertices) float64 positions in domain units."""
        return self.vertex_positions().T.astype(np.float64) / self.S

    def pidt_bins(self):
        n, d = self.n_pidt, self.dim
        key = np.zeros(n, np.uint64)
        level = np.zeros(n, np.int32)
        b = np.zeros((n, d), np.int64)
        vid = np.zeros(n, np.int32)
        self._L.orc_tree_pidt(self._h, _p(key), _p(level), _p(b), _p(vid))
        return {"key": key, "level": level, "b": b, "vid": vid}

    # -- per-particle operations; x, v are (dim, n) float64 --------------------
    def locate(self, x):
        x = np.ascontiguousarray(x, np.float64)
        n = x.shape[1]
        leaf = np.zeros(n, np.int32)
        pidt = np.zeros(n, np.int32)
        cell = np.zeros((n, self.dim), np.int64)
        if self._L.orc_locate(self._h, n, _p(x), _p(leaf), _p(pidt), _p(cell)):
            raise ValueError("oracle: position outside [0,1)")
        return leaf, pidt, cell

    def weights(self, x):
        x = np.ascontiguousarray(x, np.float64)
        n = x.shape[1]
        w = np.zeros((n, self.n_corners))
        vtx = np.zeros((n, self.n_corners), np.int32)
        if self._L.orc_weights(self._h, n, _p(x), _p(w), _p(vtx)):
            raise ValueError("oracle: position outside [0,1)")
        return w, vtx

    def gather_push(self, x, v, E, qmdt, dt, scheme=PIT):
        """One leapfrog step; returns (x', v', E_p, new_bin) without touching inputs."""
        x = np.array(x, np.float64, order="C", copy=True)
        v = np.array(v, np.float64, order="C", copy=True)
        E = np.ascontiguousarray(E, np.float64)
        assert E.shape == (self.dim, self.n_vertices)
        n = x.shape[1]
        ep = np.zeros((self.dim, n))
        bins = np.zeros(n, np.int32)
        if self._L.orc_gather_push(self._h, n, _p(x), _p(v), _p(E), float(qmdt), float(dt),
                                 _p(ep), _p(bins), int(scheme)):
            raise ValueError("oracle: position outside [0,1)")
        return x, v, ep, bins

    def free_stream(self, x, v, dt, boundary=REFLECT, flops=0, scheme=PIT):
        """One free-streaming move (no field): returns (x', v', new_bin)
        without touching the inputs."""
        x = np.array(x, np.float64, order="C", copy=True)
        v = np.array(v, np.float64, order="C", copy=True)
        n = x.shape[1]
        bins = np.zeros(n, np.int32)
        if self._L.orc_free_stream(self._h, n, _p(x), _p(v), float(dt), int(boundary), int(flops), _p(bins),
                                   int(scheme)):
            raise ValueError("oracle: position outside [0,1) or a move longer than the box")
        return x, v, bins

    def deposit(self, x, q=None, q_uniform=0.0):
        x = np.ascontiguousarray(x, np.float64)
        n = x.shape[1]
        rho = np.zeros(self.n_vertices)
        qa = None if q is None else np.ascontiguousarray(q, np.float64)
        if self._L.orc_deposit(self._h, n, _p(x), _p(qa), float(q_uniform), _p(rho)):
            raise ValueError("oracle: position outside [0,1)")
        return rho

    def bin_of(self, x, scheme):
        leaf, pidt, _ = self.locate(x)
        return leaf if scheme == PIT else pidt

    def rebin_stats(self, old_start, new_bin, scheme, n_hist: int = STATS_LEVELS):
        """Re-bin statistics of a sorted set (offsets ``old_start``) moving to
        ``new_bin`` (paper Sec. 6.1, lifts per particle): dict of particles,
        movers, lifts, max_tunnel and lift_hist."""
        os_ = np.ascontiguousarray(old_start, np.int64)
        nb = np.ascontiguousarray(new_bin, np.int32)
        out = np.zeros(4 + n_hist, np.int64)
        if self._L.orc_rebin_stats(self._h, int(scheme), nb.size, _p(os_), _p(nb), n_hist, _p(out)):
            raise ValueError("oracle: bad offsets or bins")
        return {"particles": int(out[0]), "movers": int(out[1]), "lifts": int(out[2]), "max_tunnel": int(out[3]),
                "lift_hist": [int(v) for v in out[4:]]}


def rebin(new_bin, n_bins: int, old_start=None):
    """Stable re-bin: returns (perm, new_start) with out[j] = in[perm[j]]."""
    nb = np.ascontiguousarray(new_bin, np.int32)
    n = nb.size
    perm = np.zeros(n, np.int64)
    start = np.zeros(n_bins + 1, np.int64)
    os_ = None if old_start is None else np.ascontiguousarray(old_start, np.int64)
    if lib().orc_rebin(n, n_bins, _p(nb), _p(os_), _p(perm), _p(start)):
        raise ValueError("oracle: bad bins")
    return perm, start


def initial_sort(tree: OracleTree, x, v, q=None, scheme=PIT):
    """Bin an unsorted particle set: returns (x, v, q, bin_start, perm)."""
    nb = tree.bin_of(x, scheme)
    perm, start = rebin(nb, tree.n_bins(scheme), None)
    return x[:, perm], v[:, perm], (None if q is None else q[perm]), start, perm


def step(tree: OracleTree, x, v, E, qmdt, dt, bin_start, scheme=PIT, q=None, q_uniform=0.0):
    """One hot-path step: gather + push, re-bin, deposit.

    Returns dict(x, v, q, bin_start, perm, Ep, new_bin, rho).
    """
    x1, v1, ep, nb = tree.gather_push(x, v, E, qmdt, dt, scheme)
    perm, start = rebin(nb, tree.n_bins(scheme), bin_start)
    x2, v2 = x1[:, perm], v1[:, perm]
    q2 = None if q is None else q[perm]
    rho = tree.deposit(x2, q2, q_uniform)
    return {"x": x2, "v": v2, "q": q2, "bin_start": start, "perm": perm, "Ep": ep,
            "new_bin": nb, "rho": rho}


# ---------------------------------------------------------------------------
# Support outside the hot path (regular periodic trees only): Poisson + field
# ---------------------------------------------------------------------------
# raPIDT's analysed attribute (paper Sec. 5.4, Eq. (vmax))
# ---------------------------------------------------------------------------

def vmax_cells(spec, x, v, scheme, dt=None):
    """The per-cell maximum velocity component of raPIDT, from its
    definition: for a leaf, the largest |v_k| over the particles it holds
    (PIT) or over the particles of the 2^d dual cells of its corners at its
    level (PIDT); for a refined cell, the largest value of its children,
    i.e. of every leaf below it.  Returned as one float64 array per level in
    the layout of the refine masks (lexicographic, 0 for cells that do not
    exist); with ``dt`` also the predicate v_max(c) dt <= h(c) per cell
    (uint8, 0 for cells that do not exist)."""
    d, L = spec.dim, spec.max_level
    t = OracleTree(spec)
    speed = np.max(np.abs(np.asarray(v, np.float64)), axis=0) if np.asarray(v).size else np.zeros(0)
    leaf, pidt, _ = t.locate(x) if speed.size else (np.zeros(0, np.int32),) * 3
    lv = t.leaves()
    per_leaf = np.zeros(t.n_leaves)
    if scheme == PIT:
        np.maximum.at(per_leaf, leaf, speed)
    else:
        per_bin = np.zeros(t.n_pidt)
        np.maximum.at(per_bin, pidt, speed)
        per_leaf = per_bin[lv["pidt"]].max(axis=1)
    out = [np.zeros((3 ** l) ** d) for l in range(L + 1)]
    exists = [np.zeros((3 ** l) ** d, bool) for l in range(L + 1)]
    for r in range(t.n_leaves):
        l, a = int(lv["level"][r]), [int(c) for c in lv["coord"][r]]
        for up in range(l, -1, -1):          # the leaf and every ancestor
            n = 3 ** up
            i = sum(a[k] * n ** k for k in range(d))
            out[up][i] = max(out[up][i], per_leaf[r])
            exists[up][i] = True
            a = [c // 3 for c in a]
    if dt is None:
        return out
    quiet = [(exists[l] & (out[l] * dt <= 1.0 / 3 ** l)).astype(np.uint8) for l in range(L + 1)]
    return out, quiet


# ---------------------------------------------------------------------------
# ppc-driven dynamic adaptivity (paper Sec. 6 setup; Sec. 5 opening remark)
# ---------------------------------------------------------------------------

def _cells_of(spec):
    """Existing cells per level: a set of integer coordinate tuples, and of
    those the refined ones, read from the masks (lexicographic, axis 0
    fastest)."""
    d = spec.dim
    exist = [{(0,) * d}]
    refined = []
    for l in range(spec.max_level):
        n = 3 ** l
        m = np.asarray(spec.refine[l]).ravel()
        ref = {a for a in exist[l] if m[sum(a[k] * n ** k for k in range(d))]}
        refined.append(ref)
        nxt = set()
        for a in ref:
            for c in itertools.product(range(3), repeat=d):
                nxt.add(tuple(3 * a[k] + c[k] for k in range(d)))
        exist.append(nxt)
    refined.append(set())
    return exist, refined


def adapt(spec, x, ppc: int, max_level: int):
    """One adaptation of the tree to the particles ``x`` (dim, n): a leaf
    holding more than ``ppc`` particles is refined (below ``max_level``); a
    refined cell other than the root whose children are all leaves holding
    together at most ``ppc`` particles loses its children.  Returns the new
    spec; refine masks are 0 for every cell that does not exist."""
    import workloads as W
    d, L, S = spec.dim, spec.max_level, 3 ** spec.max_level
    exist, refined = _cells_of(spec)
    # particles per leaf, by the leaf box holding the finest cell of fl(x S)
    I = np.minimum(np.floor(np.asarray(x, np.float64) * S), S - 1).astype(np.int64)
    count = {}
    for l in range(L + 1):
        leaves = exist[l] - refined[l]
        if not leaves:
            continue
        s = 3 ** (L - l)
        a = I // s
        for p in range(I.shape[1]):
            key = tuple(int(a[k, p]) for k in range(d))
            if key in leaves:
                count[(l, key)] = count.get((l, key), 0) + 1
    new_ref = [set(r) for r in refined]
    for l in range(L + 1):
        for a in exist[l] - refined[l]:
            if l < max_level and count.get((l, a), 0) > ppc:
                while len(new_ref) <= l:
                    new_ref.append(set())
                new_ref[l].add(a)
    for l in range(1, L):
        for a in refined[l]:
            kids = [tuple(3 * a[k] + c[k] for k in range(d)) for c in itertools.product(range(3), repeat=d)]
            if any(kk in refined[l + 1] for kk in kids):
                continue
            if sum(count.get((l + 1, kk), 0) for kk in kids) <= ppc:
                new_ref[l].discard(a)
    # the new tree: cells reached from the root through refined cells
    levels = []
    live = {(0,) * d}
    l = 0
    while l < len(new_ref):
        ref = {a for a in live if a in new_ref[l]}
        if not ref:
            break
        n = 3 ** l
        m = np.zeros(n ** d, np.uint8)
        for a in ref:
            m[sum(a[k] * n ** k for k in range(d))] = 1
        levels.append(m)
        live = {tuple(3 * a[k] + c[k] for k in range(d)) for a in ref for c in itertools.product(range(3), repeat=d)}
        l += 1
    return W.TreeSpec(d, len(levels), levels)


# ---------------------------------------------------------------------------

def _grid(a, dim, n):
    """Vertex array (lexicographic, axis 0 fastest) -> numpy grid indexed [axis d-1, ..., axis 0]."""
    return a.reshape((n,) * dim)


def poisson_periodic(rho_charge, dim: int, level: int, background: float = 1.0):
    """Solve -Lap_h V = rho_charge/h^d + background on the periodic vertex grid.

    The (2d+1)-point Laplacian is diagonalised by the DFT, whose eigenvalues
    are sum_k (2 - 2 cos(2 pi m_k / n)) / h^2.  The mean of V is fixed to 0.
    ``rho_charge`` is vertex charge (what the deposit returns); dividing by the
    dual-cell volume h^d gives the density.
    """
    n = 3 ** level
    h = 1.0 / n
    dens = _grid(np.asarray(rho_charge, np.float64), dim, n) / h ** dim + background
    f = np.fft.fftn(dens)
    lam = np.zeros((n,) * dim)
    m = np.arange(n)
    eig = (2.0 - 2.0 * np.cos(2.0 * np.pi * m / n)) / (h * h)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = n
        lam = lam + eig.reshape(shape)
    lam.flat[0] = 1.0
    vh = f / lam
    vh.flat[0] = 0.0
    return np.real(np.fft.ifftn(vh)).ravel()


def field_from_potential(V, dim: int, level: int):
    """E = -grad V by central differences on the periodic vertex grid; (dim, n^d)."""
    n = 3 ** level
    h = 1.0 / n
    g = _grid(np.asarray(V, np.float64), dim, n)
    E = np.zeros((dim, n ** dim))
    for k in range(dim):
        ax = dim - 1 - k                 # axis k of the domain is numpy axis d-1-k
        E[k] = (-(np.roll(g, -1, axis=ax) - np.roll(g, 1, axis=ax)) / (2.0 * h)).ravel()
    return E


def langmuir_run(tree: OracleTree, x, v, qmdt, dt, steps, q_uniform, record=None):
    """Free-running PIC (deposit, Poisson, field, gather, push) on a regular periodic tree.

    The leapfrog starts from v^{-1/2} = v^0 - (qmdt/2) E(x^0).  ``record(step,
    rho, V, E, x, v)`` is called after each field solve.  Returns (x, v).
    """
    assert tree.n_vertices == tree.S ** tree.dim, "regular trees only"
    x = np.array(x, np.float64, copy=True)
    v = np.array(v, np.float64, copy=True)
    for it in range(steps + 1):
        rho = tree.deposit(x, None, q_uniform)
        V = poisson_periodic(rho, tree.dim, tree.L)
        E = field_from_potential(V, tree.dim, tree.L)
        if record is not None:
            record(it, rho, V, E, x, v)
        if it == steps:
            break
        if it == 0:
            # half kick back in time: a zero-length step with qmdt -> -qmdt/2
            _, v, _, _ = tree.gather_push(x, v, E, -0.5 * qmdt, 0.0, PIT)
        x, v, _, _ = tree.gather_push(x, v, E, qmdt, dt, PIT)
    return x, v
