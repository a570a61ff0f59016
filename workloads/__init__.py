"""Seeded synthetic inputs for the spacetree particle-in-cell hot path.

This module is shared by the oracle tests, the GPU tests and the benchmark.
It holds only *inputs*: the refinement geometry of a spacetree (which cells
are refined), particle positions, velocities and charges drawn from seeded
generators, and fields evaluated at given vertex positions.  It computes none
of the method's arithmetic: no cell location, no space-filling-curve order, no
shape-function weights, no binning and no deposit.  Particles come out in
generation order (unsorted); each consumer bins them itself.

Units (the paper's validation appendix, App. A): the plasma frequency is 1,
the electron charge density is -1 (so every macro-particle has charge -1/N in
a unit box with N particles and q/m = -1) and a neutralising ion background of
density +1 sits outside the particle set.  A workload fixes a reference cell
width h and a Debye length lambda_D = h, so v_th = h and a time step of
dt = sigma (in cells per step) gives a thermal displacement of sigma cells.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

__all__ = [
    "TreeSpec", "Workload", "regular_tree", "disc_tree", "leaf_cells",
    "config1", "config2", "config3", "config4", "config5", "small_adaptive",
    "small_3d", "small_3d_adaptive", "random_field", "langmuir_field",
    "cosine_potential_field", "CONFIG_NAMES", "by_name",
]


# ---------------------------------------------------------------------------
# Tree geometry: refine masks per level
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class TreeSpec:
    """Refinement description of a 3^d spacetree on the periodic unit box.

    ``refine[l]`` (l = 0 .. max_level-1) is a uint8 array with (3**l)**dim
    entries in lexicographic order (axis 0 fastest): 1 means the level-l cell
    with those integer coordinates is refined.  Entries of cells whose parent
    is not refined are ignored.  Cells at ``max_level`` are never refined.
    """
    dim: int
    max_level: int
    refine: List[np.ndarray]

    def masks_concat(self) -> np.ndarray:
        """All levels' masks back to back (level 0 first), as one uint8 array."""
        if self.max_level == 0:
            return np.zeros(0, np.uint8)
        return np.ascontiguousarray(
            np.concatenate([np.asarray(m, np.uint8).ravel() for m in self.refine]))

    @property
    def finest(self) -> int:
        return 3 ** self.max_level


def regular_tree(dim: int, level: int) -> TreeSpec:
    """Every cell above ``level`` refined: a regular (3^level)^dim grid."""
    return TreeSpec(dim, level, [np.ones((3 ** l) ** dim, np.uint8) for l in range(level)])


def _cell_meets_ball(dim: int, level: int, centre: Sequence[tuple], radius: tuple) -> np.ndarray:
    """Exact integer test: does the closed level-``level`` cell meet the closed ball?

    ``centre`` is a tuple of (num, den) per axis and ``radius`` is (num, den).
    Cell i spans [i/3^l, (i+1)/3^l] per axis.  All quantities are scaled to a
    common integer denominator so the comparison is exact.
    """
    n = 3 ** level
    den = radius[1]
    for c in centre:
        den = den * c[1] // math.gcd(den, c[1])
    scale = den * n                       # coordinates multiplied by this are integers
    r = radius[0] * (scale // radius[1])
    idx = np.arange(n, dtype=np.int64)
    lo = idx * den
    hi = (idx + 1) * den
    d2 = np.zeros((n,) * dim, np.int64)
    for k in range(dim):
        ck = centre[k][0] * (scale // centre[k][1])
        dk = np.maximum(np.maximum(lo - ck, 0), ck - hi)
        shape = [1] * dim
        shape[dim - 1 - k] = n            # axis 0 fastest => last numpy axis
        d2 = d2 + (dk * dk).reshape(shape)
    return (d2 <= r * r).ravel()


def disc_tree(dim: int = 2, base: int = 4, max_level: int = 6,
              centre: Optional[Sequence[tuple]] = None,
              radius: tuple = (1, 5)) -> TreeSpec:
    """Regular to ``base``; below, a cell is refined iff it meets the closed ball.

    Default: the 2D disc of radius 1/5 around (1/2, 1/2), refined from level
    4 to level 6.
    """
    if centre is None:
        centre = [(1, 2)] * dim
    masks = []
    for l in range(max_level):
        if l < base:
            masks.append(np.ones((3 ** l) ** dim, np.uint8))
        else:
            masks.append(_cell_meets_ball(dim, l, centre, radius).astype(np.uint8))
    return TreeSpec(dim, max_level, masks)


def _upsample(mask: np.ndarray, dim: int, level: int) -> np.ndarray:
    """Level-l cell flags -> flags of their 3^d children at level l+1."""
    n = 3 ** level
    a = mask.reshape((n,) * dim)
    for ax in range(dim):
        a = np.repeat(a, 3, axis=ax)
    return a.ravel()


def leaf_cells(spec: TreeSpec):
    """Geometric leaf list: for each level, the lexicographic ids of its leaves.

    Returns a list ``out[l]`` of int64 arrays of lexicographic cell indices at
    level l.  This is plain geometry (which cells exist and are unrefined); it
    implies no order of the leaves along any curve.
    """
    d = spec.dim
    exists = np.ones(1, bool)
    out = []
    for l in range(spec.max_level + 1):
        if l < spec.max_level:
            ref = spec.refine[l].astype(bool) & exists
            out.append(np.nonzero(exists & ~ref)[0])
            exists = _upsample(ref, d, l)
        else:
            out.append(np.nonzero(exists)[0])
    return out


def _lex_to_coords(idx: np.ndarray, dim: int, n: int) -> np.ndarray:
    c = np.empty((dim, idx.size), np.int64)
    r = idx.copy()
    for k in range(dim):
        c[k] = r % n
        r //= n
    return c


# ---------------------------------------------------------------------------
# Particle draws
# ---------------------------------------------------------------------------

def _perturbed_axis0(rng: np.random.Generator, n: int, eps: float, modes: Sequence[int]) -> np.ndarray:
    """Exact rejection sampling of x in [0,1) with density 1 + eps*sum_k cos(2 pi k x)."""
    bound = 1.0 + abs(eps) * len(modes)
    out = np.empty(n)
    filled = 0
    while filled < n:
        m = int((n - filled) * bound * 1.05) + 64
        x = rng.random(m)
        dens = np.ones(m)
        for k in modes:
            dens += eps * np.cos(2.0 * np.pi * k * x)
        keep = x[rng.random(m) * bound < dens]
        take = min(keep.size, n - filled)
        out[filled:filled + take] = keep[:take]
        filled += take
    return out


def _positions(rng, n, dim, eps, modes):
    x = np.empty((dim, n))
    x[0] = _perturbed_axis0(rng, n, eps, modes) if eps else rng.random(n)
    for k in range(1, dim):
        x[k] = rng.random(n)
    return x


def _isotropic(rng, n, dim):
    g = rng.standard_normal((dim, n))
    g /= np.linalg.norm(g, axis=0, keepdims=True)
    return g


# ---------------------------------------------------------------------------
# Fields at vertex positions
# ---------------------------------------------------------------------------

def random_field(rng: np.random.Generator, dim: int, n_vertices: int, scale: float = 1.0) -> np.ndarray:
    """Independent normal field values per vertex id, shape (dim, n_vertices)."""
    return scale * rng.standard_normal((dim, n_vertices))


def langmuir_field(pos: np.ndarray, eps: float, modes: Sequence[int]) -> np.ndarray:
    """Linear-theory field of the density 1 + eps*sum cos(2 pi k x0) over a +1 background.

    Gauss's law div E = rho with rho = -eps*sum cos(2 pi k x0) gives
    E0 = -sum eps/(2 pi k) sin(2 pi k x0); other components vanish.
    ``pos`` has shape (dim, nv) in domain units.
    """
    e = np.zeros(pos.shape)
    for k in modes:
        e[0] -= eps / (2.0 * np.pi * k) * np.sin(2.0 * np.pi * k * pos[0])
    return e


def cosine_potential_field(pos: np.ndarray, phi0: float) -> np.ndarray:
    """E = -grad V for V = phi0 * sum_k cos(2 pi x_k)."""
    return np.ascontiguousarray(2.0 * np.pi * phi0 * np.sin(2.0 * np.pi * pos))


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """One synthetic instance: tree, particles and push parameters.

    ``x``, ``v``: float64 arrays of shape (dim, N) in domain units (x in [0,1)).
    ``q``: per-particle charge (N,) or None, in which case every particle
    carries ``q_uniform``.  ``qm`` is the charge-to-mass ratio and ``dt`` the
    time step; the push uses qm*dt and dt.  ``field(pos)`` evaluates the
    prescribed field at vertex positions (dim, nv) in domain units.
    """
    name: str
    tree: TreeSpec
    x: np.ndarray
    v: np.ndarray
    q: Optional[np.ndarray]
    q_uniform: float
    qm: float
    dt: float
    steps: int
    field: Callable[[np.ndarray], np.ndarray]
    h: float
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[1]

    @property
    def dim(self) -> int:
        return self.tree.dim


def _langmuir_instance(name, tree, rng, ppc_total, sigma_cells, eps, modes, steps,
                       beam_frac=0.0, beam_range=None, tunnel_frac=0.0, tunnel_max=0.0):
    """Uniform plasma with a density perturbation; lambda_D = h (finest width)."""
    d = tree.dim
    h = 1.0 / tree.finest
    n = ppc_total
    dt = float(sigma_cells)
    vscale = h / dt                       # one cell per step in domain units per time
    x = _positions(rng, n, d, eps, modes)
    v = rng.standard_normal((d, n)) * (sigma_cells * vscale)
    meta = {"sigma_cells": sigma_cells, "eps": eps, "modes": list(modes)}
    if beam_frac:
        nb = int(round(beam_frac * n))
        sel = rng.choice(n, nb, replace=False)
        v[0, sel] = rng.uniform(beam_range[0], beam_range[1], nb) * vscale
        for k in range(1, d):
            v[k, sel] = rng.standard_normal(nb) * vscale
        meta["beam"] = nb
    if tunnel_frac:
        nt = int(round(tunnel_frac * n))
        sel = rng.choice(n, nt, replace=False)
        speed = rng.uniform(1.0, tunnel_max, nt) * vscale
        v[:, sel] = _isotropic(rng, nt, d) * speed
        meta["tunnelers"] = nt
    return Workload(name, tree, x, v, None, -1.0 / n, -1.0, dt, steps,
                    lambda pos: langmuir_field(pos, eps, modes), h, meta)


def config1(seed: int = 0) -> Workload:
    """2D periodic regular depth 3 (27x27), 64 electrons/cell, v_th 0.5 cell/step."""
    rng = np.random.default_rng(seed)
    tree = regular_tree(2, 3)
    return _langmuir_instance("config1_2d_L3_pit", tree, rng, 64 * 27 * 27, 0.5, 0.01, [1], 20)


def config2(seed: int = 0, ppc: int = 256) -> Workload:
    """2D periodic regular depth 5 (243x243), 256/cell, v_th 1 + 1% beam at 8-20 cells/step."""
    rng = np.random.default_rng(seed)
    tree = regular_tree(2, 5)
    return _langmuir_instance("config2_2d_L5", tree, rng, ppc * 243 * 243, 1.0, 0.01,
                              [1, 2, 3, 4], 50, beam_frac=0.01, beam_range=(8.0, 20.0))


def config3(seed: int = 0, per_leaf: int = 128) -> Workload:
    """2D adaptive: depth 4 base, refined to depth 6 inside the disc r=1/5 around the centre.

    ``per_leaf`` particles are drawn uniformly inside every leaf; each carries a
    charge proportional to the leaf volume times a 20% Gaussian bump
    (centre (1/2,1/2), width 0.1) so that the charge density follows the bump.
    The velocity spread is one coarse (level-4) cell per step and the field is
    the prescribed cosine potential.
    """
    rng = np.random.default_rng(seed)
    tree = disc_tree(2, 4, 6)
    return _leafwise_instance("config3_2d_adaptive", tree, rng, per_leaf, base_level=4,
                              sigma_cells=1.0, steps=50)


def _leafwise_instance(name, tree, rng, per_leaf, base_level, sigma_cells, steps):
    d = tree.dim
    leaves = leaf_cells(tree)
    xs, qs = [], []
    for l, ids in enumerate(leaves):
        if ids.size == 0:
            continue
        n_l = 3 ** l
        a = _lex_to_coords(ids, d, n_l)
        a = np.repeat(a, per_leaf, axis=1)
        pos = (a + rng.random(a.shape)) / n_l
        pos[pos >= 1.0] = 0.0
        xs.append(pos)
        vol = float(n_l) ** (-d)
        qs.append(np.full(pos.shape[1], vol / per_leaf))
    x = np.concatenate(xs, axis=1)
    qv = np.concatenate(qs)
    g = np.exp(-np.sum((x - 0.5) ** 2, axis=0) / (2 * 0.1 ** 2))
    q = -(1.0 + 0.2 * g) * qv
    h = 1.0 / 3 ** base_level
    dt = float(sigma_cells)
    vth = h / dt * sigma_cells
    v = rng.standard_normal(x.shape) * vth
    phi0 = 0.05 * vth / (2.0 * np.pi * dt)
    return Workload(name, tree, x, v, q, 0.0, -1.0, dt, steps,
                    lambda pos: cosine_potential_field(pos, phi0), h,
                    {"sigma_coarse_cells": sigma_cells, "per_leaf": per_leaf})


def config4(seed: int = 0, ppc: int = 64) -> Workload:
    """3D periodic regular depth 4 (81^3), 64/cell, v_th 1 cell/step, 5% tunnelers to 10 cells/step."""
    rng = np.random.default_rng(seed)
    tree = regular_tree(3, 4)
    return _langmuir_instance("config4_3d_L4", tree, rng, ppc * 81 ** 3, 1.0, 0.01, [1], 50,
                              tunnel_frac=0.05, tunnel_max=10.0)


def config5(seed: int = 0, n_inst: int = 64, n_min: float = 1e5, n_max: float = 4e6,
            scale: float = 1.0) -> List[Workload]:
    """64 independent 2D Langmuir instances of mixed depth (3-5) and size.

    Instance i draws from ``SeedSequence(seed).spawn(n_inst)[i]``: depth
    uniform in {3,4,5}, particle count log-uniform in [n_min, n_max] (times
    ``scale``), v_th in [0.5, 2] cells/step and k*lambda_D in [0.1, 0.6] for
    the k = 2*pi mode.  Since lambda_D = v_th (plasma frequency 1), the time
    step is dt = sigma*h/lambda_D; draws with dt > 1 are redrawn from the same
    stream so that the leapfrog stays well inside its stability limit.
    """
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(n_inst)):
        rng = np.random.default_rng(ss)
        while True:
            level = int(rng.integers(3, 6))
            n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) * scale))
            sigma = float(rng.uniform(0.5, 2.0))
            klam = float(rng.uniform(0.1, 0.6))
            h = 3.0 ** (-level)
            lam = klam / (2.0 * math.pi)
            dt = sigma * h / lam
            if dt <= 1.0:
                break
        n = max(n, 1)
        tree = regular_tree(2, level)
        eps = 0.01
        x = _positions(rng, n, 2, eps, [1])
        v = rng.standard_normal((2, n)) * lam
        out.append(Workload(f"config5_inst{i:02d}", tree, x, v, None, -1.0 / n, -1.0, dt, 50,
                            lambda pos, eps=eps: langmuir_field(pos, eps, [1]), h,
                            {"sigma_cells": sigma, "k_lambda_D": klam, "level": level}))
    return out


def small_adaptive(seed: int = 0, per_leaf: int = 16, sigma_cells: float = 1.0) -> Workload:
    """2D adaptive parity case: depth 2 base refined to depth 4 inside the disc r=1/5."""
    rng = np.random.default_rng(seed)
    tree = disc_tree(2, 2, 4)
    return _leafwise_instance("small_2d_adaptive", tree, rng, per_leaf, base_level=2,
                              sigma_cells=sigma_cells, steps=5)


def small_3d(seed: int = 0, ppc: int = 8) -> Workload:
    """3D periodic regular depth 2 (9^3) parity case with 5% tunnelers."""
    rng = np.random.default_rng(seed)
    tree = regular_tree(3, 2)
    return _langmuir_instance("small_3d_L2", tree, rng, ppc * 9 ** 3, 1.0, 0.01, [1], 5,
                              tunnel_frac=0.05, tunnel_max=10.0)


def small_3d_adaptive(seed: int = 0, per_leaf: int = 8) -> Workload:
    """3D adaptive parity case: depth 1 base refined to depth 3 inside the ball r=1/5."""
    rng = np.random.default_rng(seed)
    tree = disc_tree(3, 1, 3)
    return _leafwise_instance("small_3d_adaptive", tree, rng, per_leaf, base_level=1,
                              sigma_cells=1.0, steps=5)


CONFIG_NAMES = {
    "config1": config1, "config2": config2, "config3": config3, "config4": config4,
    "small_adaptive": small_adaptive, "small_3d": small_3d,
    "small_3d_adaptive": small_3d_adaptive,
}


def by_name(name: str, **kw):
    return CONFIG_NAMES[name](**kw)
