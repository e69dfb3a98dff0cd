"""Seeded synthetic particle sets for the short-range force.

This module only draws inputs: positions, masses, cotangents and sample
indices.  It holds none of the force arithmetic, so both the device path and
the CPU oracle can take their inputs from here.

Units follow the paper's production run (Sec. 3.1): lengths in PM grid cells
and one particle per cell on average (8192^3 particles on an 8192^3 grid), so
the Plummer length that matches the stated 2 kpc/h force resolution is about
0.02 cells.  One node of that run owns about 2^25 particles (Sec. 3, 16,384
nodes), which sets the size of the largest workload ("node_share").

Recipes (numpy PCG64 through ``default_rng(seed)``; coordinates drawn in
float64, wrapped into the generation box, cast to float32, and any value that
rounds up to the upper face folded back to the lower face):

* uniform: i.i.d. uniform positions in the box.
* clustered: a uniform background plus Plummer spheres.  Halo sizes follow
  log-uniform relative weights scaled to the halo share of the particle budget
  (largest-remainder rounding), scale radii are log-uniform in [0.5, 4] cells,
  centres are uniform, radii are drawn from the Plummer mass profile truncated
  at ten scale radii, directions are isotropic.  The particle order is then
  shuffled, as in a real particle store.
* slab with ghosts: a clustered periodic generation box [-w, S+w)^3; particles
  inside [0, S)^3 are active (stored first), the rest form the overloaded ghost
  shell of width w (Sec. 2: overload scheme; Sec. 2.1: active and passive
  particles).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import filter_fit

F32 = np.float32


def f32(x: float) -> float:
    """Round a Python float to the nearest float32 value."""
    return float(F32(x))


@dataclass(frozen=True)
class Problem:
    """One short-range problem: domain, cutoff, softening and filter."""

    lo: Tuple[float, float, float]
    len: Tuple[float, float, float]
    periodic: bool
    r_s: float
    eps: float
    poly: Tuple[float, ...]
    leaf_depth: int = 1  # octree levels of the in-cell order (1 = octants)

    @staticmethod
    def make(lo, length, periodic, r_s, eps, poly, leaf_depth: int = 1) -> "Problem":
        lo = tuple(f32(v) for v in lo)
        length = tuple(f32(v) for v in length)
        poly = tuple(f32(v) for v in poly)
        if len(poly) != 6:
            raise ValueError("poly needs 6 coefficients")
        return Problem(lo, length, bool(periodic), f32(r_s), f32(eps), poly, int(leaf_depth))

    def with_leaf_depth(self, depth: int) -> "Problem":
        return replace(self, leaf_depth=int(depth))


def filter_poly(r_s: float, eps: float) -> Tuple[float, ...]:
    return tuple(f32(c) for c in filter_fit.load(r_s, eps))


@dataclass
class Workload:
    name: str
    pos: np.ndarray  # float32 [N, 3]
    mass: np.ndarray  # float32 [N]
    n_active: int
    problem: Problem
    notes: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


@dataclass
class Batch:
    """Many independent problems stored back to back."""

    name: str
    pos: np.ndarray  # float32 [sum N_b, 3]
    mass: np.ndarray  # float32 [sum N_b]
    offsets: np.ndarray  # int64 [B+1]
    n_active: np.ndarray  # int64 [B]
    problems: List[Problem]
    notes: dict = field(default_factory=dict)

    @property
    def size(self) -> int:
        return len(self.problems)

    def part(self, b: int) -> Workload:
        s, e = int(self.offsets[b]), int(self.offsets[b + 1])
        return Workload(f"{self.name}[{b}]", self.pos[s:e], self.mass[s:e],
                        int(self.n_active[b]), self.problems[b])


@dataclass
class HaloCatalogue:
    """Friends-of-friends style halo membership: halo h holds particles
    [offsets[h], offsets[h+1]), coordinates unwrapped."""

    name: str
    pos: np.ndarray  # float32 [n, 3]
    mass: np.ndarray  # float32 [n]
    offsets: np.ndarray  # int64 [H+1]
    eps: float
    notes: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_halos(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def pairs(self) -> int:
        """Ordered pairs (i, j != i) inside halos: the centre finder's work."""
        c = np.diff(self.offsets).astype(np.int64)
        return int(np.sum(c * (c - 1)))


# --------------------------------------------------------------------------
# primitive draws
# --------------------------------------------------------------------------

def _to_box32(x64: np.ndarray, lo: float, length: float) -> np.ndarray:
    """Wrap float64 coordinates into [lo, lo+length) and cast to float32."""
    u = np.mod(x64 - lo, length)
    x = (u + lo).astype(F32)
    hi = F32(lo + length)
    x[x >= hi] = F32(lo)
    return x


def largest_remainder(budget: int, weights: np.ndarray) -> np.ndarray:
    """Integer counts proportional to weights that sum exactly to budget."""
    quota = budget * weights / weights.sum()
    counts = np.floor(quota).astype(np.int64)
    rest = budget - int(counts.sum())
    if rest > 0:
        frac = quota - counts
        order = np.argsort(-frac, kind="stable")
        counts[order[:rest]] += 1
    return counts


def plummer_offsets(rng: np.random.Generator, scale: np.ndarray) -> np.ndarray:
    """Offsets from the halo centre for particles with Plummer scale radii."""
    n = scale.shape[0]
    umax = (100.0 / 101.0) ** 1.5  # truncation at 10 scale radii
    u = rng.random(n) * umax
    with np.errstate(divide="ignore"):
        r = scale / np.sqrt(np.power(u, -2.0 / 3.0) - 1.0)
    r[~np.isfinite(r)] = 0.0
    cz = rng.random(n) * 2.0 - 1.0
    phi = rng.random(n) * (2.0 * math.pi)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([r * sz * np.cos(phi), r * sz * np.sin(phi), r * cz], axis=1)


def clustered_positions(rng: np.random.Generator, n: int, lo: float, length: float,
                        halo_frac: float, n_halos: int, mass_range=(1e2, 1e5),
                        scale_range=(0.5, 4.0)) -> Tuple[np.ndarray, dict]:
    """float64 positions in the periodic box [lo, lo+length)^3 (unwrapped)."""
    budget = int(round(halo_frac * n))
    n_bg = n - budget
    bg = lo + rng.random((n_bg, 3)) * length
    logm = rng.uniform(math.log(mass_range[0]), math.log(mass_range[1]), n_halos)
    loga = rng.uniform(math.log(scale_range[0]), math.log(scale_range[1]), n_halos)
    centres = lo + rng.random((n_halos, 3)) * length
    counts = largest_remainder(budget, np.exp(logm))
    halo_id = np.repeat(np.arange(n_halos), counts)
    off = plummer_offsets(rng, np.exp(loga)[halo_id])
    halo = centres[halo_id] + off
    pos = np.concatenate([bg, halo], axis=0)
    pos = pos[rng.permutation(n)]
    return pos, {"halo_budget": budget, "max_halo": int(counts.max()) if n_halos else 0}


def power_law_counts(rng: np.random.Generator, k: int, n_min: float, n_max: float,
                     slope: float) -> np.ndarray:
    """k integers with dN/dn proportional to n^-slope on [n_min, n_max] (inverse CDF)."""
    a = 1.0 - slope
    u = rng.random(k)
    x = (n_min ** a + u * (n_max ** a - n_min ** a)) ** (1.0 / a)
    return np.floor(x).astype(np.int64)


def halo_members(rng: np.random.Generator, counts: np.ndarray, box: float) -> np.ndarray:
    """float64 positions of Plummer halos with the given particle counts: scale
    radius R200 / 5 with R200 = (3 n / (800 pi))^(1/3) (200 times a mean density
    of one particle per cell), centres uniform in [0, box)^3, particles shuffled
    inside each halo."""
    H = counts.shape[0]
    centres = rng.random((H, 3)) * box
    r200 = np.cbrt(3.0 * np.maximum(counts, 1) / (800.0 * math.pi))
    hid = np.repeat(np.arange(H), counts)
    pos = centres[hid] + plummer_offsets(rng, (r200 / 5.0)[hid])
    offsets = np.concatenate([[0], np.cumsum(counts)])
    for h in range(H):
        a, b = offsets[h], offsets[h + 1]
        if b - a > 1:
            pos[a:b] = pos[a:b][rng.permutation(b - a)]
    return pos


def halo_catalogue(n_halos: int, seed: int, n_min: float = 40, n_max: float = 1e6,
                   slope: float = 1.9, box: float = 320.0, eps: float = 0.02,
                   name: str = "halos") -> HaloCatalogue:
    rng = np.random.default_rng(seed)
    counts = power_law_counts(rng, n_halos, n_min, n_max, slope)
    pos = halo_members(rng, counts, box).astype(F32)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return HaloCatalogue(name, pos, np.ones(pos.shape[0], F32), offsets, eps,
                         {"seed": seed, "slope": slope, "n_min": n_min, "n_max": n_max,
                          "max_halo": int(counts.max()) if n_halos else 0})


def halos_small() -> HaloCatalogue:
    """Halo sizes around the kernel's group boundaries, empty halos included,
    random masses."""
    counts = np.array([0, 1, 2, 3, 40, 63, 64, 65, 0, 127, 128, 129, 255, 256, 257, 500, 1000,
                       4099, 7, 0], np.int64)
    rng = np.random.default_rng(11)
    pos = halo_members(rng, counts, 64.0).astype(F32)
    mass = rng.uniform(0.5, 2.0, pos.shape[0]).astype(F32)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return HaloCatalogue("halos_small", pos, mass, offsets, 0.02, {"seed": 11})


def halos_node() -> HaloCatalogue:
    """One node's halo catalogue at late times: 10,200 halos of 40 particles and
    up, dN/dn ~ n^-1.9 up to 1e6 (mean about 630 particles per halo)."""
    return halo_catalogue(10200, 0, name="halos_node")


def clustered_positions_absolute(rng: np.random.Generator, n: int, lo: float, length: float,
                                 halo_frac: float, mass_range=(1e2, 1e5),
                                 scale_range=(0.5, 4.0)) -> Tuple[np.ndarray, dict]:
    """Halo masses taken as absolute particle counts, drawn log-uniform until
    the halo budget is full (the last halo takes what is left): few, very
    large halos (float64 positions, unwrapped)."""
    budget = int(round(halo_frac * n))
    counts = []
    total = 0
    while total < budget:
        m = int(math.exp(rng.uniform(math.log(mass_range[0]), math.log(mass_range[1]))))
        m = max(1, min(m, budget - total))
        counts.append(m)
        total += m
    counts = np.array(counts, np.int64)
    H = counts.shape[0]
    loga = rng.uniform(math.log(scale_range[0]), math.log(scale_range[1]), H)
    centres = lo + rng.random((H, 3)) * length
    hid = np.repeat(np.arange(H), counts)
    halo = centres[hid] + plummer_offsets(rng, np.exp(loga)[hid])
    bg = lo + rng.random((n - budget, 3)) * length
    pos = np.concatenate([bg, halo], axis=0)
    pos = pos[rng.permutation(n)]
    return pos, {"halo_budget": budget, "halos": H, "max_halo": int(counts.max()) if H else 0}


def clustered_box_absolute(n: int, length: float, seed: int, halo_frac: float = 0.4,
                           mass_range=(1e2, 1e5), r_s: float = 3.0, eps: float = 0.05,
                           name: str = "clustered_abs") -> Workload:
    rng = np.random.default_rng(seed)
    p64, info = clustered_positions_absolute(rng, n, 0.0, length, halo_frac, mass_range)
    prob = Problem.make((0, 0, 0), (length,) * 3, True, r_s, eps, filter_poly(r_s, eps))
    info["seed"] = seed
    return Workload(name, _to_box32(p64, 0.0, length), np.ones(n, F32), n, prob, info)


def clustered_2m_extreme() -> Workload:
    """The 2M box with halo masses as absolute counts (a few halos up to ~1e5
    particles): the extreme-clustering stress case."""
    return clustered_box_absolute(2097152, 128.0, 0, name="clustered_2m_extreme")


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def uniform_box(n: int, length: float, seed: int, r_s: float = 3.0, eps: float = 0.05,
                name: str = "uniform") -> Workload:
    rng = np.random.default_rng(seed)
    pos = _to_box32(rng.random((n, 3)) * length, 0.0, length)
    prob = Problem.make((0, 0, 0), (length,) * 3, True, r_s, eps, filter_poly(r_s, eps))
    return Workload(name, pos, np.ones(n, F32), n, prob, {"seed": seed})


def clustered_box(n: int, length: float, n_halos: int, seed: int, halo_frac: float = 0.4,
                  mass_range=(1e2, 1e5), r_s: float = 3.0, eps: float = 0.05,
                  name: str = "clustered") -> Workload:
    rng = np.random.default_rng(seed)
    p64, info = clustered_positions(rng, n, 0.0, length, halo_frac, n_halos, mass_range)
    pos = _to_box32(p64, 0.0, length)
    prob = Problem.make((0, 0, 0), (length,) * 3, True, r_s, eps, filter_poly(r_s, eps))
    info["seed"] = seed
    return Workload(name, pos, np.ones(n, F32), n, prob, info)


def slab_with_ghosts(side: int, ghost: float, n_halos: int, seed: int, halo_frac: float = 0.75,
                     mass_range=(1e2, 1e6), r_s: float = 3.0, eps: float = 0.02,
                     name: str = "slab") -> Workload:
    """Active cube [0, side)^3 plus a ghost shell of width ``ghost``, open domain."""
    ext = side + 2.0 * ghost
    n = int(round(ext ** 3))  # one particle per cell on average
    rng = np.random.default_rng(seed)
    p64, info = clustered_positions(rng, n, -ghost, ext, halo_frac, n_halos, mass_range)
    pos = _to_box32(p64, -ghost, ext)
    inside = np.all((pos >= F32(0.0)) & (pos < F32(side)), axis=1)
    order = np.concatenate([np.nonzero(inside)[0], np.nonzero(~inside)[0]])
    pos = np.ascontiguousarray(pos[order])
    n_act = int(inside.sum())
    prob = Problem.make((-ghost,) * 3, (ext,) * 3, False, r_s, eps, filter_poly(r_s, eps))
    info.update(seed=seed, n_ghost=n - n_act)
    return Workload(name, pos, np.ones(n, F32), n_act, prob, info)


def subvolume_batch(n_sub: int = 96, count_range=(1e4, 1e6), count_seed: int = 3,
                    seed_base: int = 1000, r_s: float = 3.0, eps: float = 0.05,
                    name: str = "subvolumes") -> Batch:
    """Independent periodic uniform subvolumes at one particle per cell."""
    rng = np.random.default_rng(count_seed)
    counts = np.floor(np.exp(rng.uniform(math.log(count_range[0]), math.log(count_range[1]),
                                         n_sub))).astype(np.int64)
    poly = filter_poly(r_s, eps)
    parts, probs = [], []
    for b, nb in enumerate(counts):
        length = float(nb) ** (1.0 / 3.0)
        r = np.random.default_rng(seed_base + b)
        parts.append(_to_box32(r.random((int(nb), 3)) * length, 0.0, length))
        probs.append(Problem.make((0, 0, 0), (length,) * 3, True, r_s, eps, poly))
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    pos = np.ascontiguousarray(np.concatenate(parts, axis=0))
    return Batch(name, pos, np.ones(pos.shape[0], F32), offsets, counts.copy(), probs,
                 {"count_seed": count_seed, "seed_base": seed_base})


def cotangent(n: int, seed: int) -> np.ndarray:
    """N(0,1) float32 cotangent on the forces, shape [n, 3]."""
    return np.random.default_rng(seed).standard_normal((n, 3)).astype(F32)


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct sorted indices in [0, n)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def uniform_32k() -> Workload:
    """32^3 equal-mass particles, uniform in a periodic box of 32 cells, seed 0."""
    return uniform_box(32768, 32.0, 0, name="uniform_32k")


def clustered_2m() -> Workload:
    """128^3 particles, box 128: 60% uniform, 40% in 2000 Plummer halos, seed 0."""
    return clustered_box(2097152, 128.0, 2000, 0, name="clustered_2m")


def subvolumes_96() -> Batch:
    """96 periodic subvolumes, 1e4..1e6 particles each (log-uniform), seeds 3 / 1000+b."""
    return subvolume_batch(name="subvolumes_96")


def clustered_16m() -> Workload:
    """256^3 particles, box 256, 60% uniform, 40% in 16,000 Plummer halos, seed 0."""
    return clustered_box(16777216, 256.0, 16000, 0, name="clustered_16m")


def node_share() -> Workload:
    """320^3 active cells plus a 3-cell ghost shell, 25% uniform, 75% in 20,000 halos."""
    return slab_with_ghosts(320, 3.0, 20000, 0, name="node_share")


WORKLOADS = {
    "uniform_32k": uniform_32k,
    "clustered_2m": clustered_2m,
    "subvolumes_96": subvolumes_96,
    "clustered_16m": clustered_16m,
    "node_share": node_share,
    "clustered_2m_extreme": clustered_2m_extreme,
    "halos_small": halos_small,
    "halos_node": halos_node,
}


def get(name: str):
    return WORKLOADS[name]()
