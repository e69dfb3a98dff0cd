"""Membership of the overlapping data blocks (paper Sec. 2.1), written out
directly from the rule, in numpy (test infrastructure only).

A block is a rectangle [gx0, gx1) x [gy0, gy1) of whole grid units of the
domain; the edge of unit g along an axis is lo + g * len / ng, evaluated in
float64 and rounded once to float32, and the rectangles at the outer edges of
the tiling reach to infinity.  A particle's home is the rectangle that holds
its (x, y) (block 0 when none does, i.e. for a NaN coordinate).  It is a
member of every block whose rectangle, widened by r_s (1 + 1e-5) in float32,
holds (x, y), and always of its home; it is active in its home block if it is
active in the domain, and passive everywhere else.  A block lists its active
members first, each group by increasing domain index.

Exact forces of the blocks follow from the domain's own forces (the oracle's
force on the whole domain), so this module only needs the membership.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

F32 = np.float32


def _edge(lo, length, ng, g) -> np.float32:
    return F32(float(lo) + g * float(length) / ng)


def rectangles(domain, ng: Sequence[int], blocks: Sequence[Sequence[int]]):
    """Per block: home bounds (x0, x1, y0, y1) and widened bounds, float32."""
    rs = F32(float(F32(domain.r_s)) * (1.0 + 1e-5))
    inf = F32(np.inf)
    home, wide = [], []
    for gx0, gx1, gy0, gy1 in blocks:
        h = []
        for a, (g0, g1) in enumerate(((gx0, gx1), (gy0, gy1))):
            lo = -inf if g0 == 0 else _edge(domain.lo[a], domain.len[a], ng[a], g0)
            hi = inf if g1 == ng[a] else _edge(domain.lo[a], domain.len[a], ng[a], g1)
            h += [lo, hi]
        home.append(h)
        wide.append([F32(h[0] - rs), F32(h[1] + rs), F32(h[2] - rs), F32(h[3] + rs)])
    return np.array(home, F32), np.array(wide, F32)


def members(pos: np.ndarray, n_active: int, domain, ng, blocks) -> List[Tuple[np.ndarray, np.ndarray]]:
    """(active indices, passive indices) of every block, each ascending."""
    pos = np.asarray(pos, F32)
    x, y = pos[:, 0], pos[:, 1]
    home_r, wide_r = rectangles(domain, ng, blocks)
    n = pos.shape[0]
    home = np.full(n, -1, np.int64)
    with np.errstate(invalid="ignore"):
        for b in range(len(blocks)):
            x0, x1, y0, y1 = home_r[b]
            inside = (x >= x0) & (x < x1) & (y >= y0) & (y < y1) & (home < 0)
            home[inside] = b
    home[home < 0] = 0
    idx = np.arange(n)
    out = []
    with np.errstate(invalid="ignore"):
        for b in range(len(blocks)):
            x0, x1, y0, y1 = wide_r[b]
            mem = ((x >= x0) & (x < x1) & (y >= y0) & (y < y1)) | (home == b)
            act = mem & (home == b) & (idx < n_active)
            out.append((idx[act], idx[mem & ~act]))
    return out


def order(memb) -> np.ndarray:
    """Domain index of every block member, blocks back to back."""
    parts = [np.concatenate([a, p]) for a, p in memb]
    return np.concatenate(parts) if parts else np.zeros(0, np.int64)
