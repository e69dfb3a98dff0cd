"""Overlapping data blocks on one GPU (paper Sec. 2.1).

A domain is split into blocks that each hold their own active particles plus
passive copies of every particle within r_s; the blocks are solved as
independent problems (here: one batched launch, ``sr_batch_force``) and the
results reconciled, keeping each active particle's acceleration from its home
block.  The blocks are rectangles of whole grid units in x and y, made by an
equal partition (``equal_blocks``); a block whose measured cost exceeds twice
the mean is split in two along its longer side (``refine``), repeatedly, so
that blocks stay as large as the balance allows.

All device work (partition, gathers, forces, reconcile) runs in libsr; this
module only sequences the calls and applies the host-side refinement rule.
"""
from __future__ import annotations

import os
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _sr

Rect = Tuple[int, int, int, int]  # (gx0, gx1, gy0, gy1), grid units, half-open



def grid_units(domain) -> Tuple[int, int]:
    """Grid units across the domain in x and y: the side in grid cells, at least 1."""
    return (max(1, int(round(float(domain.len[0])))), max(1, int(round(float(domain.len[1])))))


def _cuts(n: int, k: int) -> List[int]:
    k = max(1, min(int(k), n))
    return [(n * j) // k for j in range(k + 1)]


def equal_blocks(ng: Sequence[int], nbx: int, nby: int = 1) -> List[Rect]:
    """nbx x nby rectangles of (nearly) equal size in whole grid units, x-major."""
    xs, ys = _cuts(int(ng[0]), nbx), _cuts(int(ng[1]), nby)
    return [(xs[i], xs[i + 1], ys[j], ys[j + 1]) for i in range(len(xs) - 1)
            for j in range(len(ys) - 1)]


def split(rect: Rect) -> List[Rect]:
    """Halve a rectangle along its longer side (x on ties); a 1x1 rectangle stays whole."""
    x0, x1, y0, y1 = rect
    if x1 - x0 >= y1 - y0 and x1 - x0 >= 2:
        xm = (x0 + x1) // 2
        return [(x0, xm, y0, y1), (xm, x1, y0, y1)]
    if y1 - y0 >= 2:
        ym = (y0 + y1) // 2
        return [(x0, x1, y0, ym), (x0, x1, ym, y1)]
    return [rect]


def refine(blocks: Sequence[Rect], cost: Sequence[float], factor: float = 2.0) -> List[Rect]:
    """One refinement step: every block whose cost is more than ``factor`` times
    the mean block cost is divided a factor of two finer; the others are kept.
    Order is preserved (a split block is replaced by its halves in place)."""
    cost = np.asarray(cost, dtype=np.float64)
    if cost.shape != (len(blocks),):
        raise ValueError("one cost per block")
    mean = float(cost.mean()) if len(blocks) else 0.0
    out: List[Rect] = []
    for b, c in zip(blocks, cost):
        out.extend(split(b) if c > factor * mean else [b])
    return out


class _PhaseClock:
    def __init__(self, times: Optional[dict]):
        self.times = times
        if times is not None:
            import time

            self._now = time.perf_counter
            torch.cuda.synchronize()
            self.t = self._now()

    def tick(self, name: str) -> None:
        if self.times is None:
            return
        torch.cuda.synchronize()
        t = self._now()
        self.times[name] = self.times.get(name, 0.0) + 1e3 * (t - self.t)
        self.t = t


def membership_estimate(domain, ng: Sequence[int], blocks: Sequence[Rect]) -> float:
    """Memberships per particle for a uniform density: the widened rectangles'
    areas inside the domain, over the domain's area."""
    lo = [float(domain.lo[0]), float(domain.lo[1])]
    ln = [float(domain.len[0]), float(domain.len[1])]
    r = float(domain.r_s)
    total = 0.0
    for b in blocks:
        area = 1.0
        for a, (g0, g1) in enumerate(((b[0], b[1]), (b[2], b[3]))):
            x0 = lo[a] + g0 * ln[a] / ng[a] - (r if g0 > 0 else 0.0)
            x1 = lo[a] + g1 * ln[a] / ng[a] + (r if g1 < ng[a] else 0.0)
            area *= max(0.0, min(x1, lo[a] + ln[a]) - max(x0, lo[a]))
        total += area
    return total / (ln[0] * ln[1])


class BlockForce:
    """Short-range forces of one open domain computed block by block.

    ``capacity`` bounds the total memberships; by default it is 1.3 times the
    uniform-density estimate.  When a partition needs more (clustering), the
    plan is rebuilt with the reported need."""

    def __init__(self, domain, blocks: Sequence[Rect], n: int, n_active: Optional[int] = None,
                 ng: Optional[Sequence[int]] = None, capacity: Optional[int] = None, device="cuda",
                 tune_cache: Optional[str] = None):
        self.domain = domain
        self.ng = tuple(ng) if ng is not None else grid_units(domain)
        self.blocks = [tuple(int(v) for v in b) for b in blocks]
        self.n = int(n)
        if capacity is None:
            capacity = int(1.3 * membership_estimate(domain, self.ng, self.blocks) * self.n) + 4096
        self.n_active = self.n if n_active is None else int(n_active)
        self.device = device
        self.tune_cache = tune_cache if tune_cache is not None else _sr.default_tune_cache()
        self._make_plan(capacity)
        self.problems = self.plan.problems()
        self._batch = None
        self._batch_key = None
        self._batch_ws = None
        self._bufs = None

    def _make_plan(self, capacity: int) -> None:
        self.plan = _sr.BlocksPlan(self.domain, self.ng, self.blocks, self.n, self.n_active, capacity)
        self.ws = _sr.new_workspace(self.plan.ws_bytes, self.device)

    def partition(self, pos):
        try:
            return self.plan.partition(pos, self.ws)
        except _sr.SRError as e:
            if e.code != 2 or getattr(e, "needed", 0) <= 0:
                raise
            self.plan.close()
            self._make_plan(int(e.needed * 1.05) + 1024)
            return self.plan.partition(pos, self.ws)

    @property
    def counts(self) -> np.ndarray:
        return self.plan.counts

    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.counts.sum(axis=1))]).astype(np.int64)

    def batch_plan(self) -> "_sr.BatchPlan":
        key = tuple(self.counts.reshape(-1).tolist())
        if self._batch is None or self._batch_key != key:
            if self._batch is not None:
                self._batch.close()
            self._batch = _sr.BatchPlan(self.offsets(), self.counts[:, 0], self.problems,
                                        tune_cache=self.tune_cache)
            self._batch_key = key
            if self._batch_ws is None or self._batch_ws.numel() < self._batch.ws_bytes:
                self._batch_ws = _sr.new_workspace(self._batch.ws_bytes, self.device)
        return self._batch

    def _buffers(self, device):
        """Block inputs and outputs, kept while the membership count holds so
        that a captured batch graph stays bound to the same pointers."""
        m = self.plan.members
        if self._bufs is None or self._bufs[0].shape[0] != m:
            self._bufs = (torch.empty((m, 3), dtype=torch.float32, device=device),
                          torch.empty((m,), dtype=torch.float32, device=device),
                          torch.empty((self.n_active, 3), dtype=torch.float32, device=device))
        return self._bufs

    def forward(self, pos, mass, mode: str = "graph", partition: bool = True,
                times: Optional[dict] = None):
        """Accelerations [n_active, 3] of the domain's active particles.

        With ``times`` (a dict), the device is synchronised after each phase
        and the phase's wall-clock milliseconds are added under its name."""
        clock = _PhaseClock(times)
        if partition:
            self.partition(pos)
            clock.tick("partition")
        bpos, bmass, bacc = self._buffers(pos.device)
        self.plan.gather(pos, mass, self.ws, bpos=bpos, bmass=bmass, want_src=False)
        clock.tick("gather")
        plan = self.batch_plan()
        # the block buffers are reallocated when the membership count changes:
        # let a graph-mode plan capture again for them
        plan.run(bpos, bmass, self._batch_ws, bacc, None, mode, recapture=True)
        clock.tick("force")
        acc = self.plan.reconcile(bacc, self.ws)
        clock.tick("reconcile")
        return acc

    def vjp(self, pos, mass, g, partition: bool = True):
        """Position gradient [n, 3] of sum_i g_i . a_i, each block's copies summed."""
        if partition:
            self.partition(pos)
        bpos, bmass, _, bg = self.plan.gather(pos, mass, self.ws, g=g)
        off = self.offsets()
        rows = np.concatenate([[0], np.cumsum(self.counts[:, 0])])
        bgrad = torch.empty((self.plan.members, 3), dtype=torch.float32, device=pos.device)
        for b, prob in enumerate(self.problems):
            lo, hi = int(off[b]), int(off[b + 1])
            if hi == lo:
                continue
            na = int(self.counts[b, 0])
            _sr.force_vjp(bpos[lo:hi], bmass[lo:hi], prob, bg[int(rows[b]): int(rows[b]) + na], na,
                          out=bgrad[lo:hi])
        return self.plan.reconcile_grad(bgrad, self.ws)

    def block_costs(self, pos, mass, kind: str = "time", repeats: int = 2) -> np.ndarray:
        """Cost of each block of the current partition: the wall-clock time of its
        force on the GPU in ms (``time``, the paper's measure) or its number of
        interacting pairs (``pairs``, deterministic)."""
        bpos, bmass, _, _ = self.plan.gather(pos, mass, self.ws)
        off = self.offsets()
        out = np.zeros(len(self.blocks))
        for b, prob in enumerate(self.problems):
            lo, hi = int(off[b]), int(off[b + 1])
            na = int(self.counts[b, 0])
            if hi == lo or na == 0:
                continue
            ws = _sr.new_workspace(_sr.workspace_bytes(hi - lo, prob), pos.device)
            if kind == "pairs":
                _sr.bin(bpos[lo:hi], bmass[lo:hi], prob, na, ws=ws)
                out[b] = float(_sr.count_pairs(ws, hi - lo, prob, na).item())
                continue
            acc = torch.empty((na, 3), dtype=torch.float32, device=pos.device)
            _sr.force(bpos[lo:hi], bmass[lo:hi], prob, na, ws=ws, out=acc)  # warm
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(repeats):
                _sr.force(bpos[lo:hi], bmass[lo:hi], prob, na, ws=ws, out=acc)
            t1.record()
            t1.synchronize()
            out[b] = t0.elapsed_time(t1) / repeats
        return out

    def close(self):
        if self._batch is not None:
            self._batch.close()
            self._batch = None
        self.plan.close()


def balanced_blocks(pos, mass, domain, n_active: Optional[int] = None, nbx: int = 2, nby: int = 2,
                    kind: str = "time", factor: float = 2.0, max_rounds: int = 6,
                    ng: Optional[Sequence[int]] = None) -> Tuple[List[Rect], List[np.ndarray]]:
    """Start from an equal nbx x nby partition and refine slow blocks until no
    block costs more than ``factor`` times the mean (or nothing can split).
    Returns the blocks and the cost vector of every round."""
    ng = tuple(ng) if ng is not None else grid_units(domain)
    blocks = equal_blocks(ng, nbx, nby)
    history = []
    n = int(pos.shape[0])
    for _ in range(max_rounds):
        bf = BlockForce(domain, blocks, n, n_active, ng=ng, device=pos.device)
        bf.partition(pos)
        cost = bf.block_costs(pos, mass, kind)
        bf.close()
        history.append(cost)
        nxt = refine(blocks, cost, factor)
        if nxt == blocks:
            break
        blocks = nxt
    return blocks, history
