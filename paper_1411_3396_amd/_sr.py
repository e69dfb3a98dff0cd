"""ctypes binding of libsr (argument marshalling only).

Every step of the force path runs in the library's HIP kernels; torch
supplies device memory (inputs, outputs, workspaces) and the current stream.
The binding raises if the library or a GPU is missing: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsr.so")

SR_OK = 0
STATUS = {0: "SR_OK", 1: "SR_E_ARG", 2: "SR_E_WORKSPACE", 3: "SR_E_DEVICE", 4: "SR_E_PLAN",
          5: "SR_E_UNSUPPORTED"}
REUSE_BINS = 1
BATCH_PER_SUBVOLUME = 1
BATCH_EAGER = 2
BATCH_RECAPTURE = 4
COUNT_ADJOINT = 1
FLAG_NONFINITE = 1
FLAG_OUT_OF_DOMAIN = 2
FLAG_NOT_BINNED = 4
FLAG_QUEUE = 8

# the exported names of sr.h, in declaration order
EXPORTS = ("sr_abi_version", "sr_status_str", "sr_grid", "sr_workspace_bytes", "sr_bin",
           "sr_bin_view", "sr_force", "sr_force_static", "sr_force_vjp", "sr_count_pairs", "sr_momentum",
           "sr_ws_flags", "sr_batch_plan_create", "sr_batch_force", "sr_batch_plan_destroy",
           "sr_batch_plan_info", "sr_blocks_plan_create", "sr_blocks_plan_destroy",
           "sr_blocks_problems", "sr_blocks_partition", "sr_blocks_gather", "sr_blocks_reconcile",
           "sr_blocks_reconcile_grad", "sr_centres_plan_create", "sr_centres_plan_destroy",
           "sr_centres", "sr_pk_plan_create", "sr_pk_plan_destroy", "sr_pk_deposit", "sr_pk_grid",
           "sr_power_spectrum", "sr_launch_config", "sr_launch_config_kernel", "sr_tile_config", "sr_tile_balance", "sr_sparse_group",
           "sr_timing_enable",
           "sr_timing_read")


def default_tune_cache() -> str:
    """Where batch plans keep tuned launch parameters: $SR_TUNE_CACHE, else a
    file in the user's cache directory (never inside the package)."""
    path = os.environ.get("SR_TUNE_CACHE")
    if path:
        return path
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    d = os.path.join(base, "paper_1411_3396_amd")
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, "tune_cache.json")


class SRError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = int(code)
        super().__init__(f"{what}: {STATUS.get(self.code, self.code)}")


class Problem(C.Structure):
    _fields_ = [("lo", C.c_float * 3), ("len", C.c_float * 3), ("periodic", C.c_int32),
                ("r_s", C.c_float), ("eps", C.c_float), ("poly", C.c_float * 6),
                ("leaf_depth", C.c_int32)]


class Block(C.Structure):
    _fields_ = [("gx0", C.c_int32), ("gx1", C.c_int32), ("gy0", C.c_int32), ("gy1", C.c_int32)]


class BinLayout(C.Structure):
    _fields_ = [("nc", C.c_int32 * 3), ("ncell", C.c_int64), ("cell_of", C.c_void_p),
                ("cell_start", C.c_void_p), ("cell_nact", C.c_void_p), ("perm", C.c_void_p),
                ("off_x", C.c_void_p), ("off_y", C.c_void_p), ("off_z", C.c_void_p),
                ("mass", C.c_void_p)]


# sr_problem layout and entry points of include/sr.h (SR_ABI_VERSION)
ABI_VERSION = 6

_lib = None


def lib():
    """Load libsr.so; raise if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsr.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        p, i64, u = C.c_void_p, C.c_int64, C.c_uint
        L.sr_abi_version.restype = C.c_int
        L.sr_status_str.restype = C.c_char_p
        L.sr_status_str.argtypes = [C.c_int]
        L.sr_grid.argtypes = [p, p]
        L.sr_workspace_bytes.argtypes = [i64, p, p]
        L.sr_bin.argtypes = [p, p, i64, i64, p, p, C.c_size_t, p]
        L.sr_bin_view.argtypes = [p, i64, i64, p, p]
        L.sr_force.argtypes = [p, p, i64, i64, p, p, C.c_size_t, u, p, p]
        L.sr_force_static.argtypes = [p, p, i64, i64, p, p, p]
        L.sr_force_vjp.argtypes = [p, p, i64, i64, p, p, C.c_size_t, u, p, p, p]
        L.sr_count_pairs.argtypes = [i64, i64, p, p, C.c_size_t, u, p, p]
        L.sr_momentum.argtypes = [p, p, i64, p, C.c_size_t, p, p]
        L.sr_ws_flags.argtypes = [p, p, p]
        L.sr_batch_plan_create.argtypes = [C.c_int32, p, p, p, C.c_char_p, p, p]
        L.sr_batch_force.argtypes = [p, p, p, p, C.c_size_t, p, p, u, p]
        L.sr_batch_plan_destroy.argtypes = [p]
        L.sr_batch_plan_info.argtypes = [p, p, C.c_size_t]
        L.sr_blocks_plan_create.argtypes = [p, p, C.c_int32, p, i64, i64, i64, p, p]
        L.sr_blocks_plan_destroy.argtypes = [p]
        L.sr_blocks_problems.argtypes = [p, p]
        L.sr_blocks_partition.argtypes = [p, p, p, C.c_size_t, p, p, p]
        L.sr_blocks_gather.argtypes = [p, p, p, p, p, C.c_size_t, p, p, p, p, p]
        L.sr_blocks_reconcile.argtypes = [p, p, C.c_size_t, p, p, p]
        L.sr_blocks_reconcile_grad.argtypes = [p, p, C.c_size_t, p, p, p]
        L.sr_centres_plan_create.argtypes = [C.c_int32, p, p, p]
        L.sr_centres_plan_destroy.argtypes = [p]
        L.sr_centres.argtypes = [p, p, p, C.c_float, p, C.c_size_t, p, p, p, p]
        L.sr_pk_plan_create.argtypes = [C.c_int32, C.c_double, C.c_int32, C.c_double, i64, p, p]
        L.sr_pk_plan_destroy.argtypes = [p]
        L.sr_pk_deposit.argtypes = [p, p, p, i64, p, C.c_size_t, p]
        L.sr_pk_grid.argtypes = [p, p, p, p, p]
        L.sr_power_spectrum.argtypes = [p, p, p, i64, p, C.c_size_t, p, p, p, p]
        L.sr_launch_config.argtypes = [C.c_int, C.c_int, C.c_int, p]
        L.sr_launch_config_kernel.argtypes = [C.c_char_p, C.c_int, C.c_int, C.c_int, p]
        L.sr_tile_config.argtypes = [C.c_char_p, C.c_int, C.c_int, p]
        L.sr_tile_balance.argtypes = [C.c_double, p]
        L.sr_sparse_group.argtypes = [C.c_int, p]
        L.sr_timing_enable.argtypes = [C.c_int]
        L.sr_timing_read.argtypes = [C.c_char_p, p, p]
        for name in EXPORTS:
            if name not in ("sr_abi_version", "sr_status_str"):
                getattr(L, name).restype = C.c_int
        if L.sr_abi_version() != ABI_VERSION:
            raise ImportError(f"libsr.so has ABI {L.sr_abi_version()}, this binding expects {ABI_VERSION}; "
                              "rebuild with __graft_entry__.build()")
        _lib = L
    return _lib


def _check(code: int, what: str) -> None:
    if code != SR_OK:
        raise SRError(code, what)


def as_problem(prob) -> Problem:
    """Problem struct from an object with lo, len, periodic, r_s, eps, poly (and
    optionally leaf_depth)."""
    if isinstance(prob, Problem):
        return prob
    s = Problem()
    for d in range(3):
        s.lo[d] = float(prob.lo[d])
        s.len[d] = float(prob.len[d])
    s.periodic = 1 if prob.periodic else 0
    s.r_s = float(prob.r_s)
    s.eps = float(prob.eps)
    for k in range(6):
        s.poly[k] = float(prob.poly[k])
    s.leaf_depth = int(getattr(prob, "leaf_depth", 1))
    return s


def _stream(stream=None) -> C.c_void_p:
    st = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(st.cuda_stream)


def _dev_f32(t: torch.Tensor, name: str, shape: Sequence[int]) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


def _out_f32(t: torch.Tensor, name: str, shape: Sequence[int]) -> torch.Tensor:
    """An output tensor is written in place, so it must already be contiguous."""
    if isinstance(t, torch.Tensor) and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _dev_f32(t, name, shape)


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def grid(prob):
    nc = (C.c_int32 * 3)()
    _check(lib().sr_grid(C.byref(as_problem(prob)), nc), "sr_grid")
    return tuple(nc)


def workspace_bytes(n: int, prob) -> int:
    b = C.c_size_t()
    _check(lib().sr_workspace_bytes(int(n), C.byref(as_problem(prob)), C.byref(b)),
           "sr_workspace_bytes")
    return int(b.value)


def new_workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return ws


def bin(pos, mass, prob, n_active=None, ws=None, stream=None):  # noqa: A001 (paper's verb)
    n = int(pos.shape[0])
    n_active = n if n_active is None else int(n_active)
    pos = _dev_f32(pos, "pos", (n, 3))
    mass = _dev_f32(mass, "mass", (n,))
    P = as_problem(prob)
    if ws is None:
        ws = new_workspace(workspace_bytes(n, P), pos.device)
    _check(lib().sr_bin(_ptr(pos), _ptr(mass), n, n_active, C.byref(P), _ptr(ws), ws.numel(),
                        _stream(stream)), "sr_bin")
    return ws


def bin_view(ws: torch.Tensor, n: int, prob, n_active=None) -> dict:
    """Views of the binned arrays inside a workspace (int32/float32 tensors)."""
    out = BinLayout()
    P = as_problem(prob)
    n_active = int(n) if n_active is None else int(n_active)
    _check(lib().sr_bin_view(_ptr(ws), int(n), n_active, C.byref(P), C.byref(out)), "sr_bin_view")
    base = ws.data_ptr()

    def view(ptr, count, dtype):
        off = int(ptr) - base
        return ws[off: off + 4 * count].view(dtype)

    ncell = int(out.ncell)
    return {"nc": tuple(out.nc), "ncell": ncell,
            "cell_of": view(out.cell_of, n, torch.int32),
            "cell_start": view(out.cell_start, ncell + 1, torch.int32),
            "cell_nact": view(out.cell_nact, ncell, torch.int32),
            "perm": view(out.perm, n, torch.int32),
            "off_x": view(out.off_x, n, torch.float32),
            "off_y": view(out.off_y, n, torch.float32),
            "off_z": view(out.off_z, n, torch.float32),
            "mass": view(out.mass, n, torch.float32)}


def force(pos, mass, prob, n_active=None, ws=None, reuse_bins=False, out=None, stream=None):
    """Short-range accelerations of the first n_active particles, [n_active, 3]."""
    n = int(pos.shape[0])
    n_active = n if n_active is None else int(n_active)
    pos = _dev_f32(pos, "pos", (n, 3))
    mass = _dev_f32(mass, "mass", (n,))
    P = as_problem(prob)
    if ws is None:
        if reuse_bins:
            raise ValueError("reuse_bins needs the binned workspace")
        ws = new_workspace(workspace_bytes(n, P), pos.device)
    if out is None:
        out = torch.empty((n_active, 3), dtype=torch.float32, device=pos.device)
    else:
        out = _out_f32(out, "out", (n_active, 3))
    _check(lib().sr_force(_ptr(pos), _ptr(mass), n, n_active, C.byref(P), _ptr(ws), ws.numel(),
                          REUSE_BINS if reuse_bins else 0, _ptr(out), _stream(stream)), "sr_force")
    return out


def force_static(pos, mass, prob, n_active=None, out=None, stream=None):
    """sr_force_static: the forward on the library's fixed device workspace (no allocation
    by the library; `out` may be passed so that nothing is allocated here either)."""
    n = int(pos.shape[0])
    n_active = n if n_active is None else int(n_active)
    pos = _dev_f32(pos, "pos", (n, 3))
    mass = _dev_f32(mass, "mass", (n,))
    P = as_problem(prob)
    if out is None:
        out = torch.empty((n_active, 3), dtype=torch.float32, device=pos.device)
    else:
        out = _out_f32(out, "out", (n_active, 3))
    _check(lib().sr_force_static(_ptr(pos), _ptr(mass), n, n_active, C.byref(P), _ptr(out), _stream(stream)),
           "sr_force_static")
    return out


def force_vjp(pos, mass, prob, g, n_active=None, ws=None, reuse_bins=False, out=None, stream=None):
    """Gradient of sum_i g_i . a_i with respect to the positions, [n, 3]."""
    n = int(pos.shape[0])
    n_active = n if n_active is None else int(n_active)
    pos = _dev_f32(pos, "pos", (n, 3))
    mass = _dev_f32(mass, "mass", (n,))
    g = _dev_f32(g, "g", (n_active, 3))
    P = as_problem(prob)
    if ws is None:
        if reuse_bins:
            raise ValueError("reuse_bins needs the binned workspace")
        ws = new_workspace(workspace_bytes(n, P), pos.device)
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    else:
        out = _out_f32(out, "out", (n, 3))
    _check(lib().sr_force_vjp(_ptr(pos), _ptr(mass), n, n_active, C.byref(P), _ptr(ws), ws.numel(),
                              REUSE_BINS if reuse_bins else 0, _ptr(g), _ptr(out), _stream(stream)),
           "sr_force_vjp")
    return out


def count_pairs(ws, n, prob, n_active=None, adjoint=False, stream=None) -> torch.Tensor:
    """Device int64 scalar: ordered pairs (active i, j) with 0 < s < r_s^2; with
    adjoint=True the pairs with at least one active end (those the adjoint evaluates)."""
    n_active = int(n) if n_active is None else int(n_active)
    out = torch.zeros(1, dtype=torch.int64, device=ws.device)
    P = as_problem(prob)
    _check(lib().sr_count_pairs(int(n), n_active, C.byref(P), _ptr(ws), ws.numel(),
                                COUNT_ADJOINT if adjoint else 0, _ptr(out), _stream(stream)),
           "sr_count_pairs")
    return out


def momentum(acc, mass, ws=None, stream=None) -> torch.Tensor:
    """float64 [3]: sum_i mass[i] * acc[i] over the rows of acc."""
    rows = int(acc.shape[0])
    acc = _dev_f32(acc, "acc", (rows, 3))
    mass = _dev_f32(mass[:rows], "mass", (rows,))
    if ws is None:
        ws = new_workspace(8 * (3 * (rows // 65536 + 2) + 3) + 1024, acc.device)
    out = torch.empty(3, dtype=torch.float64, device=acc.device)
    _check(lib().sr_momentum(_ptr(acc), _ptr(mass), rows, _ptr(ws), ws.numel(), _ptr(out),
                             _stream(stream)), "sr_momentum")
    return out


def ws_flags(ws, stream=None) -> int:
    v = C.c_uint32()
    _check(lib().sr_ws_flags(_ptr(ws), _stream(stream), C.byref(v)), "sr_ws_flags")
    return int(v.value)


class SRForce(torch.autograd.Function):
    """Differentiable short-range force: gradient with respect to positions only."""

    @staticmethod
    def forward(ctx, pos, mass, prob, n_active=None):
        n = int(pos.shape[0])
        n_act = n if n_active is None else int(n_active)
        ws = new_workspace(workspace_bytes(n, prob), pos.device)
        acc = force(pos, mass, prob, n_act, ws=ws)
        ctx.save_for_backward(pos, mass)
        ctx.ws = ws
        ctx.prob = prob
        ctx.n_active = n_act
        return acc

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        pos, mass = ctx.saved_tensors
        grad = force_vjp(pos, mass, ctx.prob, g.contiguous().float(), ctx.n_active, ws=ctx.ws,
                         reuse_bins=True)
        return grad, None, None, None


def sr_force(pos, mass, prob, n_active=None):
    return SRForce.apply(pos, mass, prob, n_active)


class BatchPlan:
    """A plan for B independent problems stored back to back."""

    def __init__(self, offsets, n_active, problems, tune_cache: Optional[str] = None):
        import numpy as np

        offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        n_active = np.ascontiguousarray(np.asarray(n_active, dtype=np.int64))
        B = len(problems)
        if offsets.shape != (B + 1,) or n_active.shape != (B,):
            raise ValueError("offsets must have B+1 entries and n_active B")
        arr = (Problem * B)(*[as_problem(p) for p in problems])
        self._plan = C.c_void_p()
        nb = C.c_size_t()
        cache = tune_cache.encode() if tune_cache else None
        _check(lib().sr_batch_plan_create(B, offsets.ctypes.data_as(C.c_void_p),
                                          n_active.ctypes.data_as(C.c_void_p), arr, cache,
                                          C.byref(self._plan), C.byref(nb)), "sr_batch_plan_create")
        self.B = B
        self.offsets = offsets
        self.n_active = n_active
        self.ws_bytes = int(nb.value)
        self.total_active = int(n_active.sum())

    def run(self, pos, mass, ws, acc, momentum=None, mode: str = "graph", stream=None,
            recapture: bool = False):
        """mode: "graph" (replay of the captured graph; with recapture=True new
        pointers capture again instead of raising SR_E_PLAN), "eager" or
        "per_subvolume"."""
        flags = {"graph": 0, "eager": BATCH_EAGER, "per_subvolume": BATCH_PER_SUBVOLUME}[mode]
        if recapture:
            flags |= BATCH_RECAPTURE
        n = int(self.offsets[-1])
        pos = _dev_f32(pos, "pos", (n, 3))
        mass = _dev_f32(mass, "mass", (n,))
        acc = _out_f32(acc, "acc", (self.total_active, 3))
        if momentum is not None and (momentum.dtype != torch.float64 or momentum.numel() != 3 * self.B):
            raise ValueError("momentum must be float64 [B, 3]")
        _check(lib().sr_batch_force(self._plan, _ptr(pos), _ptr(mass), _ptr(ws), ws.numel(), _ptr(acc),
                                    _ptr(momentum), flags, _stream(stream)), "sr_batch_force")

    def info(self) -> dict:
        import json

        buf = C.create_string_buffer(1024)
        _check(lib().sr_batch_plan_info(self._plan, buf, 1024), "sr_batch_plan_info")
        return json.loads(buf.value.decode())

    def close(self):
        if self._plan:
            lib().sr_batch_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_force(pos, mass, offsets, problems, n_active=None, mode="graph", momentum=False,
                tune_cache=None):
    import numpy as np

    offsets = np.asarray(offsets, dtype=np.int64)
    if n_active is None:
        n_active = np.diff(offsets)
    plan = BatchPlan(offsets, n_active, problems, tune_cache)
    ws = new_workspace(plan.ws_bytes, pos.device)
    acc = torch.empty((plan.total_active, 3), dtype=torch.float32, device=pos.device)
    mom = torch.empty((plan.B, 3), dtype=torch.float64, device=pos.device) if momentum else None
    plan.run(pos, mass, ws, acc, mom, mode)
    plan.close()
    return (acc, mom) if momentum else acc


class BlocksPlan:
    """Overlapping data blocks of one open domain (sr_blocks_*): partition,
    gather of the block inputs, reconcile of the block results.

    blocks: rectangles (gx0, gx1, gy0, gy1) in grid units tiling
    [0, ng[0]) x [0, ng[1]).  The workspace holds the partition between the
    calls, so it serves one partition at a time."""

    def __init__(self, domain, ng, blocks, n: int, n_active: Optional[int] = None,
                 capacity: int = 0):
        import numpy as np

        self.nb = len(blocks)
        arr = (Block * max(1, self.nb))(*[Block(*[int(v) for v in b]) for b in blocks])
        ngs = (C.c_int32 * 2)(int(ng[0]), int(ng[1]))
        self.n = int(n)
        self.n_active = self.n if n_active is None else int(n_active)
        self._plan = C.c_void_p()
        nbytes = C.c_size_t()
        _check(lib().sr_blocks_plan_create(C.byref(as_problem(domain)), ngs, self.nb, arr, self.n,
                                           self.n_active, int(capacity), C.byref(self._plan),
                                           C.byref(nbytes)), "sr_blocks_plan_create")
        self.ws_bytes = int(nbytes.value)
        self.blocks = [tuple(int(v) for v in b) for b in blocks]
        self.members = -1
        self.counts = np.zeros((self.nb, 2), np.int64)

    def problems(self) -> list:
        out = (Problem * self.nb)()
        _check(lib().sr_blocks_problems(self._plan, out), "sr_blocks_problems")
        return list(out)

    def partition(self, pos, ws, stream=None):
        """Assign particles to blocks; returns counts [nb, 2] (active, passive).
        Raises SRError(SR_E_WORKSPACE) with .needed set when the plan's
        capacity is too small."""
        import numpy as np

        pos = _dev_f32(pos, "pos", (self.n, 3))
        members = C.c_int64()
        counts = np.zeros((self.nb, 2), np.int64)
        code = lib().sr_blocks_partition(self._plan, _ptr(pos), _ptr(ws), ws.numel(), C.byref(members),
                                         counts.ctypes.data_as(C.c_void_p), _stream(stream))
        if code != SR_OK:
            err = SRError(code, "sr_blocks_partition")
            err.needed = int(members.value)
            raise err
        self.members = int(members.value)
        self.counts = counts
        return counts

    def gather(self, pos, mass, ws, g=None, bpos=None, bmass=None, want_src=True, stream=None):
        """Block inputs (bpos [members, 3], bmass [members], src [members] int32
        or None, and bg [n_active, 3] when g is given).  bpos and bmass may be
        given to be written in place."""
        pos = _dev_f32(pos, "pos", (self.n, 3))
        mass = _dev_f32(mass, "mass", (self.n,))
        dev = pos.device
        m = self.members
        if m < 0:
            raise SRError(4, "sr_blocks_gather")
        bpos = (_out_f32(bpos, "bpos", (m, 3)) if bpos is not None
                else torch.empty((m, 3), dtype=torch.float32, device=dev))
        bmass = (_out_f32(bmass, "bmass", (m,)) if bmass is not None
                 else torch.empty((m,), dtype=torch.float32, device=dev))
        src = torch.empty((m,), dtype=torch.int32, device=dev) if want_src else None
        bg = None
        if g is not None:
            g = _dev_f32(g, "g", (self.n_active, 3))
            bg = torch.empty((self.n_active, 3), dtype=torch.float32, device=dev)
        _check(lib().sr_blocks_gather(self._plan, _ptr(pos), _ptr(mass), _ptr(g), _ptr(ws), ws.numel(),
                                      _ptr(bpos), _ptr(bmass), _ptr(bg), _ptr(src), _stream(stream)),
               "sr_blocks_gather")
        return bpos, bmass, src, bg

    def reconcile(self, bacc, ws, out=None, stream=None):
        bacc = _dev_f32(bacc, "bacc", (self.n_active, 3))
        acc = out if out is not None else torch.empty((self.n_active, 3), dtype=torch.float32,
                                                      device=bacc.device)
        acc = _out_f32(acc, "acc", (self.n_active, 3))
        _check(lib().sr_blocks_reconcile(self._plan, _ptr(ws), ws.numel(), _ptr(bacc), _ptr(acc),
                                         _stream(stream)), "sr_blocks_reconcile")
        return acc

    def reconcile_grad(self, bgrad, ws, out=None, stream=None):
        bgrad = _dev_f32(bgrad, "bgrad", (self.members, 3))
        grad = out if out is not None else torch.empty((self.n, 3), dtype=torch.float32,
                                                       device=bgrad.device)
        grad = _out_f32(grad, "grad", (self.n, 3))
        _check(lib().sr_blocks_reconcile_grad(self._plan, _ptr(ws), ws.numel(), _ptr(bgrad), _ptr(grad),
                                              _stream(stream)), "sr_blocks_reconcile_grad")
        return grad

    def close(self):
        if self._plan:
            lib().sr_blocks_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CentresPlan:
    """Most-bound-particle centres of a halo catalogue (sr_centres_*): halo h
    holds particles [offsets[h], offsets[h+1])."""

    def __init__(self, offsets):
        import numpy as np

        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.n_halos = int(self.offsets.shape[0] - 1)
        self.n = int(self.offsets[-1]) if self.n_halos >= 0 else 0
        self._plan = C.c_void_p()
        nbytes = C.c_size_t()
        _check(lib().sr_centres_plan_create(self.n_halos, self.offsets.ctypes.data_as(C.c_void_p),
                                            C.byref(self._plan), C.byref(nbytes)), "sr_centres_plan_create")
        self.ws_bytes = int(nbytes.value)

    def run(self, pos, mass, eps, ws, phi=None, mbp=None, phi_min=None, stream=None):
        """Returns (phi [n], mbp [n_halos] int64, phi_min [n_halos])."""
        pos = _dev_f32(pos, "pos", (self.n, 3))
        mass = _dev_f32(mass, "mass", (self.n,))
        dev = pos.device
        phi = (_out_f32(phi, "phi", (self.n,)) if phi is not None
               else torch.empty((self.n,), dtype=torch.float32, device=dev))
        if mbp is None:
            mbp = torch.empty((self.n_halos,), dtype=torch.int64, device=dev)
        elif mbp.dtype != torch.int64 or tuple(mbp.shape) != (self.n_halos,) or not mbp.is_contiguous():
            raise ValueError("mbp must be a contiguous int64 [n_halos] tensor")
        phi_min = (_out_f32(phi_min, "phi_min", (self.n_halos,)) if phi_min is not None
                   else torch.empty((self.n_halos,), dtype=torch.float32, device=dev))
        _check(lib().sr_centres(self._plan, _ptr(pos), _ptr(mass), float(eps), _ptr(ws), ws.numel(),
                                _ptr(phi), _ptr(mbp), _ptr(phi_min), _stream(stream)), "sr_centres")
        return phi, mbp, phi_min

    def close(self):
        if self._plan:
            lib().sr_centres_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def halo_centres(pos, mass, offsets, eps):
    """phi, most-bound index and its phi per halo (one-shot plan and workspace)."""
    plan = CentresPlan(offsets)
    ws = new_workspace(plan.ws_bytes, pos.device)
    out = plan.run(pos, mass, eps, ws)
    plan.close()
    return out


class PkPlan:
    """Power spectrum of particles on an ng^3 periodic grid (sr_pk_*)."""

    def __init__(self, ng: int, box: float, n_bins: int, dn: float = 1.0, n_max: int = 0):
        self.ng, self.box, self.n_bins, self.dn = int(ng), float(box), int(n_bins), float(dn)
        self.n_max = int(n_max)
        self._plan = C.c_void_p()
        nbytes = C.c_size_t()
        _check(lib().sr_pk_plan_create(self.ng, self.box, self.n_bins, self.dn, self.n_max,
                                       C.byref(self._plan), C.byref(nbytes)), "sr_pk_plan_create")
        self.ws_bytes = int(nbytes.value)

    def deposit(self, pos, mass, ws, stream=None):
        """The CIC mass grid [ng, ng, ng] (a view into the workspace) and the total mass (device)."""
        n = int(pos.shape[0])
        pos = _dev_f32(pos, "pos", (n, 3))
        mass = _dev_f32(mass, "mass", (n,))
        _check(lib().sr_pk_deposit(self._plan, _ptr(pos), _ptr(mass), n, _ptr(ws), ws.numel(),
                                   _stream(stream)), "sr_pk_deposit")
        return self.grid(ws)

    def grid(self, ws):
        g = C.c_void_p()
        pitch = C.c_int32()
        mt = C.c_void_p()
        _check(lib().sr_pk_grid(self._plan, _ptr(ws), C.byref(g), C.byref(pitch), C.byref(mt)), "sr_pk_grid")
        base = ws.data_ptr()
        off, moff = (g.value or 0) - base, (mt.value or 0) - base
        ng, pitch = self.ng, int(pitch.value)
        full = ws[off: off + 4 * ng * ng * pitch].view(torch.float32).view(ng, ng, pitch)
        return full[:, :, :ng], ws[moff: moff + 8].view(torch.float64)

    def run(self, pos, mass, ws, stream=None):
        """(P per bin, mean |k| per bin, modes per bin) as device tensors."""
        n = int(pos.shape[0])
        pos = _dev_f32(pos, "pos", (n, 3))
        mass = _dev_f32(mass, "mass", (n,))
        dev = pos.device
        pk = torch.empty(self.n_bins, dtype=torch.float64, device=dev)
        km = torch.empty(self.n_bins, dtype=torch.float64, device=dev)
        modes = torch.empty(self.n_bins, dtype=torch.int64, device=dev)
        _check(lib().sr_power_spectrum(self._plan, _ptr(pos), _ptr(mass), n, _ptr(ws), ws.numel(), _ptr(pk),
                                       _ptr(km), _ptr(modes), _stream(stream)), "sr_power_spectrum")
        return pk, km, modes

    def close(self):
        if self._plan:
            lib().sr_pk_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def launch_config(waves_per_cu: int = 0, targets_per_lane: int = 0, occupancy: int = -1,
                  kernel: Optional[str] = None):
    """Set and return (waves_per_cu, targets_per_lane, occupancy) of the single-problem calls:
    both pair kernels, or only ``kernel`` ("force" or "vjp").

    0 keeps waves_per_cu / targets_per_lane, -1 keeps occupancy."""
    cur = (C.c_int * 3)()
    if kernel is None:
        _check(lib().sr_launch_config(int(waves_per_cu), int(targets_per_lane), int(occupancy), cur),
               "sr_launch_config")
    else:
        _check(lib().sr_launch_config_kernel(kernel.encode(), int(waves_per_cu), int(targets_per_lane),
                                             int(occupancy), cur), "sr_launch_config_kernel")
    return int(cur[0]), int(cur[1]), int(cur[2])


def sparse_group(group: int = -1) -> int:
    """Set and return the most targets per item of cells with fewer than 64 targets
    (8, 16, 32 or 64; -1 keeps the value)."""
    cur = C.c_int()
    _check(lib().sr_sparse_group(int(group), C.byref(cur)), "sr_sparse_group")
    return int(cur.value)


def tile_balance(min_ratio: float = -1.0) -> float:
    """Set and return the balance rule of the symmetric tiles: they run only if their work per
    wave of the persistent grid is at least min_ratio longest items (0: whenever the partial
    slots fit; -1 keeps the value)."""
    cur = C.c_double()
    _check(lib().sr_tile_balance(float(min_ratio), C.byref(cur)), "sr_tile_balance")
    return float(cur.value)


def tile_config(blocks_per_item: int = -1, window: int = -1, kernel: str = "force"):
    """Set and return (blocks_per_item, window) of the symmetric tiles of one pair kernel
    ("force" or "vjp"); blocks_per_item 0 switches them off, -1 keeps a value."""
    cur = (C.c_int * 2)()
    _check(lib().sr_tile_config(kernel.encode(), int(blocks_per_item), int(window), cur), "sr_tile_config")
    return int(cur[0]), int(cur[1])


def timing_enable(on: bool = True) -> None:
    _check(lib().sr_timing_enable(1 if on else 0), "sr_timing_enable")


def timing_read(kernel: str):
    ms = C.c_double()
    cnt = C.c_int64()
    _check(lib().sr_timing_read(kernel.encode(), C.byref(ms), C.byref(cnt)), "sr_timing_read")
    return float(ms.value), int(cnt.value)
