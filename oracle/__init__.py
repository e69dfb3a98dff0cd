"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
use this module.  It reads a problem from any object with the attributes
``lo, len, periodic, r_s, eps, poly`` and widens float32 inputs to float64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("SR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

NONFINITE = 1
OUT_OF_DOMAIN = 2

_p = C.c_void_p
_i64 = C.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.argtypes = [C.c_int]
        L.oracle_set_num_threads.restype = None
        L.oracle_grid.argtypes = [_p, C.c_float, C.c_int, _p]
        L.oracle_bin_reference.argtypes = [_p, _i64, _i64, _p, _p, C.c_int, C.c_float, C.c_int, _p, _p,
                                           _p, _p, _p]
        L.oracle_force.argtypes = [_p, _p, _i64, _i64, _p, _p, C.c_int, C.c_double, C.c_double, _p,
                                   _p, _i64, _p, _p]
        L.oracle_force_brute.argtypes = [_p, _p, _i64, _i64, _p, _p, C.c_int, C.c_double,
                                         C.c_double, _p, _p]
        L.oracle_vjp.argtypes = [_p, _p, _i64, _i64, _p, _p, C.c_int, C.c_double, C.c_double, _p,
                                 _p, _p, _i64, _p]
        L.oracle_vjp_brute.argtypes = [_p, _p, _i64, _i64, _p, _p, C.c_int, C.c_double, C.c_double,
                                       _p, _p, _p]
        L.oracle_halo_potential.argtypes = [_p, _p, _i64, _p, _i64, C.c_double, _p, _i64, _p]
        for fn in ("oracle_grid", "oracle_bin_reference", "oracle_force", "oracle_force_brute",
                   "oracle_vjp", "oracle_vjp_brute", "oracle_halo_potential"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the calling thread's later oracle calls (for callers that
    run many small calls from a thread pool; ctypes releases the GIL)."""
    lib().oracle_set_num_threads(int(n))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _d3(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))


def _args(prob):
    lo = _d3([float(np.float32(v)) for v in prob.lo])
    ln = _d3([float(np.float32(v)) for v in prob.len])
    poly = np.ascontiguousarray(np.asarray([float(np.float32(c)) for c in prob.poly], np.float64))
    return lo, ln, int(bool(prob.periodic)), float(np.float32(prob.r_s)), \
        float(np.float32(prob.eps)), poly


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"{what} rejected its arguments (code {rc})")


def grid(prob) -> np.ndarray:
    nc = np.zeros(3, np.int32)
    ln = np.ascontiguousarray(np.asarray(prob.len, np.float32))
    _check(lib().oracle_grid(_ptr(ln), C.c_float(prob.r_s), int(bool(prob.periodic)), _ptr(nc)),
           "oracle_grid")
    return nc


def bin_reference(pos32: np.ndarray, prob, n_active=None) -> dict:
    """Float32 binning rule: cell ids, cell starts, permutation, offsets; each
    cell ordered by the leaves of an octree of prob.leaf_depth levels (1 when
    absent or 0)."""
    pos32 = np.ascontiguousarray(pos32, dtype=np.float32).reshape(-1, 3)
    n = pos32.shape[0]
    n_active = n if n_active is None else int(n_active)
    nc = grid(prob)
    ncell = int(np.prod(nc.astype(np.int64)))
    cell_of = np.zeros(n, np.int32)
    start = np.zeros(ncell + 1, np.int32)
    perm = np.zeros(n, np.int32)
    off = np.zeros((n, 3), np.float32)
    flags = np.zeros(1, np.uint32)
    lo = np.ascontiguousarray(np.asarray(prob.lo, np.float32))
    ln = np.ascontiguousarray(np.asarray(prob.len, np.float32))
    depth = int(getattr(prob, "leaf_depth", 1)) or 1
    rc = lib().oracle_bin_reference(_ptr(pos32), n, n_active, _ptr(lo), _ptr(ln), int(bool(prob.periodic)),
                                    C.c_float(prob.r_s), depth, _ptr(cell_of), _ptr(start), _ptr(perm),
                                    _ptr(off), _ptr(flags))
    _check(rc, "oracle_bin_reference")
    return {"nc": nc, "cell_of": cell_of, "cell_start": start, "perm": perm, "off": off,
            "flags": int(flags[0])}


def force(pos, mass, n_active, prob, targets=None):
    """float64 accelerations of the target particles and the useful-pair count."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
    n = pos.shape[0]
    if targets is None:
        tptr, nt = None, int(n_active)
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        tptr, nt = _ptr(targets), targets.shape[0]
    acc = np.zeros((nt, 3), np.float64)
    pairs = np.zeros(1, np.int64)
    lo, ln, per, rs, eps, poly = _args(prob)
    rc = lib().oracle_force(_ptr(pos), _ptr(mass), n, int(n_active), _ptr(lo), _ptr(ln), per, rs,
                            eps, _ptr(poly), tptr, nt, _ptr(acc), _ptr(pairs))
    _check(rc, "oracle_force")
    return acc, int(pairs[0])


def force_brute(pos, mass, n_active, prob):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
    acc = np.zeros((int(n_active), 3), np.float64)
    lo, ln, per, rs, eps, poly = _args(prob)
    rc = lib().oracle_force_brute(_ptr(pos), _ptr(mass), pos.shape[0], int(n_active), _ptr(lo),
                                  _ptr(ln), per, rs, eps, _ptr(poly), _ptr(acc))
    _check(rc, "oracle_force_brute")
    return acc


def vjp(pos, mass, n_active, prob, g, targets=None):
    """float64 gradient of sum_i g_i . a_i with respect to the positions."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    if g.shape[0] != int(n_active):
        raise ValueError("g must have n_active rows")
    if targets is None:
        tptr, nt = None, n
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        tptr, nt = _ptr(targets), targets.shape[0]
    out = np.zeros((nt, 3), np.float64)
    lo, ln, per, rs, eps, poly = _args(prob)
    rc = lib().oracle_vjp(_ptr(pos), _ptr(mass), n, int(n_active), _ptr(lo), _ptr(ln), per, rs, eps,
                          _ptr(poly), _ptr(g), tptr, nt, _ptr(out))
    _check(rc, "oracle_vjp")
    return out


def vjp_brute(pos, mass, n_active, prob, g):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((pos.shape[0], 3), np.float64)
    lo, ln, per, rs, eps, poly = _args(prob)
    rc = lib().oracle_vjp_brute(_ptr(pos), _ptr(mass), pos.shape[0], int(n_active), _ptr(lo),
                                _ptr(ln), per, rs, eps, _ptr(poly), _ptr(g), _ptr(out))
    _check(rc, "oracle_vjp_brute")
    return out


def rms_rel(x, ref) -> float:
    """sqrt(sum |x - ref|^2 / sum |ref|^2) over rows."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = float(np.sum(ref * ref))
    num = float(np.sum((x - ref) ** 2))
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def halo_potential(pos, mass, offsets, eps, targets=None):
    """float64 potential of each target from the other particles of its halo
    (halo h holds particles [offsets[h], offsets[h+1]))."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = pos.shape[0]
    if targets is None:
        tptr, nt = None, n
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        tptr, nt = _ptr(targets), targets.shape[0]
    phi = np.zeros(nt, np.float64)
    rc = lib().oracle_halo_potential(_ptr(pos), _ptr(mass), n, _ptr(offsets), offsets.shape[0] - 1,
                                     float(np.float32(eps)), tptr, nt, _ptr(phi))
    _check(rc, "oracle_halo_potential")
    return phi


def most_bound(phi, offsets):
    """Per halo: index of the smallest phi (the first on ties) and that phi;
    -1 and 0 for an empty halo."""
    offsets = np.asarray(offsets, dtype=np.int64)
    H = offsets.shape[0] - 1
    idx = np.full(H, -1, np.int64)
    val = np.zeros(H, np.float64)
    for h in range(H):
        a, b = offsets[h], offsets[h + 1]
        if b > a:
            k = int(np.argmin(phi[a:b]))
            idx[h] = a + k
            val[h] = phi[a + k]
    return idx, val
