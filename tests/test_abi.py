"""The C ABI on the CPU: the library loads, exports what sr.h declares, and
rejects bad arguments on the host before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1411_3396_amd import _sr, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sr.h")
FAKE = C.c_void_p(0x10000)  # never dereferenced: every case fails validation first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sr_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function():
    L = _sr.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_sr.EXPORTS)
    assert L.sr_abi_version() == 6 == _sr.ABI_VERSION
    assert L.sr_status_str(0) == b"ok"


def header_defines(prefix):
    text = open(HEADER).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(" + prefix + r"\w+)\s+(\d+)u?", text)}


def test_flag_and_option_constants_match_the_header():
    # the binding decodes sr_ws_flags and passes flags with the header's values;
    # a renumbered bit would silently change their meaning
    flags = header_defines("SR_FLAG_")
    assert flags == {"SR_FLAG_NONFINITE": _sr.FLAG_NONFINITE, "SR_FLAG_OUT_OF_DOMAIN": _sr.FLAG_OUT_OF_DOMAIN,
                     "SR_FLAG_NOT_BINNED": _sr.FLAG_NOT_BINNED, "SR_FLAG_QUEUE": _sr.FLAG_QUEUE}
    assert len(set(flags.values())) == len(flags) and all(v & (v - 1) == 0 for v in flags.values())
    opts = header_defines("SR_(?:REUSE|BATCH|COUNT)_")
    assert opts == {"SR_REUSE_BINS": _sr.REUSE_BINS, "SR_BATCH_PER_SUBVOLUME": _sr.BATCH_PER_SUBVOLUME,
                    "SR_BATCH_EAGER": _sr.BATCH_EAGER, "SR_BATCH_RECAPTURE": _sr.BATCH_RECAPTURE,
                    "SR_COUNT_ADJOINT": _sr.COUNT_ADJOINT}
    assert header_defines("SR_ABI_")["SR_ABI_VERSION"] == _sr.ABI_VERSION


def prob(length=32.0, periodic=True, r_s=3.0, eps=0.05, lo=(0, 0, 0)):
    return _sr.as_problem(synth.Problem.make(lo, (length,) * 3, periodic, r_s, eps,
                                             synth.filter_poly(3.0, 0.05)))


def test_grid_matches_binning_rule():
    for L_, per in [(32.0, True), (9.0, True), (326.0, False), (2.0, False), (128.0, True),
                    (21.544347, True)]:
        p = synth.Problem.make((0, 0, 0) if per else (-3, -3, -3), (L_,) * 3, per, 3.0, 0.05,
                               (0,) * 6)
        assert tuple(_sr.grid(p)) == tuple(oracle.grid(p))


def test_workspace_bytes_grows_with_n():
    p = prob()
    sizes = [_sr.workspace_bytes(n, p) for n in (0, 1, 1000, 100000)]
    assert all(b > 0 and b % 256 == 0 for b in sizes)
    assert sizes == sorted(sizes)


def _force(n=100, n_active=100, p=None, ws=FAKE, ws_bytes=None, flags=0, pos=FAKE, mass=FAKE,
           acc=FAKE):
    p = p if p is not None else prob()
    if ws_bytes is None:
        ws_bytes = _sr.workspace_bytes(max(n, 0), prob()) + (1 << 20)
    return _sr.lib().sr_force(pos, mass, n, n_active, C.byref(p), ws, ws_bytes, flags, acc, None)


def test_host_validation_codes():
    E_ARG, E_WS = 1, 2
    assert _force(n=-1) == E_ARG
    assert _force(n=10, n_active=11) == E_ARG
    assert _force(n=10, n_active=-1) == E_ARG
    assert _force(pos=None) == E_ARG
    assert _force(mass=None) == E_ARG
    assert _force(acc=None) == E_ARG
    assert _force(flags=8) == E_ARG
    assert _force(p=prob(length=8.9)) == E_ARG          # periodic box below 3 r_s
    assert _force(p=prob(r_s=0.0)) == E_ARG
    assert _force(p=prob(r_s=-1.0)) == E_ARG
    assert _force(p=prob(eps=-0.1)) == E_ARG
    assert _force(p=prob(lo=(1, 0, 0))) == E_ARG        # periodic needs lo = 0
    bad = prob()
    bad.poly[3] = float("nan")
    assert _force(p=bad) == E_ARG
    bad = prob()
    bad.len[1] = float("inf")
    assert _force(p=bad) == E_ARG
    assert _force(ws=None) == E_WS
    assert _force(ws=C.c_void_p(0x10010)) == E_WS       # not 256-byte aligned
    assert _force(ws_bytes=1024) == E_WS


def test_leaf_depth_validation_and_key_width():
    E_ARG, E_UNSUP = 1, 5
    L = _sr.lib()
    nc = (C.c_int32 * 3)()
    nbytes = C.c_size_t()
    for d in (-1, 5, 99):
        p = prob()
        p.leaf_depth = d
        assert L.sr_grid(C.byref(p), nc) == E_ARG
        assert _force(p=p) == E_ARG
    for d in (0, 1, 2, 3, 4):  # 0 means 1
        p = prob()
        p.leaf_depth = d
        assert L.sr_workspace_bytes(1000, C.byref(p), C.byref(nbytes)) == 0
    # ncell * 2^(3D + 1) must fit the 31-bit key: 108^3 cells take D = 3, not D = 4
    big = _sr.as_problem(synth.Problem.make((-3, -3, -3), (326.0,) * 3, False, 3.0, 0.05, (0,) * 6))
    for d, want in ((3, 0), (4, E_UNSUP)):
        big.leaf_depth = d
        assert L.sr_workspace_bytes(1000, C.byref(big), C.byref(nbytes)) == want, d
    # a batch keys on its deepest subvolume: each fits alone, not together
    offs = np.array([0, 10, 20], np.int64)
    nact = np.array([10, 10], np.int64)
    small = prob()
    small.leaf_depth = 4
    big.leaf_depth = 1
    assert L.sr_workspace_bytes(10, C.byref(small), C.byref(nbytes)) == 0
    assert L.sr_workspace_bytes(10, C.byref(big), C.byref(nbytes)) == 0
    probs = (_sr.Problem * 2)(small, big)
    plan = C.c_void_p()
    rc = L.sr_batch_plan_create(2, offs.ctypes.data_as(C.c_void_p), nact.ctypes.data_as(C.c_void_p), probs,
                                None, C.byref(plan), C.byref(nbytes))
    assert rc == E_UNSUP and not plan.value


def test_empty_problem_is_a_noop_without_device():
    p = prob()
    assert _force(n=0, n_active=0, pos=None, mass=None, acc=None) == 0
    L = _sr.lib()
    assert L.sr_bin(None, None, 0, 0, C.byref(p), FAKE, _sr.workspace_bytes(0, p), None) == 0
    assert L.sr_force_vjp(None, None, 0, 0, C.byref(p), FAKE, _sr.workspace_bytes(0, p), 0, None,
                          None, None) == 0


def test_vjp_and_bin_validation():
    L = _sr.lib()
    p = prob()
    nb = _sr.workspace_bytes(100, p)
    assert L.sr_force_vjp(FAKE, FAKE, 100, 100, C.byref(p), FAKE, nb, 0, None, FAKE, None) == 1
    assert L.sr_force_vjp(FAKE, FAKE, 100, 100, C.byref(p), FAKE, nb, 0, FAKE, None, None) == 1
    assert L.sr_bin(FAKE, FAKE, 100, 101, C.byref(p), FAKE, nb, None) == 1
    assert L.sr_bin(FAKE, FAKE, 100, 100, C.byref(p), FAKE, nb - 256, None) == 2
    assert L.sr_momentum(FAKE, FAKE, -1, FAKE, 4096, FAKE, None) == 1
    assert L.sr_count_pairs(100, 100, C.byref(p), FAKE, nb, 0, None, None) == 1
    assert L.sr_count_pairs(100, 100, C.byref(p), FAKE, nb, 2, FAKE, None) == 1  # unknown flag


def test_launch_config_validation():
    L = _sr.lib()
    cur = (C.c_int * 3)()
    assert L.sr_launch_config(65, 0, -1, cur) == 1
    assert L.sr_launch_config(0, 3, -1, cur) == 1
    assert L.sr_launch_config(0, 0, 7, cur) == 1
    saved = {k: _sr.launch_config(kernel=k) for k in ("force", "vjp")}
    assert saved["force"] == (32, 1, 6) and saved["vjp"] == (24, 2, 0)  # defaults differ per kernel
    assert _sr.launch_config(16, 2, 6) == (16, 2, 6)
    assert _sr.launch_config() == (16, 2, 6) and _sr.launch_config(kernel="vjp") == (16, 2, 6)
    assert _sr.launch_config(8, 1, 0, kernel="vjp") == (8, 1, 0)
    assert _sr.launch_config() == (16, 2, 6)  # the forward kernel's values are untouched
    assert L.sr_launch_config_kernel(b"bogus", 0, 0, -1, cur) == 1
    assert L.sr_launch_config_kernel(b"vjp", 0, 0, 7, cur) == 1
    for k, v in saved.items():
        _sr.launch_config(*v, kernel=k)
    assert {k: _sr.launch_config(kernel=k) for k in ("force", "vjp")} == saved


def test_batch_plan_validation_and_layout():
    L = _sr.lib()
    probs = [prob(), prob(length=40.0)]
    arr = (_sr.Problem * 2)(*probs)
    plan = C.c_void_p()
    nb = C.c_size_t()
    off = np.array([0, 100, 250], np.int64)
    act = np.array([100, 120], np.int64)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    assert L.sr_batch_plan_create(2, ptr(np.array([1, 100, 250], np.int64)), ptr(act), arr, None,
                                  C.byref(plan), C.byref(nb)) == 1
    assert L.sr_batch_plan_create(2, ptr(off), ptr(np.array([101, 10], np.int64)), arr, None,
                                  C.byref(plan), C.byref(nb)) == 1
    assert L.sr_batch_plan_create(0, ptr(off), ptr(act), arr, None, C.byref(plan), C.byref(nb)) == 1
    bad = (_sr.Problem * 2)(prob(), prob(length=5.0))
    assert L.sr_batch_plan_create(2, ptr(off), ptr(act), bad, None, C.byref(plan), C.byref(nb)) == 1
    assert L.sr_batch_force(None, FAKE, FAKE, FAKE, 1 << 20, FAKE, None, 0, None) == 4


def test_static_forward_validation_before_the_device():
    # the allocation-free forward rejects, on the host, inputs whose workspace
    # would not fit its fixed array, and bad arguments, without a device call
    E_ARG, E_UNSUP = 1, 5
    L = _sr.lib()
    p = prob()
    limit = header_defines("SR_STATIC_")  # "((size_t)64 << 20)" is not a plain number
    assert limit == {}
    text = open(HEADER).read()
    m = re.search(r"#define\s+SR_STATIC_WORKSPACE_BYTES\s+\(\(size_t\)(\d+)\s*<<\s*(\d+)\)", text)
    cap = int(m.group(1)) << int(m.group(2))
    fits = max(n for n in range(0, 2_000_000, 1000) if _sr.workspace_bytes(n, p) <= cap)
    assert 100_000 < fits < 2_000_000
    big = fits + 1000
    assert _sr.workspace_bytes(big, p) > cap
    assert L.sr_force_static(FAKE, FAKE, big, big, C.byref(p), FAKE, None) == E_UNSUP
    assert L.sr_force_static(FAKE, FAKE, 100, 101, C.byref(p), FAKE, None) == E_ARG
    assert L.sr_force_static(None, FAKE, 100, 100, C.byref(p), FAKE, None) == E_ARG
    assert L.sr_force_static(FAKE, FAKE, 100, 100, C.byref(p), None, None) == E_ARG
    assert L.sr_force_static(FAKE, FAKE, 100, 100, None, FAKE, None) == E_ARG
    assert L.sr_force_static(None, None, 0, 0, C.byref(p), None, None) == 0


def test_tile_config_validation():
    L = _sr.lib()
    cur = (C.c_int * 2)()
    saved = {k: _sr.tile_config(kernel=k) for k in ("force", "vjp")}
    assert saved["force"] == (16, 256) and saved["vjp"] == (16, 256)
    assert L.sr_tile_config(b"bogus", 4, 256, cur) == 1
    assert L.sr_tile_config(None, 4, 256, cur) == 1
    assert L.sr_tile_config(b"force", 257, -1, cur) == 1
    assert L.sr_tile_config(b"force", -2, -1, cur) == 1
    assert L.sr_tile_config(b"force", -1, 384, cur) == 1
    assert _sr.tile_config(4, 256, kernel="force") == (4, 256)
    assert _sr.tile_config(kernel="vjp") == saved["vjp"]  # the other kernel is untouched
    assert _sr.tile_config(0, kernel="force") == (0, 256)  # 0 switches the tiles off
    for k, v in saved.items():
        _sr.tile_config(*v, kernel=k)
    assert {k: _sr.tile_config(kernel=k) for k in ("force", "vjp")} == saved


def test_tile_balance_validation():
    L = _sr.lib()
    cur = C.c_double()
    saved = _sr.tile_balance()
    assert saved == 1.0
    for bad in (-2.0, -0.5, float("nan"), float("inf")):
        assert L.sr_tile_balance(bad, C.byref(cur)) == 1, bad
    assert _sr.tile_balance() == saved  # rejected values change nothing
    assert _sr.tile_balance(0.0) == 0.0
    assert _sr.tile_balance(2.5) == 2.5
    assert L.sr_tile_balance(-1.0, None) == 0
    _sr.tile_balance(saved)
    assert _sr.tile_balance() == saved


def test_sparse_group_validation():
    L = _sr.lib()
    cur = C.c_int()
    saved = _sr.sparse_group()
    assert saved == 16
    for bad in (0, 4, 12, 48, 128, -2):
        assert L.sr_sparse_group(bad, C.byref(cur)) == 1, bad
    assert _sr.sparse_group() == saved
    for g in (8, 32, 64, 16):
        assert _sr.sparse_group(g) == g
    assert L.sr_sparse_group(-1, None) == 0
    _sr.sparse_group(saved)
