"""The allocation-free forward (sr_force_static) against sr_force with a
caller workspace: the same kernels on a fixed device array, so the
accelerations must be bitwise equal, and within the forward tolerance of the
float64 oracle.  Two calls in a row, the second on a smaller input, so the
second call runs on the first call's leftover contents."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1411_3396_amd import _sr, synth
from gpu_helpers import DEV, FWD_TOL, announce, assert_force_close, oracle_force, to_dev

pytestmark = pytest.mark.gpu


def _static_via_abi(w):
    # straight through the C ABI: inputs and the output are the only buffers
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    out = torch.full((w.n_active, 3), float("nan"), dtype=torch.float32, device=DEV)
    P = _sr.as_problem(w.problem)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = _sr.lib().sr_force_static(C.c_void_p(pos.data_ptr()), C.c_void_p(mass.data_ptr()), w.n, w.n_active,
                                   C.byref(P), C.c_void_p(out.data_ptr()), stream)
    assert rc == 0, _sr.lib().sr_status_str(rc)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _with_workspace(w):
    acc = _sr.force(to_dev(w.pos), to_dev(w.mass), w.problem, w.n_active)
    torch.cuda.synchronize()
    return acc.cpu().numpy()


def test_static_forward_matches_workspace_forward_twice():
    big = synth.slab_with_ghosts(36, 3.0, 120, 5)  # open slab with ghosts, clustered
    big.problem = big.problem.with_leaf_depth(2)
    big.mass = np.random.default_rng(3).uniform(0.5, 2.0, big.n).astype(np.float32)
    small = synth.uniform_box(9000, 24.0, 8)  # periodic, equal masses, fewer cells
    for name, w in (("slab", big), ("uniform", small)):
        announce(f"static forward {name} n={w.n} n_active={w.n_active}")
        got = _static_via_abi(w)
        ref = _with_workspace(w)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), name
        assert_force_close(got, oracle_force(w), FWD_TOL, what=f"static {name}")


def test_static_forward_rejects_oversize():
    w = synth.uniform_box(2_000_000, 126.0, 1)
    P = _sr.as_problem(w.problem)
    assert _sr.workspace_bytes(w.n, w.problem) > (64 << 20)
    rc = _sr.lib().sr_force_static(C.c_void_p(0x10000), C.c_void_p(0x10000), w.n, w.n, C.byref(P),
                                   C.c_void_p(0x10000), None)
    assert rc == 5
