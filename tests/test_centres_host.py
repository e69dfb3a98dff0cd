"""Centre-finder entry points on the CPU: exports and host validation (no
device work)."""
import ctypes as C

import numpy as np

from paper_1411_3396_amd import _sr

FAKE = C.c_void_p(0x10000)  # never dereferenced: every case fails validation first


def _create(offsets, H=None):
    off = np.ascontiguousarray(np.asarray(offsets, np.int64))
    plan = C.c_void_p()
    nbytes = C.c_size_t()
    code = _sr.lib().sr_centres_plan_create(len(off) - 1 if H is None else H, off.ctypes.data_as(C.c_void_p),
                                            C.byref(plan), C.byref(nbytes))
    return code, plan, nbytes.value


def test_plan_validation():
    assert _create([0, 3])[0] == 0
    assert _create([1, 3])[0] == 1  # must start at 0
    assert _create([0, 5, 3])[0] == 1  # decreasing
    assert _create([0], H=0)[0] == 1  # no halos
    assert _create([0, 1 << 31])[0] == 5  # more particles than 32-bit indices
    code, plan, nbytes = _create([0, 0, 1, 65, 65, 1000])
    assert code == 0 and nbytes % 256 == 0 and nbytes > 0
    assert _sr.lib().sr_centres_plan_destroy(plan) == 0


def test_run_validation_before_device():
    code, plan, nbytes = _create([0, 10, 300])
    L = _sr.lib()
    run = lambda eps, ws=FAKE, wsb=nbytes, phi=FAKE, mbp=FAKE: L.sr_centres(  # noqa: E731
        plan, FAKE, FAKE, eps, ws, wsb, phi, mbp, None, None)
    assert run(-1.0) == 1
    assert run(float("nan")) == 1
    assert run(0.02, mbp=None) == 1
    assert run(0.02, phi=None) == 1
    assert run(0.02, wsb=nbytes - 1) == 2
    assert run(0.02, ws=C.c_void_p(0x10004)) == 2  # misaligned
    assert L.sr_centres(None, FAKE, FAKE, 0.02, FAKE, nbytes, FAKE, FAKE, None, None) == 4
    assert L.sr_centres_plan_destroy(plan) == 0


def test_workspace_grows_with_items():
    a = _create([0, 100])[2]
    b = _create(np.arange(0, 100001, 100))[2]
    assert 0 < a < b
