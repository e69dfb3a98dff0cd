"""Power-spectrum entry points on the CPU: exports and host validation."""
import ctypes as C

from paper_1411_3396_amd import _sr

FAKE = C.c_void_p(0x10000)  # never dereferenced: every case fails validation first


def _create(ng, box=100.0, n_bins=10, dn=1.0, n_max=1000):
    plan = C.c_void_p()
    nbytes = C.c_size_t()
    code = _sr.lib().sr_pk_plan_create(ng, box, n_bins, dn, n_max, C.byref(plan), C.byref(nbytes))
    return code, plan, nbytes.value


def test_plan_validation_and_sizes():
    assert _create(64)[0] == 0
    for bad in (dict(ng=63), dict(ng=0), dict(ng=2048), dict(ng=64, box=0.0), dict(ng=64, box=float("inf")),
                dict(ng=64, n_bins=0), dict(ng=64, n_bins=5000), dict(ng=64, dn=0.0),
                dict(ng=64, n_max=-1), dict(ng=64, n_max=1 << 31)):
        assert _create(**bad)[0] == 1, bad
    sizes = [_create(ng)[2] for ng in (16, 64, 256)]
    assert sizes == sorted(sizes) and all(s % 256 == 0 for s in sizes)
    # the grid, ng * ng * 2 (ng/2 + 1) floats, and the FFT's work buffer of
    # about the same size; the deposits add per-particle sort buffers
    assert sizes[2] >= 2 * 256 * 256 * 258 * 4
    # the cell deposit (ng not a multiple of 8) keeps a cell-start table of ng^3 + 1
    assert _create(250)[2] >= 2 * 250 * 250 * 252 * 4 + 250 ** 3 * 4
    assert _create(64, n_max=100000)[2] > _create(64, n_max=1000)[2]


def test_run_validation_before_device():
    code, plan, nbytes = _create(32)
    L = _sr.lib()
    assert L.sr_pk_deposit(plan, FAKE, FAKE, 10, FAKE, nbytes - 1, None) == 2
    assert L.sr_pk_deposit(plan, FAKE, FAKE, -1, FAKE, nbytes, None) == 1
    assert L.sr_pk_deposit(plan, FAKE, FAKE, 1001, FAKE, nbytes, None) == 1  # above n_max
    assert L.sr_pk_deposit(plan, None, FAKE, 10, FAKE, nbytes, None) == 1
    assert L.sr_power_spectrum(plan, FAKE, FAKE, 0, FAKE, nbytes, FAKE, None, None, None) == 1
    assert L.sr_power_spectrum(plan, FAKE, FAKE, 10, FAKE, nbytes, None, None, None, None) == 1
    assert L.sr_power_spectrum(plan, FAKE, FAKE, 10, C.c_void_p(0x10004), nbytes, FAKE, None, None, None) == 2
    assert L.sr_power_spectrum(None, FAKE, FAKE, 10, FAKE, nbytes, FAKE, None, None, None) == 4
    assert L.sr_pk_plan_destroy(plan) == 0
