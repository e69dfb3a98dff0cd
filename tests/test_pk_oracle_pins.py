"""Pins of the power-spectrum oracle (paper Sec. 4.1: cloud-in-cell deposit,
DFT, |delta(k)|^2 binned in |k|, divided by the CIC window) against hand
weights, an analytic plane wave, shot noise and invariances."""
import itertools
import math

import numpy as np
import pytest

from oracle import pk


def test_cic_weights_by_hand():
    ng, box = 8, 8.0
    rho = pk.cic_deposit([[1.25, 2.5, 3.0]], [2.0], ng, box)
    want = np.zeros((ng, ng, ng))
    for ix, wx in ((1, 0.75), (2, 0.25)):
        for iy, wy in ((2, 0.5), (3, 0.5)):
            want[ix, iy, 3] += 2.0 * wx * wy
    np.testing.assert_allclose(rho, want, atol=1e-15)
    # wrap across the periodic face, and a particle on a grid point
    rho = pk.cic_deposit([[7.75, 0.0, 0.0]], [1.0], ng, box)
    assert rho[7, 0, 0] == pytest.approx(0.25) and rho[0, 0, 0] == pytest.approx(0.75)
    assert np.count_nonzero(rho) == 2
    rho = pk.cic_deposit([[3.0, 4.0, 5.0]], [1.0], ng, 16.0)  # h = 2: point (1.5, 2, 2.5)
    assert np.count_nonzero(rho) == 4 and rho.sum() == pytest.approx(1.0)


def test_mass_is_conserved():
    rng = np.random.default_rng(1)
    pos = rng.random((5000, 3)) * 10.0 - 3.0  # outside [0, box) too: periodic
    mass = rng.uniform(0.5, 2.0, 5000)
    rho = pk.cic_deposit(pos, mass, 16, 10.0)
    assert rho.sum() == pytest.approx(mass.sum(), rel=1e-12)


def shell_count(ng, lo, hi):
    half = ng // 2
    r = range(-half + 1, half + 1)
    return sum(1 for n in itertools.product(r, r, r) if lo <= math.sqrt(sum(v * v for v in n)) < hi)


def test_plane_wave_amplitude_window_and_counts():
    ng, box, amp = 16, 50.0, 0.3
    x = np.arange(ng)
    rho = 1.0 + amp * np.cos(2 * np.pi * 3 * x / ng)[:, None, None] * np.ones((1, ng, ng))
    p, k, cnt = pk.power_spectrum(rho, box, n_bins=12)
    for b in range(12):
        assert cnt[b] == shell_count(ng, b if b > 0 else 1e-9, b + 1)
    w = (math.sin(math.pi * 3 / ng) / (math.pi * 3 / ng)) ** 2
    per_mode = amp ** 2 * box ** 3 / 4.0 / w ** 2
    assert p[3] == pytest.approx(2 * per_mode / cnt[3], rel=1e-10)
    assert np.all(np.abs(np.delete(p, 3)) < 1e-20 * per_mode)
    assert k[3] > 2 * np.pi / box * 3 and k[3] < 2 * np.pi / box * 4


def test_shot_noise_of_random_particles():
    # uniform random particles: at low k the deconvolved spectrum is the shot
    # noise box^3 / N (the CIC aliasing correction is below 2% for |n| <= 3 of 32)
    rng = np.random.default_rng(2)
    n, ng, box = 200000, 32, 100.0
    rho = pk.cic_deposit(rng.random((n, 3)) * box, np.ones(n), ng, box)
    p, _, cnt = pk.power_spectrum(rho, box, n_bins=4)
    shot = box ** 3 / n
    for b in (1, 2, 3):
        sigma = shot / math.sqrt(cnt[b] / 2)
        assert abs(p[b] - shot) < 5 * sigma + 0.02 * shot, (b, p[b], shot)


def test_translation_by_a_cell_and_mass_scale():
    rng = np.random.default_rng(3)
    pos = rng.random((3000, 3)) * 20.0
    ng, box = 16, 20.0
    a = pk.power_spectrum(pk.cic_deposit(pos, np.ones(3000), ng, box), box, 10)[0]
    b = pk.power_spectrum(pk.cic_deposit(pos + box / ng, np.ones(3000), ng, box), box, 10)[0]
    c = pk.power_spectrum(pk.cic_deposit(pos, 7.0 * np.ones(3000), ng, box), box, 10)[0]
    np.testing.assert_allclose(b, a, rtol=1e-9)
    np.testing.assert_allclose(c, a, rtol=1e-9)  # delta does not depend on the mass unit
