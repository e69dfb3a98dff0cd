"""Seeded generators: reproducibility, sizes, domains and the halo budget."""
import hashlib

import numpy as np

from paper_1411_3396_amd import filter_fit, synth


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_reproducible_and_seed_sensitive():
    a = synth.clustered_box(50000, 32.0, 30, 7)
    b = synth.clustered_box(50000, 32.0, 30, 7)
    c = synth.clustered_box(50000, 32.0, 30, 8)
    assert _h(a.pos) == _h(b.pos)
    assert _h(a.pos) != _h(c.pos)


def test_uniform_32k_shape_and_domain():
    w = synth.uniform_32k()
    assert w.pos.shape == (32768, 3) and w.pos.dtype == np.float32
    assert np.all(w.pos >= 0) and np.all(w.pos < 32.0)
    assert w.problem.periodic and w.n_active == w.n
    assert np.all(w.mass == 1.0)


def test_largest_remainder_sums_exactly():
    rng = np.random.default_rng(0)
    for _ in range(20):
        w = np.exp(rng.uniform(0, 10, 57))
        c = synth.largest_remainder(12345, w)
        assert c.sum() == 12345 and np.all(c >= 0)


def test_halo_share_and_budget():
    w = synth.clustered_box(100000, 40.0, 50, 1, halo_frac=0.4)
    assert w.notes["halo_budget"] == 40000
    assert w.notes["max_halo"] >= 40000 // 50


def test_slab_active_first_and_ghost_shell():
    w = synth.slab_with_ghosts(24, 3.0, 40, 2)
    act = w.pos[: w.n_active]
    gho = w.pos[w.n_active:]
    assert w.n == 30 ** 3
    assert np.all((act >= 0) & (act < 24))
    assert np.all(np.any((gho < 0) | (gho >= 24), axis=1))
    assert np.all((w.pos >= -3.0) & (w.pos < 27.0))
    assert not w.problem.periodic and w.problem.lo == (-3.0, -3.0, -3.0)


def test_subvolume_batch_layout():
    b = synth.subvolume_batch(n_sub=6, count_range=(1e3, 1e4))
    assert b.offsets[0] == 0 and b.offsets[-1] == b.pos.shape[0]
    for k in range(b.size):
        p = b.part(k)
        L = p.problem.len[0]
        assert np.all((p.pos >= 0) & (p.pos < L))
        assert abs(p.n / L ** 3 - 1.0) < 1e-3


def test_filter_coefficients_vanish_at_cutoff():
    for rs, eps in [(3.0, 0.05), (3.0, 0.02)]:
        c = filter_fit.load(rs, eps)
        s = rs * rs
        assert abs(np.polyval(c[::-1], s) - (s + eps * eps) ** -1.5) < 1e-15
        # the polynomial follows the Gaussian long-range kernel to within 1% of Newton
        r = np.linspace(0.05, rs, 500)
        err = np.abs(np.polyval(c[::-1], r * r) - filter_fit.long_range_kernel(r))
        assert np.all(err <= 0.01 * r ** -3)


def test_long_range_kernel_series_and_closed_form_agree():
    # the small-argument series and the closed form meet at x = 0.5 (r = 2 sigma x)
    r = np.array([2 * filter_fit.SIGMA * 0.5 * (1 - 1e-9), 2 * filter_fit.SIGMA * 0.5 * (1 + 1e-9)])
    v = filter_fit.long_range_kernel(r)
    assert abs(v[0] - v[1]) < 1e-9 * v[0]
    # limit at r -> 0: 1 / (6 sqrt(pi) sigma^3)
    v0 = filter_fit.long_range_kernel(np.array([1e-8]))[0]
    assert abs(v0 - 1.0 / (6 * np.sqrt(np.pi) * filter_fit.SIGMA ** 3)) < 1e-12
