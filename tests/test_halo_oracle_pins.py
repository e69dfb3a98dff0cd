"""Pins of the centre-finder oracle (paper Sec. 2.2: the halo centre is the
most bound particle, the one at the potential minimum) against facts that do
not come from the oracle: closed forms, scipy's pairwise distances, the
symmetry of a lattice, the virial pair sum, the Plummer sphere's central
potential, and the independence of halos."""
import math

import numpy as np
import pytest
from scipy.spatial.distance import pdist, squareform

import oracle
from paper_1411_3396_amd import synth


def test_two_and_three_bodies():
    pos = np.array([[0, 0, 0], [3, 4, 0]], float)
    phi = oracle.halo_potential(pos, [2.0, 5.0], [0, 2], 0.0)
    assert phi[0] == pytest.approx(-5.0 / 5.0) and phi[1] == pytest.approx(-2.0 / 5.0)
    phi = oracle.halo_potential(pos, [2.0, 5.0], [0, 2], 1.0)
    assert phi[0] == pytest.approx(-5.0 / math.sqrt(26.0))
    pos = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0]], float)
    phi = oracle.halo_potential(pos, [1.0, 1.0, 1.0], [0, 3], 0.0)
    np.testing.assert_allclose(phi, [-(1 + 0.5), -(1 + 1 / math.sqrt(5)), -(0.5 + 1 / math.sqrt(5))])


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_matches_scipy_pairwise_distances(eps):
    rng = np.random.default_rng(3)
    counts = [0, 1, 2, 17, 64, 129, 300]
    pos = rng.normal(size=(sum(counts), 3)) * 2.0 + 100.0
    mass = rng.uniform(0.5, 2.0, sum(counts))
    off = np.concatenate([[0], np.cumsum(counts)])
    phi = oracle.halo_potential(pos, mass, off, eps)
    for h in range(len(counts)):
        a, b = off[h], off[h + 1]
        if b - a < 2:
            assert np.all(phi[a:b] == 0.0)
            continue
        r2 = squareform(pdist(pos[a:b], "sqeuclidean"))
        with np.errstate(divide="ignore"):
            e32 = float(np.float32(eps))  # the softening is a float32 parameter
            inv = 1.0 / np.sqrt(r2 + e32 * e32)
        np.fill_diagonal(inv, 0.0)
        np.testing.assert_allclose(phi[a:b], -(inv @ mass[a:b]), rtol=1e-12)


def test_lattice_centre_is_most_bound():
    g = np.arange(5, dtype=float)
    pos = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T
    perm = np.random.default_rng(0).permutation(len(pos))
    pos = pos[perm]
    phi = oracle.halo_potential(pos, np.ones(len(pos)), [0, len(pos)], 0.0)
    idx, val = oracle.most_bound(phi, [0, len(pos)])
    assert np.array_equal(pos[idx[0]], [2, 2, 2])
    # the eight corners are equivalent under the cube's symmetries
    corners = np.all((pos == 0) | (pos == 4), axis=1)
    assert np.ptp(phi[corners]) < 1e-12 and val[0] == phi.min()


def test_virial_pair_sum_and_translation():
    rng = np.random.default_rng(5)
    pos = rng.normal(size=(60, 3))
    mass = rng.uniform(0.5, 2.0, 60)
    phi = oracle.halo_potential(pos, mass, [0, 60], 0.0)
    w = 0.0
    for i in range(60):
        for j in range(i):
            w -= mass[i] * mass[j] / math.dist(pos[i], pos[j])
    assert np.dot(mass, phi) == pytest.approx(2.0 * w, rel=1e-12)
    shifted = oracle.halo_potential(pos + 64.0, mass, [0, 60], 0.0)
    np.testing.assert_allclose(shifted, phi, rtol=1e-12)


def test_plummer_central_potential():
    # a truncated Plummer sphere of N unit masses and scale a: the potential at
    # its centre is -N / a, less the truncation (a fraction 1 - (100/101)^1.5
    # of the mass sits beyond 10 a, which shifts the centre value by about 1%)
    rng = np.random.default_rng(7)
    n, a = 20000, 2.0
    pos = synth.plummer_offsets(rng, np.full(n, a))
    pos = np.concatenate([[[0.0, 0.0, 0.0]], pos])
    phi = oracle.halo_potential(pos, np.ones(n + 1), [0, n + 1], 0.0, targets=[0])
    m_in = (100.0 / 101.0) ** 1.5
    exact = -n / a * (m_in * 1.0)  # mass inside 10 a at its Plummer weight
    assert phi[0] == pytest.approx(exact, rel=0.03)


def test_halos_are_independent_and_targets_select():
    c = synth.halos_small()
    phi = oracle.halo_potential(c.pos, c.mass, c.offsets, c.eps)
    for h in (4, 10, 16):
        a, b = c.offsets[h], c.offsets[h + 1]
        alone = oracle.halo_potential(c.pos[a:b], c.mass[a:b], [0, b - a], c.eps)
        np.testing.assert_array_equal(alone, phi[a:b])
    t = np.array([5, 70, 300, c.n - 1])
    np.testing.assert_array_equal(oracle.halo_potential(c.pos, c.mass, c.offsets, c.eps, targets=t), phi[t])


def test_coincident_particles_and_most_bound_ties():
    pos = np.array([[0, 0, 0], [0, 0, 0], [1, 0, 0]], float)
    phi = oracle.halo_potential(pos, [1.0, 1.0, 1.0], [0, 3], 0.0)
    np.testing.assert_allclose(phi, [-1.0, -1.0, -2.0])  # coincident pair skipped at eps = 0
    phi = oracle.halo_potential(pos, [1.0, 1.0, 1.0], [0, 3], 0.5)
    np.testing.assert_allclose(phi[:2], -(2.0 + 1 / math.sqrt(1.25)))
    idx, _ = oracle.most_bound(np.array([-2.0, -3.0, -3.0, 1.0]), [0, 1, 1, 4])
    assert idx.tolist() == [0, -1, 1]  # the first of equal minima; -1 for an empty halo


def test_rejects_bad_offsets():
    pos = np.zeros((3, 3))
    for off in ([0, 2], [1, 3], [0, 2, 1, 3]):
        with pytest.raises(ValueError):
            oracle.halo_potential(pos, np.ones(3), off, 0.0)
