"""Symmetric (Newton's third law) tiles of the dense cells: every unordered
pair of dense particles evaluated once, both opposite terms kept in partial
slots and gathered in a fixed order.  Checked against the float64 oracle at
several tile sizes, against the one-sided kernels (tiles off), run to run
bitwise, on a problem whose partial slots do not fit the pool (the tiles
then stay off and the one-sided kernels do all the work), and under the
balance rule that keeps them off when a few long items would dominate.
These test problems are small, so the balance rule is switched off (0)
wherever the tiles are meant to run."""
import numpy as np
import pytest
import torch

import oracle
import paper_1411_3396_amd as sr
from paper_1411_3396_amd import synth
from gpu_helpers import DEV, FWD_TOL, VJP_TOL, announce, assert_force_close, oracle_force, to_dev

pytestmark = pytest.mark.gpu

HDR_SYM_OK = 518  # header word: the symmetric tiles ran


def run(w, g, kernel_tiles=None, extra_slots=80, balance=0.0):
    """Forward and adjoint on a fresh workspace with room for extra_slots more partial slots
    per particle than sr_workspace_bytes reserves; returns (acc, grad, sym_ok_fwd, sym_ok_vjp)."""
    saved = {k: sr.tile_config(kernel=k) for k in ("force", "vjp")}
    saved_balance = sr.tile_balance()
    try:
        sr.tile_balance(balance)
        if kernel_tiles is not None:
            for k in ("force", "vjp"):
                sr.tile_config(*kernel_tiles, kernel=k)
        pos, mass = to_dev(w.pos), to_dev(w.mass)
        nb = sr.workspace_bytes(w.n, w.problem) + int(12.25 * extra_slots * w.n)
        ws = sr.new_workspace(nb, DEV)
        acc = sr.force(pos, mass, w.problem, w.n_active, ws=ws)
        torch.cuda.synchronize()
        ok_f = int(ws[4 * HDR_SYM_OK:4 * HDR_SYM_OK + 4].view(torch.int32).item())
        gr = sr.force_vjp(pos, mass, w.problem, to_dev(g), w.n_active, ws=ws, reuse_bins=True)
        torch.cuda.synchronize()
        ok_v = int(ws[4 * HDR_SYM_OK:4 * HDR_SYM_OK + 4].view(torch.int32).item())
        assert sr.ws_flags(ws) == 0
        return acc.cpu().numpy(), gr.cpu().numpy(), ok_f, ok_v
    finally:
        for k, v in saved.items():
            sr.tile_config(*v, kernel=k)
        sr.tile_balance(saved_balance)


def dense_cases():
    def halos_random_mass():
        w = synth.clustered_box(150000, 40.0, 80, 5, halo_frac=0.5, mass_range=(1e2, 1e4))
        w.mass = np.random.default_rng(5).uniform(0.5, 2.0, w.n).astype(np.float32)
        return w

    def slab_ghosts():
        w = synth.slab_with_ghosts(30, 3.0, 60, 4)
        w.problem = w.problem.with_leaf_depth(2)
        return w

    def small_periodic():
        # three cells per dimension: every cell pair is a neighbour, wrapping
        w = synth.uniform_box(27 * 300, 9.3, 6)
        return w

    def unsoftened():
        w = synth.clustered_box(60000, 24.0, 10, 8, halo_frac=0.8, mass_range=(1e3, 1e4))
        w.problem = synth.Problem.make((0, 0, 0), w.problem.len, True, 3.0, 0.0, synth.filter_poly(3.0, 0.05))
        return w

    return {"halos_random_mass": halos_random_mass, "slab_ghosts": slab_ghosts,
            "small_periodic": small_periodic, "unsoftened": unsoftened}


@pytest.mark.parametrize("name", list(dense_cases()))
def test_symmetric_tiles_match_oracle_and_one_sided(name):
    w = dense_cases()[name]()
    g = synth.cotangent(w.n_active, 3)
    ref = oracle_force(w)
    gref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g)
    announce(f"symmetric tiles {name} n={w.n} n_active={w.n_active}")
    a0, g0, f0, v0 = run(w, g, (0, -1))
    assert f0 == 0 and v0 == 0
    assert_force_close(a0, ref, what=f"{name} one-sided")
    for tiles in [(16, 256), (16, 512), (1, 256), (3, 512), (256, 256)]:
        a, gr, ok_f, ok_v = run(w, g, tiles)
        assert ok_f == 1 and ok_v == 1, (tiles, ok_f, ok_v)
        assert_force_close(a, ref, what=f"{name} tiles {tiles}")
        e = oracle.rms_rel(gr, gref)
        print(f"  vjp tiles {tiles} rms_rel={e:.3e}", flush=True)
        assert e <= VJP_TOL
        # the same pair terms summed in another order: far inside the tolerances
        assert oracle.rms_rel(a, a0) <= 2e-6, tiles
        assert oracle.rms_rel(gr, g0) <= 2e-5, tiles
        a2, g2, _, _ = run(w, g, tiles)
        assert np.array_equal(a.view(np.uint32), a2.view(np.uint32)), tiles
        assert np.array_equal(gr.view(np.uint32), g2.view(np.uint32)), tiles


def test_symmetric_tiles_random_filter_dense():
    # a filter that is not continuous at r_s, on dense cells; targets with a
    # pair within 1e-4 of r_s are left out (float32 and float64 may decide them
    # differently)
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(31)
    poly = tuple(float(np.float32(rng.uniform(-1, 1) * 0.05 / 9.0 ** k)) for k in range(6))
    w = synth.uniform_box(27 * 400, 9.6, 9)
    w.mass = rng.uniform(0.5, 2.0, w.n).astype(np.float32)
    w.problem = synth.Problem.make((0, 0, 0), (9.6,) * 3, True, 3.0, 0.05, poly)
    t = cKDTree(w.pos.astype(np.float64), boxsize=9.6)
    close = t.query_pairs(3.0 + 1e-4) - t.query_pairs(3.0 - 1e-4)
    bad = np.zeros(w.n, bool)
    for i, j in close:
        bad[i] = bad[j] = True
    keep = np.nonzero(~bad)[0]
    announce(f"symmetric random filter: {int(bad.sum())} of {w.n} targets near the cutoff left out")
    assert len(keep) >= 0.7 * w.n  # about 24% of targets have a pair in the shell at this density
    g = synth.cotangent(w.n, 4)
    a, gr, ok_f, ok_v = run(w, g, (16, 512))
    assert ok_f == 1 and ok_v == 1
    assert_force_close(a[keep], oracle_force(w)[keep], what="random filter, tiles on")
    gref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g)
    assert oracle.rms_rel(gr[keep], gref[keep]) <= VJP_TOL


def test_partial_slots_beyond_the_pool_fall_back():
    # 27 cells of about 2000 particles need ~83 partial slots per particle:
    # with the workspace sr_workspace_bytes gives (about 15 per particle) the
    # tiles stay off and the one-sided kernels sum every pair; a larger
    # workspace lends its tail to the slots and the tiles run
    w = synth.uniform_box(27 * 2000, 9.3, 11)
    w.mass = np.random.default_rng(8).uniform(0.5, 2.0, w.n).astype(np.float32)
    g = synth.cotangent(w.n, 6)
    idx = synth.sample_indices(w.n, 3000, 1)
    acc_ref, _ = oracle.force(w.pos, w.mass, w.n_active, w.problem, targets=idx)
    gref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g, targets=idx)
    for extra, want in ((0, 0), (100, 1)):
        announce(f"pool n={w.n} extra slots per particle {extra}")
        a, gr, ok_f, ok_v = run(w, g, (16, 512), extra_slots=extra)
        assert ok_f == want and ok_v == want
        assert_force_close(a[idx], acc_ref, what=f"extra {extra}")
        assert oracle.rms_rel(gr[idx], gref) <= VJP_TOL


def test_balance_rule_keeps_long_items_off():
    # 27 cells of 300 particles: at 256 blocks per item each cell is one item,
    # far longer than the work per wave of the persistent grid, so the default
    # balance rule keeps the tiles off; with the rule at 0 they run.  Either
    # way the forces match the oracle and each other to rounding order.
    w = dense_cases()["small_periodic"]()
    g = synth.cotangent(w.n_active, 5)
    ref = oracle_force(w)
    announce(f"balance rule n={w.n}")
    a1, g1, f1, v1 = run(w, g, (256, 256), balance=1.0)
    assert f1 == 0 and v1 == 0
    a0, g0, f0, v0 = run(w, g, (256, 256), balance=0.0)
    assert f0 == 1 and v0 == 1
    for a in (a0, a1):
        assert_force_close(a, ref, what="balance rule")
    assert oracle.rms_rel(a0, a1) <= 2e-6
    assert oracle.rms_rel(g0, g1) <= 2e-5


@pytest.mark.parametrize("rest", [1, 15, 16, 17, 33, 48, 49, 63])
def test_stream_tails_of_every_row_count(rest):
    # one cluster of 128 + rest particles inside one cell of a 3-cell periodic
    # box, every pair within reach: block 0 streams block 1 and the rest, block
    # 1 the rest, so both streams end with `rest` survivors and finish with
    # ceil(rest / 16) row chunks (a full 64-step tile past 48), on top of the
    # triangles of both blocks and the one-sided items of the rest
    rng = np.random.default_rng(100 + rest)
    n = 128 + rest
    w = synth.uniform_box(n, 9.3, 12)
    w.pos = (np.float32(4.65) + rng.uniform(-0.5, 0.5, (n, 3))).astype(np.float32)
    w.mass = rng.uniform(0.5, 2.0, n).astype(np.float32)
    g = synth.cotangent(n, 13)
    ref = oracle_force(w)
    gref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g)
    announce(f"stream tails rest={rest} n={n}")
    a0, g0, f0, v0 = run(w, g, (0, -1))
    assert f0 == 0 and v0 == 0
    a, gr, ok_f, ok_v = run(w, g, (16, 256))
    assert ok_f == 1 and ok_v == 1
    assert_force_close(a, ref, what=f"tails rest={rest}")
    assert oracle.rms_rel(gr, gref) <= VJP_TOL
    assert oracle.rms_rel(a, a0) <= 2e-6
    assert oracle.rms_rel(gr, g0) <= 2e-5
