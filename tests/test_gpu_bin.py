"""Binning on the GPU is bit-exact against the oracle's float32 rule: cell of
every particle, cell starts, stable permutation, offsets, masses, active
counts and condition flags."""
import numpy as np
import pytest
import torch

import oracle
import paper_1411_3396_amd as sr
from paper_1411_3396_amd import synth
from gpu_helpers import DEV, announce, to_dev

pytestmark = pytest.mark.gpu


def check_bins(w):
    announce(f"bin {w.name} n={w.n} n_active={w.n_active} leaf_depth={w.problem.leaf_depth}")
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    ws = sr.bin(pos, mass, w.problem, w.n_active)
    v = sr.bin_view(ws, w.n, w.problem, w.n_active)
    torch.cuda.synchronize()
    ref = oracle.bin_reference(w.pos, w.problem, w.n_active)
    assert tuple(v["nc"]) == tuple(ref["nc"])
    np.testing.assert_array_equal(v["cell_of"].cpu().numpy(), ref["cell_of"])
    np.testing.assert_array_equal(v["cell_start"].cpu().numpy(), ref["cell_start"])
    np.testing.assert_array_equal(v["perm"].cpu().numpy(), ref["perm"])
    off = np.stack([v["off_x"].cpu().numpy(), v["off_y"].cpu().numpy(), v["off_z"].cpu().numpy()], 1)
    assert np.array_equal(off.view(np.uint32), ref["off"].view(np.uint32))
    np.testing.assert_array_equal(v["mass"].cpu().numpy(), w.mass[ref["perm"]])
    cells = ref["cell_of"][ref["perm"]]
    nact = np.bincount(cells[ref["perm"] < w.n_active], minlength=int(np.prod(ref["nc"])))
    np.testing.assert_array_equal(v["cell_nact"].cpu().numpy(), nact)
    assert sr.ws_flags(ws) == ref["flags"]


@pytest.mark.parametrize("case", ["uniform_32k", "clustered", "slab", "tiny", "one_cell"])
def test_bins_bit_exact(case):
    if case == "uniform_32k":
        w = synth.uniform_32k()
    elif case == "clustered":
        w = synth.clustered_box(300000, 60.0, 80, 4)
    elif case == "slab":
        w = synth.slab_with_ghosts(40, 3.0, 200, 5)
    elif case == "tiny":
        w = synth.uniform_box(5, 9.0, 6)
    else:
        w = synth.uniform_box(3000, 9.0, 7)
        w.problem = synth.Problem.make((0, 0, 0), (2.5, 2.5, 2.5), False, 3.0, 0.05, w.problem.poly)
        w.pos = (w.pos / 9.0 * 2.5).astype(np.float32)
    check_bins(w)


def subcell_faces():
    """Points on and one ulp either side of every sub-cell face of a depth-4
    octree inside one cell (h = 4), plus a NaN and two outside the domain."""
    f = np.float32
    xs = [f(8 + 0.25 * j) for j in range(17)]
    xs += [np.nextafter(f(10.0), f(0)), np.nextafter(f(10.0), f(20)), np.nextafter(f(9.0), f(0)),
           np.nextafter(f(11.5), f(20)), np.nextafter(f(8.0), f(20)), np.nextafter(f(12.0), f(0))]
    xs = np.array(xs, np.float32)
    grid = np.array(np.meshgrid(xs, xs[::2], xs[1::2], indexing="ij")).reshape(3, -1).T
    extra = np.array([[np.nan, 9.0, 9.0], [-1.0, 9.0, 9.0], [9.0, 40.0, 9.0]], np.float32)
    w = synth.uniform_box(1, 32.0, 0)
    w.pos = np.concatenate([grid, extra]).astype(np.float32)
    w.mass = np.ones(w.pos.shape[0], np.float32)
    w.n_active = w.pos.shape[0] - 500
    w.problem = synth.Problem.make((0, 0, 0), (32.0, 32.0, 32.0), False, 4.0, 0.05, (0.0,) * 6)
    return w


@pytest.mark.parametrize("depth", [2, 3, 4])
@pytest.mark.parametrize("case", ["clustered", "slab", "faces"])
def test_leaf_order_bins_bit_exact(case, depth):
    if case == "clustered":
        w = synth.clustered_box(200000, 60.0, 40, 14)
    elif case == "slab":
        w = synth.slab_with_ghosts(40, 3.0, 150, 15)
    else:
        w = subcell_faces()
    w.problem = w.problem.with_leaf_depth(depth)
    check_bins(w)


def test_bins_adversarial_positions():
    L = 32.0
    h = np.float32(3.2)
    ulp = np.spacing(np.float32(L))
    pts = np.array([0.0, L - ulp, -0.0, h, 2 * h, 9 * h, L - h, 1.5, -1e-8, L + 0.5, -3 * L + 1.0,
                    np.float32(L) - np.float32(1e-7)], np.float32)
    grid = np.array(np.meshgrid(pts, pts[:5], pts[3:9], indexing="ij")).reshape(3, -1).T
    pos = np.concatenate([grid, np.repeat(grid[:7], 4, axis=0)]).astype(np.float32)
    w = synth.uniform_box(1, L, 0)
    w.pos = pos
    w.mass = np.linspace(0.5, 2.0, pos.shape[0]).astype(np.float32)
    w.n_active = pos.shape[0] - 9
    check_bins(w)


def test_flags_nonfinite_and_out_of_domain():
    w = synth.slab_with_ghosts(12, 3.0, 5, 8)
    w.pos = w.pos.copy()
    w.pos[3] = [np.nan, 1.0, 1.0]
    w.pos[7] = [-20.0, 1.0, 1.0]
    check_bins(w)
    ws = sr.bin(to_dev(w.pos), to_dev(w.mass), w.problem, w.n_active)
    f = sr.ws_flags(ws)
    assert f & sr._sr.FLAG_NONFINITE and f & sr._sr.FLAG_OUT_OF_DOMAIN


def test_reuse_bins_on_unbinned_workspace_computes_nothing():
    w = synth.uniform_box(2000, 12.0, 3)
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    ws = torch.zeros(sr.workspace_bytes(w.n, w.problem), dtype=torch.uint8, device=DEV)
    out = torch.full((w.n, 3), 7.0, device=DEV)
    sr.force(pos, mass, w.problem, w.n, ws=ws, reuse_bins=True, out=out)
    assert sr.ws_flags(ws) & 4
    assert torch.all(out == 7.0)
