"""Power spectrum on the GPU (paper Sec. 4.1) against the float64 oracle:
the CIC grid point by point, the mode counts exactly, and P(k) per bin.
Grids whose side is a multiple of 8 take the brick deposit, the others the
cell deposit; both are covered."""
import numpy as np
import pytest
import torch

from oracle import pk as opk
import paper_1411_3396_amd as sr
from paper_1411_3396_amd import synth
from gpu_helpers import DEV, announce, to_dev

pytestmark = pytest.mark.gpu

# float32 weights; the brick deposit sums them exactly per tile and adds a
# point's float32 tile values in float64, the cell deposit sums them in float64
GRID_RTOL = 1e-6
PK_RTOL = 1e-4     # float32 grid and FFT; measured float32-vs-float64 bin error <= 5e-6


def exact_scale(pos, box, ng):
    """(pos, box) with ng / box a power of two, so that u = x ng / box is exact
    in float32 on both sides: otherwise the positions are rescaled to box = ng
    (as float32) first.  The deposit defines u in float32; this keeps that
    rounding, which the float64 oracle does not make, out of the comparison."""
    r = ng / box
    if np.log2(r) == np.round(np.log2(r)):
        return pos, box
    return (pos.astype(np.float64) * r).astype(np.float32), float(ng)


def case(name):
    if name == "uniform_32k":
        w = synth.uniform_32k()
        return w.pos, w.mass, 32.0
    if name == "clustered_64":
        w = synth.clustered_box(262144, 64.0, 100, 4)
        mass = np.random.default_rng(5).uniform(0.5, 2.0, w.n).astype(np.float32)
        return w.pos, mass, 64.0
    w = synth.clustered_2m()
    return w.pos, w.mass, 128.0


@pytest.mark.parametrize("name,ng", [("uniform_32k", 32), ("uniform_32k", 64), ("clustered_64", 64),
                                     ("clustered_64", 32), ("uniform_32k", 36), ("clustered_64", 30),
                                     ("clustered_64", 8)])
def test_deposit_matches_oracle(name, ng):
    pos, mass, box = case(name)
    pos, box = exact_scale(pos, box, ng)
    announce(f"cic deposit {name} ng={ng}")
    plan = sr.PkPlan(ng, box, 8, n_max=pos.shape[0])
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    grid, mtot = plan.deposit(to_dev(pos), to_dev(mass), ws)
    got = grid.cpu().numpy().astype(np.float64)
    ref = opk.cic_deposit(pos, mass, ng, box)
    np.testing.assert_allclose(got, ref, rtol=GRID_RTOL, atol=1e-30)
    assert float(mtot.cpu()[0]) == pytest.approx(float(np.sum(mass.astype(np.float64))), rel=1e-12)
    # the sorted deposit repeats bit for bit (got holds the first run's float32 values)
    again, _ = plan.deposit(to_dev(pos), to_dev(mass), ws)
    first = got.astype(np.float32)
    assert np.array_equal(again.cpu().numpy().view(np.uint32), first.view(np.uint32))
    plan.close()


@pytest.mark.parametrize("name,ng,dn", [("uniform_32k", 32, 1.0), ("clustered_64", 64, 1.0),
                                        ("clustered_2m", 128, 2.0)])
def test_power_spectrum_matches_oracle(name, ng, dn):
    pos, mass, box = case(name)
    n_bins = int(np.ceil(np.sqrt(3) * ng / 2 / dn)) + 1
    announce(f"power spectrum {name} ng={ng} bins={n_bins}")
    plan = sr.PkPlan(ng, box, n_bins, dn, n_max=pos.shape[0])
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    p, k, modes = plan.run(to_dev(pos), to_dev(mass), ws)
    p, k, modes = p.cpu().numpy(), k.cpu().numpy(), modes.cpu().numpy()
    rp, rk, rc = opk.power_spectrum(opk.cic_deposit(pos, mass, ng, box), box, n_bins, dn)
    np.testing.assert_array_equal(modes, rc)
    ok = rc > 0
    np.testing.assert_allclose(k[ok], rk[ok], rtol=1e-12)
    rel = np.abs(p[ok] - rp[ok]) / rp[ok]
    print(f"  max rel {rel.max():.3e} median {np.median(rel):.3e}", flush=True)
    assert rel.max() <= PK_RTOL
    assert np.all(p[~ok] == 0)
    # runs on the same plan and on a fresh workspace repeat bit for bit: the
    # deposit, the FFT and the mode sums all add in a fixed order
    p2, k2, m2 = (t.cpu().numpy() for t in plan.run(to_dev(pos), to_dev(mass), ws))
    ws3 = sr.new_workspace(plan.ws_bytes, DEV)
    p3 = plan.run(to_dev(pos), to_dev(mass), ws3)[0].cpu().numpy()
    assert np.array_equal(p2.view(np.uint64), p.view(np.uint64))
    assert np.array_equal(k2.view(np.uint64), k.view(np.uint64))
    assert np.array_equal(m2, modes)
    assert np.array_equal(p3.view(np.uint64), p.view(np.uint64))
    plan.close()


@pytest.mark.parametrize("n,ng", [(1, 16), (63, 16), (64, 16), (65, 16), (128, 16), (129, 16), (5000, 16),
                                  (2731, 16), (20000, 16), (129, 12), (5000, 12)])
def test_deposit_crowded_cells_and_wrap(n, ng):
    # n particles in one cell and n // 2 in its neighbour, plus particles on
    # grid points and across the periodic faces.  Cell deposit (ng = 12): the
    # sorted slots of a crowded cell are cut into 64-slot runs whose partials
    # the grid points add back.  Brick deposit (ng = 16): both cells sit in one
    # brick, cut into chunks of 2048 particles (2731 + 1365 = 4096 exactly two,
    # more with the particles spread over the box) whose tiles the points add
    box = 16.0
    rng = np.random.default_rng(n)
    crowd = np.array([5.0, 7.0, 9.0]) + rng.random((n, 3)) * 0.999
    nbr = np.array([6.0, 7.0, 9.0]) + rng.random((n // 2, 3)) * 0.999
    faces = np.array([[0, 0, 0], [16, 16, 16], [15.5, 0, 8], [8, 8, 8], [31.5, 0.5, 0.5],
                      [-0.5, 3.25, 15.75], [4, 4, 4]])
    pos = np.concatenate([crowd, nbr, faces, rng.random((300, 3)) * 16]).astype(np.float32)
    pos = pos[rng.permutation(len(pos))]
    pos, box = exact_scale(pos, box, ng)
    mass = rng.uniform(0.5, 2.0, len(pos)).astype(np.float32)
    announce(f"cic deposit crowded cell n={n}")
    plan = sr.PkPlan(ng, box, 8, n_max=len(pos))
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    grid, _ = plan.deposit(to_dev(pos), to_dev(mass), ws)
    got = grid.cpu().numpy()
    ref = opk.cic_deposit(pos, mass, ng, box)
    np.testing.assert_allclose(got.astype(np.float64), ref, rtol=GRID_RTOL, atol=1e-30)
    again, _ = plan.deposit(to_dev(pos), to_dev(mass), ws)
    assert np.array_equal(again.cpu().numpy().view(np.uint32), got.view(np.uint32))
    plan.close()


@pytest.mark.parametrize("ng", [16, 12])
def test_non_finite_position_reaches_the_spectrum(ng):
    # a NaN or infinite coordinate gives NaN weights: the grid points they reach
    # and then every P(k) bin with modes are NaN (never a finite wrong value)
    rng = np.random.default_rng(ng)
    box = float(ng)
    pos = (rng.random((2000, 3)) * box).astype(np.float32)
    mass = rng.uniform(0.5, 2.0, 2000).astype(np.float32)
    pos[7, 1] = np.nan
    pos[11, 2] = np.inf
    announce(f"cic deposit non-finite positions ng={ng}")
    plan = sr.PkPlan(ng, box, 8, n_max=len(pos))
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    grid, _ = plan.deposit(to_dev(pos), to_dev(mass), ws)
    g = grid.cpu().numpy()
    assert np.isnan(g).any()
    ok = np.delete(np.arange(len(pos)), [7, 11])
    ref = opk.cic_deposit(pos[ok], mass[ok], ng, box)
    # the points no NaN reached (all but the 8 corners of a NaN particle's cell,
    # or the 9^3 tile of its brick) hold the deposit of the finite particles
    fin = np.isfinite(g)
    assert fin.sum() >= g.size - 2 * (8 if ng % 8 else 729)
    np.testing.assert_allclose(g[fin].astype(np.float64), ref[fin], rtol=GRID_RTOL, atol=1e-30)
    p, _, modes = (t.cpu().numpy() for t in plan.run(to_dev(pos), to_dev(mass), ws))
    assert np.all(np.isnan(p[modes > 0]))
    plan.close()


def test_deposit_large_brick_count():
    # ng = 328: 41^3 = 68,921 bricks (the largest grid here besides the bench's),
    # a grid side that is not a power of two, and a crowd of 6000 particles in
    # one brick that spans 3 chunks
    ng = 328
    box = float(ng)
    rng = np.random.default_rng(328)
    pos = np.concatenate([rng.random((60000, 3)) * box,
                          np.array([100.0, 200.0, 300.0]) + rng.random((6000, 3)) * 7.9]).astype(np.float32)
    mass = rng.uniform(0.5, 2.0, len(pos)).astype(np.float32)
    announce(f"cic deposit ng={ng} n={len(pos)}")
    plan = sr.PkPlan(ng, box, 8, n_max=len(pos))
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    grid, mtot = plan.deposit(to_dev(pos), to_dev(mass), ws)
    got = grid.cpu().numpy()
    ref = opk.cic_deposit(pos, mass, ng, box)
    np.testing.assert_allclose(got.astype(np.float64), ref, rtol=GRID_RTOL, atol=1e-30)
    assert float(mtot.cpu()[0]) == pytest.approx(float(np.sum(mass.astype(np.float64))), rel=1e-12)
    again, _ = plan.deposit(to_dev(pos), to_dev(mass), ws)
    assert np.array_equal(again.cpu().numpy().view(np.uint32), got.view(np.uint32))
    plan.close()


def test_deposit_unaligned_positions():
    # positions that start 4 bytes past a 16-byte boundary take the scalar
    # staging path of the first sort pass: the same grid bit for bit
    w = synth.clustered_box(100000, 64.0, 30, 6)
    pos, mass, box = w.pos, w.mass, 64.0
    announce("cic deposit unaligned positions")
    plan = sr.PkPlan(64, box, 8, n_max=len(pos))
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    g0 = plan.deposit(to_dev(pos), to_dev(mass), ws)[0].cpu().numpy().copy()
    flat = torch.empty(3 * len(pos) + 1, dtype=torch.float32, device=DEV)
    flat[1:] = to_dev(pos).reshape(-1)
    shifted = flat[1:].view(len(pos), 3)
    assert shifted.data_ptr() % 16 != 0
    g1 = plan.deposit(shifted, to_dev(mass), ws)[0].cpu().numpy()
    assert np.array_equal(g0.view(np.uint32), g1.view(np.uint32))
    plan.close()
