"""Overlapping data blocks (paper Sec. 2.1) on the CPU: the membership
oracle against geometry it must satisfy, the host-side partition and
refinement rules, and the host validation of the block plan."""
import ctypes as C

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle.blocks as ob
from paper_1411_3396_amd import _sr, synth
from paper_1411_3396_amd.blocks import equal_blocks, grid_units, refine, split


def slab(side=24, ghost=3.0, halos=30, seed=4):
    return synth.slab_with_ghosts(side, ghost, halos, seed)


def tiles(blocks, ng):
    cover = np.zeros(ng, np.int64)
    for gx0, gx1, gy0, gy1 in blocks:
        cover[gx0:gx1, gy0:gy1] += 1
    return np.all(cover == 1)


def test_equal_blocks_tile_the_grid():
    for ng, nbx, nby in [((30, 30), 3, 2), ((7, 5), 7, 5), ((326, 326), 4, 4), ((10, 3), 4, 1),
                         ((5, 5), 9, 9)]:
        b = equal_blocks(ng, nbx, nby)
        assert tiles(b, ng)
        w = [x1 - x0 for x0, x1, _, _ in b]
        assert max(w) - min(w) <= 1  # equal in whole grid units


def test_split_halves_the_longer_side():
    assert split((0, 8, 0, 4)) == [(0, 4, 0, 4), (4, 8, 0, 4)]
    assert split((0, 3, 2, 9)) == [(0, 3, 2, 5), (0, 3, 5, 9)]
    assert split((0, 4, 0, 4)) == [(0, 2, 0, 4), (2, 4, 0, 4)]  # x on ties
    assert split((5, 6, 5, 6)) == [(5, 6, 5, 6)]
    assert split((5, 6, 0, 3)) == [(5, 6, 0, 1), (5, 6, 1, 3)]


def test_refine_splits_only_blocks_over_twice_the_mean():
    b = equal_blocks((16, 16), 2, 2)
    # mean 2.5: only the block at 7 is more than twice the mean
    out = refine(b, [1.0, 1.0, 1.0, 7.0])
    assert out == b[:3] + split(b[3])
    assert tiles(out, (16, 16))
    assert refine(b, [1.0, 1.0, 1.0, 3.0]) == b  # exactly twice the mean (1.5) stays
    assert refine(b, [0, 0, 0, 0]) == b
    with pytest.raises(ValueError):
        refine(b, [1.0, 2.0])


def test_refinement_converges_on_a_concentrated_cost():
    # cost proportional to the area over one hot corner: repeated refinement
    # leaves no block above twice the mean, and the tiling stays exact
    ng = (64, 64)
    b = equal_blocks(ng, 2, 2)
    weight = np.ones(ng)
    weight[:8, :8] = 400.0
    for _ in range(40):
        cost = [weight[x0:x1, y0:y1].sum() for x0, x1, y0, y1 in b]
        nxt = refine(b, cost)
        if nxt == b:
            break
        b = nxt
    else:
        raise AssertionError("refinement did not settle")
    cost = np.array([weight[x0:x1, y0:y1].sum() for x0, x1, y0, y1 in b])
    assert tiles(b, ng)
    assert cost.max() <= 2 * cost.mean()
    area = np.array([(x1 - x0) * (y1 - y0) for x0, x1, y0, y1 in b])
    hot = np.array([x0 < 8 and y0 < 8 for x0, x1, y0, y1 in b])
    # blocks stay as large as the balance allows: fine over the hot corner only
    assert area[hot].max() < area[~hot].min() and area[~hot].max() == 32 * 32


@pytest.mark.parametrize("blocks_of", ["equal_3x2", "refined", "one", "strips"])
def test_oracle_membership_holds_every_interaction(blocks_of):
    w = slab()
    ng = grid_units(w.problem)
    blocks = {"equal_3x2": equal_blocks(ng, 3, 2),
              "refined": refine(equal_blocks(ng, 2, 2), [9, 1, 1, 1]),
              "one": [(0, ng[0], 0, ng[1])],
              "strips": equal_blocks(ng, ng[0] // 2, 1)}[blocks_of]
    memb = ob.members(w.pos, w.n_active, w.problem, ng, blocks)
    # every active particle is active in exactly one block, passives in none
    act = np.concatenate([a for a, _ in memb])
    assert np.array_equal(np.sort(act), np.arange(w.n_active))
    # Sec. 2.1: a block updates its active particles correctly, so each one's
    # full r_s neighbourhood (brute force over the float64 positions) is in
    # the block
    x = w.pos.astype(np.float64)
    tree = cKDTree(x)
    home = np.empty(w.n_active, np.int64)
    for b, (a, _) in enumerate(memb):
        home[a] = b
    sets = [set(np.concatenate(m).tolist()) for m in memb]
    sample = synth.sample_indices(w.n_active, 2000, 5)
    for i in sample:
        nb = tree.query_ball_point(x[i], w.problem.r_s * (1 + 1e-7))
        assert set(nb) <= sets[home[i]], i
    # and nothing farther than the widened shell (plus rounding) is a member
    home_r, _ = ob.rectangles(w.problem, ng, blocks)
    rs = w.problem.r_s * (1 + 1e-5) * (1 + 1e-6)
    for b, (a, p) in enumerate(memb):
        m = np.concatenate([a, p])
        x0, x1, y0, y1 = home_r[b].astype(np.float64)
        dx = np.maximum(np.maximum(x0 - x[m, 0], x[m, 0] - x1), 0)
        dy = np.maximum(np.maximum(y0 - x[m, 1], x[m, 1] - y1), 0)
        assert np.all((dx <= rs) & (dy <= rs))


def test_oracle_membership_orders_and_edge_cases():
    P = synth.Problem.make((-3, -3, -3), (20.0, 20.0, 20.0), False, 3.0, 0.05, (0,) * 6)
    ng = (20, 20)
    blocks = equal_blocks(ng, 2, 2)  # edges at x, y = 7
    pts = np.array([[6.999, 0, 0], [7.0, 0, 0], [-50, -50, 0], [50, 50, 0], [np.nan, 0, 0],
                    [7.0, 7.0, 1.0], [7.0 + 3.0 * (1 + 2e-5), 0, 0], [7.0 + 3.0 * (1 + 0.5e-5), 0, 0]],
                   np.float32)
    memb = ob.members(pts, 5, P, ng, blocks)
    homes = {int(i): b for b, (a, _) in enumerate(memb) for i in a}
    assert homes == {0: 0, 1: 2, 2: 0, 3: 3, 4: 0}
    # the NaN particle belongs to block 0 only; the passive point 5 at the
    # corner is in all four blocks; points 6 and 7 sit just past and just
    # inside the widened shell of block 0 (x = 7 + r_s (1 + 1e-5))
    in_blocks = lambda i: [b for b, (a, p) in enumerate(memb) if i in a or i in p]  # noqa: E731
    assert in_blocks(4) == [0]
    assert in_blocks(5) == [0, 1, 2, 3]
    assert in_blocks(6) == [2]
    assert in_blocks(7) == [0, 2]
    assert in_blocks(0) == [0, 2] and in_blocks(1) == [0, 2]
    assert in_blocks(2) == [0] and in_blocks(3) == [3]
    for a, p in memb:
        assert np.all(np.diff(a) > 0) and np.all(np.diff(p) > 0)


def _plan(domain, ng, blocks, n=1000, n_active=None, capacity=0):
    arr = (_sr.Block * max(1, len(blocks)))(*[_sr.Block(*b) for b in blocks])
    ngs = (C.c_int32 * 2)(*ng)
    plan = C.c_void_p()
    nbytes = C.c_size_t()
    code = _sr.lib().sr_blocks_plan_create(C.byref(_sr.as_problem(domain)), ngs, len(blocks), arr, n,
                                           n if n_active is None else n_active, capacity,
                                           C.byref(plan), C.byref(nbytes))
    if code == 0:
        _sr.lib().sr_blocks_plan_destroy(plan)
    return code, nbytes.value


def test_block_plan_host_validation():
    w = slab()
    ng = grid_units(w.problem)
    ok = equal_blocks(ng, 2, 2)
    assert _plan(w.problem, ng, ok)[0] == 0
    assert _plan(w.problem, ng, ok[:3])[0] == 1  # gap
    assert _plan(w.problem, ng, ok + [ok[0]])[0] == 1  # overlap
    bad = list(ok)
    bad[0] = (0, ng[0] + 1, 0, 1)
    assert _plan(w.problem, ng, bad)[0] == 1  # outside the grid
    bad[0] = (3, 3, 0, 1)
    assert _plan(w.problem, ng, bad)[0] == 1  # empty
    shifted = [(a, b, c, d) for a, b, c, d in ok]
    shifted[0], shifted[1] = (0, 14, 0, 15), (14, 15, 0, 15)  # overlaps + gap, same area
    assert _plan(w.problem, ng, shifted)[0] == 1
    assert _plan(w.problem, ng, [])[0] == 1
    assert _plan(w.problem, (ng[0], 0), ok)[0] == 1
    assert _plan(w.problem, ng, equal_blocks(ng, ng[0], ng[1]) if ng[0] * ng[1] <= 1024 else ok)[0] == 0
    assert _plan(w.problem, (64, 64), equal_blocks((64, 64), 64, 64))[0] == 1  # > 1024 blocks
    assert _plan(w.problem, ng, ok, n=10, n_active=11)[0] == 1
    per = synth.uniform_box(10, 12.0, 1).problem
    assert _plan(per, (12, 12), equal_blocks((12, 12), 2, 2))[0] == 5  # periodic: unsupported
    # workspace grows with n and with the capacity
    a = _plan(w.problem, ng, ok, n=1000)[1]
    b = _plan(w.problem, ng, ok, n=100000)[1]
    c = _plan(w.problem, ng, ok, n=100000, capacity=120000)[1]
    assert 0 < a < b and c < b and a % 256 == 0
    # the worst-case membership count must fit 32-bit indices
    assert _plan(w.problem, ng, ok, n=(1 << 30))[0] == 5


def test_block_problems_cover_their_widened_rectangles():
    w = slab()
    ng = grid_units(w.problem)
    blocks = refine(equal_blocks(ng, 3, 2), [5, 1, 1, 1, 1, 1])
    bp = _sr.BlocksPlan(w.problem, ng, blocks, 100)
    probs = bp.problems()
    home_r, wide_r = ob.rectangles(w.problem, ng, blocks)
    dlo = np.array(w.problem.lo[:2], np.float64)
    dhi = dlo + np.array(w.problem.len[:2], np.float64)
    for b, p in enumerate(probs):
        assert p.periodic == 0 and p.r_s == np.float32(w.problem.r_s)
        assert tuple(p.lo)[2] == np.float32(w.problem.lo[2]) and tuple(p.len)[2] == np.float32(w.problem.len[2])
        for a in range(2):
            lo, hi = float(p.lo[a]), float(p.lo[a]) + float(p.len[a])
            want_lo = max(dlo[a], float(wide_r[b][2 * a]))
            want_hi = min(dhi[a], float(wide_r[b][2 * a + 1]))
            assert lo <= want_lo and hi >= want_hi
            assert lo >= dlo[a] - 1e-4 and hi <= dhi[a] + 1e-4
            assert hi - lo <= float(home_r[b][2 * a + 1] if np.isfinite(home_r[b][2 * a + 1]) else dhi[a]) \
                - float(home_r[b][2 * a] if np.isfinite(home_r[b][2 * a]) else dlo[a]) + 2 * 3.0 * 1.001
    bp.close()
