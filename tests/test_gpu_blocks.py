"""Overlapping data blocks on the GPU (paper Sec. 2.1): the partition is
bit-exact against the membership oracle, and the reconciled block forces and
gradients agree with the float64 oracle of the whole domain."""
import numpy as np
import pytest
import torch

import oracle
import oracle.blocks as ob
from paper_1411_3396_amd import _sr, synth
from paper_1411_3396_amd.blocks import BlockForce, equal_blocks, grid_units, refine
from gpu_helpers import DEV, VJP_TOL, announce, assert_force_close, to_dev

pytestmark = pytest.mark.gpu


def domain_case(kind):
    w = synth.slab_with_ghosts(24, 3.0, 30, 4)
    ng = grid_units(w.problem)
    if kind == "equal_3x2":
        blocks = equal_blocks(ng, 3, 2)
    elif kind == "refined":
        blocks = refine(refine(equal_blocks(ng, 2, 2), [9, 1, 1, 1]), [9, 1, 1, 1, 1])
    elif kind == "one":
        blocks = [(0, ng[0], 0, ng[1])]
    elif kind == "strips":
        blocks = equal_blocks(ng, 10, 1)
    elif kind == "fine":
        blocks = equal_blocks(ng, 15, 15)
    else:
        raise ValueError(kind)
    return w, ng, blocks


def with_strays(w):
    """Add passive particles outside the domain and a NaN one (flags in blocks)."""
    w.pos = np.concatenate([w.pos, np.array([[-40.0, 5.0, 5.0], [5.0, 99.0, 5.0], [np.nan, 1.0, 1.0]],
                                            np.float32)])
    w.mass = np.concatenate([w.mass, np.ones(3, np.float32)])
    return w


@pytest.mark.parametrize("kind", ["equal_3x2", "refined", "one", "strips", "fine"])
def test_partition_matches_membership_oracle(kind):
    w, ng, blocks = domain_case(kind)
    w = with_strays(w)
    announce(f"blocks partition {kind} nb={len(blocks)} n={w.n}")
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    plan = _sr.BlocksPlan(w.problem, ng, blocks, w.n, w.n_active)
    ws = _sr.new_workspace(plan.ws_bytes, DEV)
    counts = plan.partition(pos, ws)
    bpos, bmass, src, _ = plan.gather(pos, mass, ws)
    torch.cuda.synchronize()
    memb = ob.members(w.pos, w.n_active, w.problem, ng, blocks)
    np.testing.assert_array_equal(counts, np.array([[len(a), len(p)] for a, p in memb]))
    ref = ob.order(memb)
    np.testing.assert_array_equal(src.cpu().numpy(), ref)
    got = bpos.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), w.pos[ref].view(np.uint32))
    np.testing.assert_array_equal(bmass.cpu().numpy(), w.mass[ref])
    plan.close()


def test_reconcile_takes_each_active_row_once():
    w, ng, blocks = domain_case("refined")
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    plan = _sr.BlocksPlan(w.problem, ng, blocks, w.n, w.n_active)
    ws = _sr.new_workspace(plan.ws_bytes, DEV)
    plan.partition(pos, ws)
    memb = ob.members(w.pos, w.n_active, w.problem, ng, blocks)
    rows = np.concatenate([a for a, _ in memb])  # domain index of each block output row
    bacc = torch.arange(3 * w.n_active, dtype=torch.float32, device=DEV).reshape(-1, 3)
    acc = torch.full((w.n_active, 3), float("nan"), device=DEV)
    plan.reconcile(bacc, ws, out=acc)
    got = acc.cpu().numpy()
    want = np.empty_like(got)
    want[rows] = bacc.cpu().numpy()
    np.testing.assert_array_equal(got, want)
    # cotangent rows are the inverse map
    g = torch.from_numpy(np.random.default_rng(1).standard_normal((w.n_active, 3)).astype(np.float32)).to(DEV)
    _, _, _, bg = plan.gather(pos, mass, ws, g=g)
    np.testing.assert_array_equal(bg.cpu().numpy(), g.cpu().numpy()[rows])
    # gradients: every copy's row summed, in block order
    m = plan.members
    bgrad = torch.from_numpy(np.random.default_rng(2).standard_normal((m, 3)).astype(np.float32)).to(DEV)
    grad = plan.reconcile_grad(bgrad, ws).cpu().numpy()
    order = ob.order(memb)
    bg_np = bgrad.cpu().numpy()
    want = np.zeros((w.n, 3), np.float32)
    for s in range(m):  # block order = slot order
        want[order[s]] += bg_np[s]
    np.testing.assert_array_equal(grad, want)
    plan.close()


@pytest.mark.parametrize("kind", ["equal_3x2", "refined", "strips", "fine"])
def test_block_forces_match_oracle(kind):
    w, ng, blocks = domain_case(kind)
    announce(f"block forces {kind} nb={len(blocks)}")
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    bf = BlockForce(w.problem, blocks, w.n, w.n_active, ng=ng, device=DEV, tune_cache=None)
    acc = bf.forward(pos, mass, mode="graph").cpu().numpy()
    acc_eager = bf.forward(pos, mass, mode="eager").cpu().numpy()
    assert np.array_equal(acc, acc_eager)
    ref, _ = oracle.force(w.pos, w.mass, w.n_active, w.problem)
    assert_force_close(acc, ref, what=f"blocks {kind}")
    # the duplicated work is the overlap of the shells
    assert bf.plan.members >= w.n
    bf.close()


def test_block_forces_with_leaf_depth():
    # the blocks inherit the domain's in-cell octree depth
    w, ng, blocks = domain_case("refined")
    w.problem = w.problem.with_leaf_depth(3)
    announce("block forces refined, leaf depth 3")
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    bf = BlockForce(w.problem, blocks, w.n, w.n_active, ng=ng, device=DEV, tune_cache=None)
    assert all(p.leaf_depth == 3 for p in bf.problems)
    acc = bf.forward(pos, mass).cpu().numpy()
    ref, _ = oracle.force(w.pos, w.mass, w.n_active, w.problem)
    assert_force_close(acc, ref, what="blocks leaf depth 3")
    bf.close()


def test_block_vjp_matches_oracle():
    w, ng, blocks = domain_case("refined")
    announce("block vjp refined")
    g = synth.cotangent(w.n_active, 3)
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    bf = BlockForce(w.problem, blocks, w.n, w.n_active, ng=ng, device=DEV, tune_cache=None)
    grad = bf.vjp(pos, mass, to_dev(g)).cpu().numpy()
    ref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g)
    err = oracle.rms_rel(grad, ref)
    print(f"  block vjp rms_rel={err:.3e}", flush=True)
    assert err <= VJP_TOL
    bf.close()


def test_capacity_too_small_is_reported_and_recovered():
    w, ng, blocks = domain_case("fine")
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    plan = _sr.BlocksPlan(w.problem, ng, blocks, w.n, w.n_active, capacity=w.n)
    ws = _sr.new_workspace(plan.ws_bytes, DEV)
    with pytest.raises(_sr.SRError) as e:
        plan.partition(pos, ws)
    assert e.value.code == 2
    memb = ob.members(w.pos, w.n_active, w.problem, ng, blocks)
    assert e.value.needed == sum(len(a) + len(p) for a, p in memb)
    with pytest.raises(_sr.SRError):  # nothing to gather after a failed partition
        plan.gather(pos, mass, ws)
    plan.close()
    bf = BlockForce(w.problem, blocks, w.n, w.n_active, ng=ng, capacity=w.n, device=DEV,
                    tune_cache=None)
    acc = bf.forward(pos, mass).cpu().numpy()
    bf2 = BlockForce(w.problem, blocks, w.n, w.n_active, ng=ng, device=DEV, tune_cache=None)
    assert np.array_equal(acc, bf2.forward(pos, mass).cpu().numpy())
    bf.close()
    bf2.close()


def test_empty_blocks_and_all_passive():
    # every particle in one corner: most blocks are empty; then no active ones
    w = synth.uniform_box(3000, 6.0, 11)
    w.problem = synth.Problem.make((0, 0, 0), (30.0, 30.0, 30.0), False, 3.0, 0.05, w.problem.poly)
    ng = (30, 30)
    blocks = equal_blocks(ng, 5, 5)
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    bf = BlockForce(w.problem, blocks, w.n, 2000, ng=ng, device=DEV, tune_cache=None)
    acc = bf.forward(pos, mass).cpu().numpy()
    assert np.sum(bf.counts.sum(axis=1) == 0) >= 16
    ref, _ = oracle.force(w.pos, w.mass, 2000, w.problem)
    assert_force_close(acc, ref, what="corner blocks")
    bf.close()
    bf = BlockForce(w.problem, blocks, w.n, 0, ng=ng, device=DEV, tune_cache=None)
    assert bf.forward(pos, mass).shape == (0, 3)
    assert np.all(bf.counts[:, 0] == 0)
    bf.close()


def test_refinement_by_pair_counts_stays_exact():
    # a clustered slab: equal 2x2 blocks, then Sec. 2.1's rule (split a block
    # costing more than twice the mean) for a few rounds by pair counts; the
    # irregular blocks that result still give the oracle's forces
    from paper_1411_3396_amd.blocks import balanced_blocks, equal_blocks as eq, refine as rf

    w = synth.slab_with_ghosts(24, 3.0, 12, 3)
    ng = grid_units(w.problem)
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    blocks, history = balanced_blocks(pos, mass, w.problem, w.n_active, nbx=2, nby=2, kind="pairs",
                                      max_rounds=4, ng=ng)
    announce(f"refined blocks: {len(history)} rounds, {len(blocks)} blocks")
    # replay the rule on the recorded costs: the same blocks come out
    replay = eq(ng, 2, 2)
    for cost in history:
        nxt = rf(replay, cost)
        if nxt == replay:
            break
        replay = nxt
    assert replay == blocks and len(blocks) > 4
    assert history[0].max() > 2.0 * history[0].mean()
    bf = BlockForce(w.problem, blocks, w.n, w.n_active, ng=ng, device=DEV, tune_cache=None)
    acc = bf.forward(pos, mass).cpu().numpy()
    times = bf.block_costs(pos, mass, kind="time", repeats=1)
    assert np.all(times[bf.counts[:, 0] > 0] > 0)
    bf.close()
    ref, _ = oracle.force(w.pos, w.mass, w.n_active, w.problem)
    assert_force_close(acc, ref, what="refined blocks")
