"""Batched subvolumes: graph replay, eager batched and per-subvolume launches
agree bitwise, each subvolume matches the oracle, and the float64 momentum
sums match the returned accelerations."""
import numpy as np
import pytest
import torch

import oracle
import paper_1411_3396_amd as sr
from paper_1411_3396_amd import synth
from gpu_helpers import DEV, FWD_TOL, announce, assert_force_close, to_dev

pytestmark = pytest.mark.gpu


def mixed_batch():
    """Uneven periodic and open subvolumes, including empty and tiny ones."""
    parts = [synth.uniform_box(5000, 17.1, 1), synth.uniform_box(0, 12.0, 2),
             synth.uniform_box(40, 12.0, 3), synth.slab_with_ghosts(20, 3.0, 30, 4),
             synth.clustered_box(30000, 30.0, 25, 5), synth.uniform_box(1, 9.0, 6),
             synth.uniform_box(12000, 22.9, 7)]
    parts[3].mass = np.random.default_rng(0).uniform(0.5, 2, parts[3].n).astype(np.float32)
    pos = np.concatenate([p.pos for p in parts]).astype(np.float32)
    mass = np.concatenate([p.mass for p in parts]).astype(np.float32)
    offsets = np.concatenate([[0], np.cumsum([p.n for p in parts])]).astype(np.int64)
    n_act = np.array([p.n_active for p in parts], np.int64)
    return synth.Batch("mixed", pos, mass, offsets, n_act, [p.problem for p in parts])


def run(plan, b, mode, momentum=True):
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    acc = torch.full((plan.total_active, 3), float("nan"), device=DEV)
    mom = torch.full((plan.B, 3), float("nan"), dtype=torch.float64, device=DEV) if momentum else None
    plan.run(to_dev(b.pos), to_dev(b.mass), ws, acc, mom, mode)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), (mom.cpu().numpy() if momentum else None)


def test_modes_agree_bitwise_and_match_oracle():
    b = mixed_batch()
    plan = sr.BatchPlan(b.offsets, b.n_active, b.problems)
    announce(f"batch modes B={b.size} n={b.pos.shape[0]}")
    a_sub, m_sub = run(plan, b, "per_subvolume")
    a_eag, m_eag = run(plan, b, "eager")
    a_gra, m_gra = run(plan, b, "graph")
    assert np.array_equal(a_sub.view(np.uint32), a_eag.view(np.uint32))
    assert np.array_equal(a_eag.view(np.uint32), a_gra.view(np.uint32))
    np.testing.assert_array_equal(m_eag, m_gra)
    row = 0
    for k in range(b.size):
        part = b.part(k)
        rows = a_gra[row: row + part.n_active]
        if part.n_active:
            ref, _ = oracle.force(part.pos, part.mass, part.n_active, part.problem)
            if np.any(ref != 0):
                assert_force_close(rows, ref, what=f"subvolume {k}")
            else:
                assert np.all(rows == 0)
        mref = np.sum(part.mass[: part.n_active, None].astype(np.float64) * rows, axis=0)
        np.testing.assert_allclose(m_gra[k], mref, rtol=1e-9, atol=1e-9 * (np.abs(rows).sum() + 1))
        np.testing.assert_allclose(m_sub[k], mref, rtol=1e-9, atol=1e-9 * (np.abs(rows).sum() + 1))
        row += part.n_active
    info = plan.info()
    assert info["graph"] and info["waves_per_cu"] > 0
    plan.close()


def test_mixed_leaf_depths_agree_bitwise():
    # subvolumes with different in-cell octree depths in one batch: the
    # batched key holds the deepest code, each subvolume orders by its own
    b = mixed_batch()
    depths = [1, 3, 2, 4, 3, 1, 2]
    b.problems = [p.with_leaf_depth(d) for p, d in zip(b.problems, depths)]
    plan = sr.BatchPlan(b.offsets, b.n_active, b.problems)
    announce(f"batch leaf depths {depths}")
    a_sub, _ = run(plan, b, "per_subvolume")
    a_eag, _ = run(plan, b, "eager")
    a_gra, _ = run(plan, b, "graph")
    assert np.array_equal(a_sub.view(np.uint32), a_eag.view(np.uint32))
    assert np.array_equal(a_eag.view(np.uint32), a_gra.view(np.uint32))
    row = 0
    for k in range(b.size):
        part = b.part(k)
        if part.n_active:
            ref, _ = oracle.force(part.pos, part.mass, part.n_active, part.problem)
            if np.any(ref != 0):
                assert_force_close(a_gra[row: row + part.n_active], ref, what=f"subvolume {k} depth {depths[k]}")
        row += part.n_active
    plan.close()


def test_graph_replays_with_eager_work_between():
    b = mixed_batch()
    plan = sr.BatchPlan(b.offsets, b.n_active, b.problems)
    pos, mass = to_dev(b.pos), to_dev(b.mass)
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    acc = torch.empty((plan.total_active, 3), device=DEV)
    mom = torch.empty((plan.B, 3), dtype=torch.float64, device=DEV)
    plan.run(pos, mass, ws, acc, mom, "eager")
    ref = acc.clone()
    mref = mom.clone()
    announce("graph replays")
    for rep in range(4):
        acc.fill_(float("nan"))
        mom.fill_(float("nan"))
        plan.run(pos, mass, ws, acc, mom, "graph")
        torch.cuda.synchronize()
        assert torch.equal(acc, ref), rep
        assert torch.equal(mom, mref), rep
        # unrelated eager work on the same workspace in between
        sr.force(pos[:5000], mass[:5000], b.problems[0], ws=ws)
        torch.cuda.synchronize()
    # new output pointers: the captured graph is bound to the old ones, so a
    # graph run refuses them (SR_E_PLAN, nothing enqueued) unless asked to
    # capture again
    acc2 = torch.full_like(acc, float("nan"))
    with pytest.raises(sr.SRError) as err:
        plan.run(pos, mass, ws, acc2, mom, "graph")
    assert err.value.code == 4
    torch.cuda.synchronize()
    assert torch.isnan(acc2).all()
    plan.run(pos, mass, ws, acc2, mom, "graph", recapture=True)
    torch.cuda.synchronize()
    assert torch.equal(acc2, ref)
    # the new graph replays; the old pointers are refused in turn
    acc2.fill_(float("nan"))
    plan.run(pos, mass, ws, acc2, mom, "graph")
    torch.cuda.synchronize()
    assert torch.equal(acc2, ref)
    with pytest.raises(sr.SRError):
        plan.run(pos, mass, ws, acc, mom, "graph")
    plan.close()


def test_tune_cache_roundtrip(tmp_path):
    b = mixed_batch()
    path = str(tmp_path / "tune.json")
    p1 = sr.BatchPlan(b.offsets, b.n_active, b.problems, tune_cache=path)
    a1, _ = run(p1, b, "graph", momentum=False)
    w1 = p1.info()["waves_per_cu"]
    p2 = sr.BatchPlan(b.offsets, b.n_active, b.problems, tune_cache=path)
    a2, _ = run(p2, b, "graph", momentum=False)
    assert p2.info()["waves_per_cu"] == w1
    # the tuner also picks the symmetric tiles (blocks per item, window; 0 blocks = off)
    t1 = (p1.info()["sym_blocks"], p1.info()["sym_window"])
    assert t1 in {(16, 512), (16, 256), (64, 512), (4, 512), (0, 512)}
    assert (p2.info()["sym_blocks"], p2.info()["sym_window"]) == t1
    # and the targets per item of sparse cells
    assert p1.info()["sparse_group"] in {16, 32, 8}
    assert p2.info()["sparse_group"] == p1.info()["sparse_group"]
    assert np.array_equal(a1.view(np.uint32), a2.view(np.uint32))
    import json
    assert p1.info()["tune_key"] in json.load(open(path))


def test_batch_force_rejects_unknown_flags():
    # host validation before the workspace or any enqueue
    import ctypes as C
    b = mixed_batch()
    plan = sr.BatchPlan(b.offsets, b.n_active, b.problems)
    L = sr._sr.lib()
    fake = C.c_void_p(0x10000)
    assert L.sr_batch_force(plan._plan, fake, fake, fake, plan.ws_bytes, fake, None, 8, None) == 1
    assert L.sr_batch_force(plan._plan, fake, fake, None, plan.ws_bytes, fake, None, 4, None) == 2
    plan.close()


def test_dense_batch_symmetric_tiles_agree_bitwise():
    # subvolumes with dense cells: the symmetric tiles run in the batched launch
    # (the workspace header records it) and give the same bits as one launch
    # sequence per subvolume; each subvolume matches the oracle
    parts = [synth.clustered_box(65536, 40.0, 61, 0),
             synth.clustered_box(150000, 40.0, 80, 5, halo_frac=0.5, mass_range=(1e2, 1e4))]
    pos = np.concatenate([p.pos for p in parts]).astype(np.float32)
    mass = np.concatenate([p.mass for p in parts]).astype(np.float32)
    offsets = np.concatenate([[0], np.cumsum([p.n for p in parts])]).astype(np.int64)
    n_act = np.array([p.n_active for p in parts], np.int64)
    b = synth.Batch("dense", pos, mass, offsets, n_act, [p.problem for p in parts])
    plan = sr.BatchPlan(b.offsets, b.n_active, b.problems)
    announce(f"dense batch n={b.pos.shape[0]}")
    ws = sr.new_workspace(plan.ws_bytes, DEV)
    out = {}
    for mode in ("per_subvolume", "graph"):
        acc = torch.full((plan.total_active, 3), float("nan"), device=DEV)
        plan.run(to_dev(b.pos), to_dev(b.mass), ws, acc, None, mode)
        torch.cuda.synchronize()
        out[mode] = acc.cpu().numpy()
        if mode == "graph":
            assert int(ws[4 * 518:4 * 519].view(torch.int32).item()) == 1  # symmetric tiles ran
    assert np.array_equal(out["per_subvolume"].view(np.uint32), out["graph"].view(np.uint32))
    row = 0
    for k in range(b.size):
        part = b.part(k)
        ref, _ = oracle.force(part.pos, part.mass, part.n_active, part.problem)
        assert_force_close(out["graph"][row: row + part.n_active], ref, what=f"dense subvolume {k}")
        row += part.n_active
    plan.close()
