"""Benchmark of the short-range force path on one MI355X.

One step = the whole hot path over the node-share workload (320^3 active
cells plus a 3-cell ghost shell, 34.6M particles, strongly clustered):
binning, forward force, adjoint (vector-Jacobian product with a fixed N(0,1)
cotangent) and the float64 momentum check.  Inputs are resident in HBM before
the timed region.  Prints one JSON line.

value = pair interactions per second over the whole step: (useful pairs of
the forward pass + useful pairs of the adjoint pass) / step time.  A useful
pair is an ordered (target, source) pair with 0 < r < r_s; the forward's have
an active target, the adjoint's at least one active end (a pair of two ghosts
adds exactly nothing to the gradient and is not evaluated).  A pass (forward
or adjoint) is three kernels: the one-sided items, the symmetric tiles of the
dense cells and the gather of their partial sums, timed together with HIP
events on the launch stream.  The forward pass's own rate (useful forward
pairs / forward pass time) is forward_pairs_per_s.  `roofline` is the
dominant pass's (the adjoint's, the longest), with both passes under
roofline_forward and roofline_adjoint.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3  # TFLOP/s, MI355X (packed), 256 CUs x 2.4 GHz x 256 flop/clk
PEAK_FP32_NONPACKED = 78.6  # TFLOP/s, one float32 FMA per lane per clock
FLOP_PER_PAIR = {"force": 30, "vjp": 61}
# the kernels of one pass: one-sided items (sparse cells, remainders and the
# non-dense sources of dense blocks), symmetric tiles of the dense cells, and
# the gather of the symmetric partial sums
PASS_KERNELS = {"force": ["k_force", "k_force_sym", "k_sym_gather"],
                "vjp": ["k_vjp", "k_vjp_sym", "k_sym_gather"]}
PASS_NAME = {"force": "forward", "vjp": "adjoint"}


# In-cell leaf order the workloads are timed at (octree depth; 1 = octants).
LEAF_DEPTH = 2


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_code_hash() -> str:
    """sha256 prefix of the pair kernels' code: sr_kernels.hip with its comments removed and its
    blank space collapsed, so that a counter summary stays valid across comment-only edits."""
    with open(os.path.join(ROOT, "paper_1411_3396_amd", "csrc", "sr_kernels.hip")) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"\s+", " ", src).strip()
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def committed_profile(kind: str, kernel: str, workload: str):
    """A committed rocprofv3 counter summary of one pass (profiles/<kind>_<pass>_<workload>.json),
    if it was taken on this kernel code; else None."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{PASS_NAME[kernel]}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_code_sha256_16") != kernel_code_hash():
        return None
    return t


def measured_traffic(kernel: str, workload: str):
    """HBM bytes of one pass (all its kernels) from committed FETCH_SIZE / WRITE_SIZE runs."""
    t = committed_profile("traffic", kernel, workload)
    return None if t is None else t.get("bytes_per_pass")


def cpu_baseline(w, g, target_seconds: float):
    """The float64 oracle on a random sample of active targets of the same workload."""
    import oracle

    rng = np.random.default_rng(7)
    pilot = np.sort(rng.choice(w.n_active, size=min(20000, w.n_active), replace=False))
    t0 = time.perf_counter()
    _, pairs = oracle.force(w.pos, w.mass, w.n_active, w.problem, targets=pilot)
    t_pilot = time.perf_counter() - t0
    rate = pairs / max(t_pilot, 1e-9)
    # forward + adjoint on the same sample, sized for about target_seconds
    want = int(min(w.n_active, max(20000, target_seconds / 2.0 * rate / max(pairs / len(pilot), 1))))
    sample = np.sort(rng.choice(w.n_active, size=want, replace=False))
    t0 = time.perf_counter()
    _, pairs = oracle.force(w.pos, w.mass, w.n_active, w.problem, targets=sample)
    t1 = time.perf_counter()
    oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g, targets=sample)
    t2 = time.perf_counter()
    out = {"value": 2.0 * pairs / (t2 - t0), "unit": "pair interactions/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"{want} random active targets of {w.name} (seed 7), forward + adjoint, "
                     f"float64 cell list incl. its own binning of all {w.n} particles per call; "
                     f"{pairs} useful pairs per pass, {t1 - t0:.1f} s + {t2 - t1:.1f} s"}
    # one host thread, on a sample sized for a few seconds of pair work
    one = np.sort(rng.choice(w.n_active, size=max(2000, want // (4 * max(1, oracle.num_threads()))),
                             replace=False))
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        _, p1 = oracle.force(w.pos, w.mass, w.n_active, w.problem, targets=one)
        t1 = time.perf_counter()
        oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g, targets=one)
        t2 = time.perf_counter()
    finally:
        oracle.set_num_threads(threads)
    out["single_thread"] = {"value": 2.0 * p1 / (t2 - t0), "unit": "pair interactions/s", "cores": 1,
                            "sample": f"{len(one)} random active targets (seed 7), forward + adjoint, "
                                      f"{p1} useful pairs per pass, {t1 - t0:.1f} s + {t2 - t1:.1f} s "
                                      f"(binning of all particles included)"}
    return out


def batch_comparison(reps: int = 5):
    """Batched persistent launch (graph) against one launch sequence per subvolume."""
    import torch

    import paper_1411_3396_amd as sr
    from paper_1411_3396_amd import synth

    b = synth.subvolumes_96()
    dev = "cuda:0"
    pos = torch.from_numpy(b.pos).to(dev)
    mass = torch.from_numpy(b.mass).to(dev)
    plan = sr.BatchPlan(b.offsets, b.n_active, b.problems, tune_cache=sr._sr.default_tune_cache())
    ws = sr.new_workspace(plan.ws_bytes, dev)
    acc = torch.empty((plan.total_active, 3), device=dev)
    mom = torch.empty((plan.B, 3), dtype=torch.float64, device=dev)
    out = {}
    for mode in ("graph", "per_subvolume"):
        plan.run(pos, mass, ws, acc, mom, mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.run(pos, mass, ws, acc, mom, mode)
        torch.cuda.synchronize()
        out[mode] = 1e3 * (time.perf_counter() - t0) / reps
    info = plan.info()
    plan.close()
    return {"workload": b.name, "subvolumes": b.size, "n": int(b.offsets[-1]),
            "ms_graph": round(out["graph"], 3), "ms_per_subvolume": round(out["per_subvolume"], 3),
            "speedup": round(out["per_subvolume"] / out["graph"], 3),
            "waves_per_cu": info["waves_per_cu"], "sym_blocks": info["sym_blocks"],
            "sym_window": info["sym_window"], "sparse_group": info["sparse_group"]}


def block_comparison(w, pos, mass, acc_mono, reps: int = 3):
    """Overlapping data blocks of the same domain: equal partitions in grid
    units, each solved as one batched launch and reconciled."""
    import torch

    from paper_1411_3396_amd.blocks import BlockForce, equal_blocks, grid_units

    ng = grid_units(w.problem)
    ref = acc_mono.double()
    out = []
    for nbx in (2, 4):
        blocks = equal_blocks(ng, nbx, nbx)
        bf = BlockForce(w.problem, blocks, w.n, w.n_active, ng=ng, device=pos.device)
        acc = bf.forward(pos, mass)  # first run: batch plan tuning
        times = {}
        for _ in range(reps):
            acc = bf.forward(pos, mass, times=times)
        diff = (acc.double() - ref).norm() / ref.norm()
        out.append({"blocks": f"{nbx}x{nbx}", "members_per_particle": round(bf.plan.members / w.n, 4),
                    "ms": {k: round(v / reps, 3) for k, v in times.items()},
                    "ms_total": round(sum(times.values()) / reps, 3),
                    "rel_diff_vs_single_domain": float(diff)})
        log(f"blocks {nbx}x{nbx}: {out[-1]}")
        bf.close()
        del bf, acc
        torch.cuda.empty_cache()
    return out


def leaf_comparison(w, reps: int = 3, depths=(1, 2, 3, 4)):
    """Bin, forward and adjoint kernel times of one workload with the cells
    ordered by the leaves of an octree of each depth (depth 1: octants)."""
    import torch

    import paper_1411_3396_amd as sr
    from paper_1411_3396_amd import synth

    dev = "cuda:0"
    pos = torch.from_numpy(w.pos).to(dev)
    mass = torch.from_numpy(w.mass).to(dev)
    g = torch.from_numpy(synth.cotangent(w.n_active, 1)).to(dev)
    acc = torch.empty((w.n_active, 3), device=dev)
    grad = torch.empty((w.n, 3), device=dev)
    out = {"workload": w.name, "n": w.n}
    for d in depths:
        prob = w.problem.with_leaf_depth(d)
        try:
            ws = sr.new_workspace(sr.workspace_bytes(w.n, prob), dev)
        except sr.SRError as e:
            out[f"depth{d}"] = str(e)
            continue
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        sr.bin(pos, mass, prob, w.n_active, ws=ws)
        sr.force(pos, mass, prob, w.n_active, ws=ws, reuse_bins=True, out=acc)
        sr.force_vjp(pos, mass, prob, g, w.n_active, ws=ws, reuse_bins=True, out=grad)
        torch.cuda.synchronize()
        bin_ms = 0.0
        sr.timing_enable(True)
        for _ in range(reps):
            ev[0].record()
            sr.bin(pos, mass, prob, w.n_active, ws=ws)
            ev[1].record()
            sr.force(pos, mass, prob, w.n_active, ws=ws, reuse_bins=True, out=acc)
            sr.force_vjp(pos, mass, prob, g, w.n_active, ws=ws, reuse_bins=True, out=grad)
            torch.cuda.synchronize()
            bin_ms += ev[0].elapsed_time(ev[1])
        f_ms, f_n = sr.timing_read("force")
        v_ms, v_n = sr.timing_read("vjp")
        sr.timing_enable(False)
        out[f"depth{d}"] = {"bin_ms": round(bin_ms / reps, 3), "force_ms": round(f_ms / f_n, 3),
                            "vjp_ms": round(v_ms / v_n, 3)}
        log(f"leaves {w.name} depth {d}: {out[f'depth{d}']}")
        del ws
        torch.cuda.empty_cache()
    return out


FLOP_PER_POTENTIAL_PAIR = 12  # 3 sub, 3 FMA, rsqrt, 1 FMA


def centres_measure(reps: int = 3, cpu_seconds: float = 0.0):
    """Most-bound-particle centres of one node's halo catalogue (all pairs
    inside each halo), with the oracle on a sample of targets beside it."""
    import torch

    import paper_1411_3396_amd as sr
    from paper_1411_3396_amd import synth

    cat = synth.halos_node()
    dev = "cuda:0"
    pos = torch.from_numpy(cat.pos).to(dev)
    mass = torch.from_numpy(cat.mass).to(dev)
    plan = sr.CentresPlan(cat.offsets)
    ws = sr.new_workspace(plan.ws_bytes, dev)
    phi, mbp, pmin = plan.run(pos, mass, cat.eps, ws)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.run(pos, mass, cat.eps, ws, phi, mbp, pmin)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pairs = cat.pairs()
    rate = pairs / (ms * 1e-3)
    achieved = FLOP_PER_POTENTIAL_PAIR * rate / 1e12
    out = {"workload": cat.name, "n": cat.n, "halos": cat.n_halos, "largest_halo": cat.notes["max_halo"],
           "pairs": pairs, "ms": round(ms, 3), "pairs_per_s": rate,
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR, 4),
                        "flop_per_pair": FLOP_PER_POTENTIAL_PAIR}}
    plan.close()
    if cpu_seconds > 0:
        import oracle

        counts = np.diff(cat.offsets)
        # pilots grow the sample until one takes a tenth of the time asked for
        k, pilot = 200, 0.0
        while True:
            t = synth.sample_indices(cat.n, k, 9)
            t0 = time.perf_counter()
            oracle.halo_potential(cat.pos, cat.mass, cat.offsets, cat.eps, targets=t)
            pilot = time.perf_counter() - t0
            if pilot >= 0.1 * cpu_seconds or k >= cat.n:
                break
            k = min(cat.n, k * 4)
        k = int(min(cat.n, max(200, k * cpu_seconds / max(pilot, 1e-3))))
        t = synth.sample_indices(cat.n, k, 10)
        hid = np.searchsorted(cat.offsets, t, side="right") - 1
        t0 = time.perf_counter()
        oracle.halo_potential(cat.pos, cat.mass, cat.offsets, cat.eps, targets=t)
        el = time.perf_counter() - t0
        sp = int(np.sum(counts[hid] - 1))
        out["cpu_baseline"] = {"value": sp / el, "unit": "pair interactions/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{k} random particles of {cat.name}, each summed over its halo "
                                         f"({sp} pairs, {el:.1f} s)"}
    return out


def pk_measure(reps: int = 5, cpu_sample: int = 0):
    """Power spectrum on the fly (CIC deposit, FFT, bins) of the 16.7M-particle
    clustered box on 256^3 and 512^3 grids; with cpu_sample > 0 the oracle
    beside the 256^3 case (deposit timed on that many particles and scaled to
    all of them, spectrum timed on the full grid)."""
    import torch

    import paper_1411_3396_amd as sr
    from paper_1411_3396_amd import synth

    w = synth.clustered_16m()
    dev = "cuda:0"
    pos = torch.from_numpy(w.pos).to(dev)
    mass = torch.from_numpy(w.mass).to(dev)
    box = float(w.problem.len[0])
    out = []
    for ng in (256, 512):
        n_bins = ng // 2
        plan = sr.PkPlan(ng, box, n_bins, n_max=w.n)
        ws = sr.new_workspace(plan.ws_bytes, dev)
        plan.run(pos, mass, ws)  # first run: FFT plan
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        dep = tot = 0.0
        for _ in range(reps):
            e[0].record()
            plan.deposit(pos, mass, ws)
            e[1].record()
            plan.run(pos, mass, ws)
            e[2].record()
            e[2].synchronize()
            dep += e[0].elapsed_time(e[1])
            tot += e[1].elapsed_time(e[2])
        dep /= reps
        tot /= reps
        # deposit, algorithmic bytes: positions and masses in (16 B per particle),
        # the float32 grid out (4 B per point)
        alg = 16 * w.n + 4 * ng ** 3
        gbs = alg / (dep * 1e-3) / 1e9
        out.append({"workload": w.name, "ng": ng, "n": w.n, "ms": round(tot, 3), "ms_deposit": round(dep, 3),
                    "particles_per_s": w.n / (tot * 1e-3),
                    "deposit_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0,
                                         "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                                         "algorithmic_bytes": alg}})
        if cpu_sample > 0 and ng == 256:
            from oracle import pk as opk

            k = min(cpu_sample, w.n)
            t0 = time.perf_counter()
            rho = opk.cic_deposit(w.pos[:k], w.mass[:k], ng, box)
            t_dep = (time.perf_counter() - t0) * w.n / k
            t0 = time.perf_counter()
            opk.power_spectrum(rho, box, n_bins)
            t_spec = time.perf_counter() - t0
            out[-1]["cpu_baseline"] = {
                "value": w.n / (t_dep + t_spec), "unit": "particles/s", "cores": 1, "kind": "oracle",
                "sample": f"deposit of the first {k} particles timed ({t_dep * k / w.n:.1f} s) and scaled to "
                          f"{w.n}; spectrum of the {ng}^3 grid timed in full ({t_spec:.1f} s); numpy float64"}
        log(f"pk ng={ng}: {out[-1]}")
        plan.close()
        del ws
        torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="node_share")
    ap.add_argument("--cpu-seconds", type=float, default=40.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-blocks", action="store_true")
    ap.add_argument("--no-centres", action="store_true")
    ap.add_argument("--no-pk", action="store_true")
    ap.add_argument("--no-leaves", action="store_true")
    ap.add_argument("--leaf-depth", type=int, default=LEAF_DEPTH,
                    help="octree depth of the in-cell order of the main workload (1: octants; 2, "
                         "4^3 leaves per cell, measured fastest on the node share)")
    ap.add_argument("--sweep", action="store_true",
                    help="time the pair kernels under every launch configuration "
                         "(waves per CU, targets per lane, occupancy variant); one JSON line each")
    ap.add_argument("--only", choices=["force", "vjp", "copy", "centres", "pk", "leaves"],
                    help="profiling mode: bin once, then run only this kernel --steps times "
                         "(copy: a 1 GiB device-to-device copy of known size; centres: the halo "
                         "catalogue's centre finder); prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the short-range path is "
              f"measured on one GPU's share of the domain", file=sys.stderr)
        return 2

    import torch

    import paper_1411_3396_amd as sr
    from paper_1411_3396_amd import synth

    dev = "cuda:0"
    if args.only == "pk":
        pk_measure(reps=args.steps)
        return 0
    if args.only == "centres":
        out = centres_measure(reps=args.steps)
        log(f"centres {args.steps} runs: {out['ms']} ms each")
        return 0
    if args.only == "leaves":
        for name in ("clustered_2m_extreme", args.workload):
            print(json.dumps(leaf_comparison(synth.get(name), reps=args.steps)), flush=True)
        return 0
    if args.only == "copy":
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.steps} x {a.numel() * 4} bytes")
        return 0
    t0 = time.perf_counter()
    w = synth.get(args.workload)
    w.problem = w.problem.with_leaf_depth(args.leaf_depth)
    g_np = synth.cotangent(w.n_active, 1)
    log(f"workload {w.name}: n={w.n} n_active={w.n_active} ({time.perf_counter() - t0:.1f} s to generate)")
    pos = torch.from_numpy(w.pos).to(dev)
    mass = torch.from_numpy(w.mass).to(dev)
    g = torch.from_numpy(g_np).to(dev)
    nb = sr.workspace_bytes(w.n, w.problem)
    ws = sr.new_workspace(nb, dev)
    acc = torch.empty((w.n_active, 3), device=dev)
    grad = torch.empty((w.n, 3), device=dev)
    mws = sr.new_workspace(1 << 20, dev)

    if args.only:
        sr.bin(pos, mass, w.problem, w.n_active, ws=ws)
        for _ in range(args.steps):
            if args.only == "force":
                sr.force(pos, mass, w.problem, w.n_active, ws=ws, reuse_bins=True, out=acc)
            else:
                sr.force_vjp(pos, mass, w.problem, g, w.n_active, ws=ws, reuse_bins=True, out=grad)
        torch.cuda.synchronize()
        log(f"ran {args.only} {args.steps} times")
        return 0

    if args.sweep:
        sr.bin(pos, mass, w.problem, w.n_active, ws=ws)
        saved = {k: sr.launch_config(kernel=k) for k in ("force", "vjp")}
        for waves in (16, 24, 32):
            for tpl in (1, 2):
                for occ in (0, 6, 8):
                    sr.launch_config(waves, tpl, occ)
                    for _ in range(args.warmup):
                        sr.force(pos, mass, w.problem, w.n_active, ws=ws, reuse_bins=True, out=acc)
                        sr.force_vjp(pos, mass, w.problem, g, w.n_active, ws=ws, reuse_bins=True, out=grad)
                    torch.cuda.synchronize()
                    sr.timing_enable(True)
                    for _ in range(args.steps):
                        sr.force(pos, mass, w.problem, w.n_active, ws=ws, reuse_bins=True, out=acc)
                        sr.force_vjp(pos, mass, w.problem, g, w.n_active, ws=ws, reuse_bins=True, out=grad)
                    torch.cuda.synchronize()
                    f_ms, f_n = sr.timing_read("force")
                    v_ms, v_n = sr.timing_read("vjp")
                    sr.timing_enable(False)
                    print(json.dumps({"waves_per_cu": waves, "targets_per_lane": tpl, "occupancy": occ,
                                      "force_ms": round(f_ms / f_n, 3), "vjp_ms": round(v_ms / v_n, 3)}),
                          flush=True)
        for k, v in saved.items():
            sr.launch_config(*v, kernel=k)
        return 0

    # useful pairs of both passes, counted once outside the timed region
    sr.bin(pos, mass, w.problem, w.n_active, ws=ws)
    pairs_fwd = int(sr.count_pairs(ws, w.n, w.problem, w.n_active).item())
    pairs_bwd = int(sr.count_pairs(ws, w.n, w.problem, w.n_active, adjoint=True).item())
    torch.cuda.synchronize()
    log(f"useful pairs: forward {pairs_fwd:.4e}, adjoint {pairs_bwd:.4e}")

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    phase = {"bin": 0.0, "force": 0.0, "vjp": 0.0, "momentum": 0.0}

    def step(record: bool):
        if record:
            ev[0].record()
        sr.bin(pos, mass, w.problem, w.n_active, ws=ws)
        if record:
            ev[1].record()
        sr.force(pos, mass, w.problem, w.n_active, ws=ws, reuse_bins=True, out=acc)
        if record:
            ev[2].record()
        sr.force_vjp(pos, mass, w.problem, g, w.n_active, ws=ws, reuse_bins=True, out=grad)
        if record:
            ev[3].record()
        mom = sr.momentum(acc, mass, ws=mws)
        if record:
            ev[4].record()
        return mom

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    sr.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(True)
        torch.cuda.synchronize()
        phase["bin"] += ev[0].elapsed_time(ev[1])
        phase["force"] += ev[1].elapsed_time(ev[2])
        phase["vjp"] += ev[2].elapsed_time(ev[3])
        phase["momentum"] += ev[3].elapsed_time(ev[4])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    kern = {}
    for k in ("force", "vjp"):
        ms, cnt = sr.timing_read(k)
        kern[k] = ms / max(cnt, 1)
    sr.timing_enable(False)
    ms_step = 1e3 * elapsed / args.steps
    for k in phase:
        phase[k] /= args.steps
    log(f"phases ms: {json.dumps({k: round(v, 3) for k, v in phase.items()})}; "
        f"kernels ms: {json.dumps({k: round(v, 3) for k, v in kern.items()})}")

    rate = (pairs_fwd + pairs_bwd) / (ms_step * 1e-3)
    flops = {"force": FLOP_PER_PAIR["force"] * pairs_fwd, "vjp": FLOP_PER_PAIR["vjp"] * pairs_bwd}

    def roof(k):
        achieved = flops[k] / (kern[k] * 1e-3) / 1e12
        r = {"bound": "alu", "kernel": " + ".join(PASS_KERNELS[k]), "achieved": round(achieved, 3),
             "peak": PEAK_FP32_VECTOR, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR, 4),
             "traffic": measured_traffic(k, w.name), "flop_per_useful_pair": FLOP_PER_PAIR[k],
             "kernel_ms": round(kern[k], 3)}
        # FP32 flops the VALU executed in one pass (rocprofv3 SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32,
        # 64 lanes x (ADD + MUL + TRANS + 2 FMA)), over the same time: counts each symmetric
        # pair term once and masked pair slots too
        c = committed_profile("flops", k, w.name)
        if c is not None:
            executed = c["executed_flop_per_pass"] / (kern[k] * 1e-3) / 1e12
            r["executed"] = round(executed, 3)
            r["executed_frac"] = round(executed / PEAK_FP32_VECTOR, 4)
        return r

    dominant = max(kern, key=lambda k: kern[k])
    result = {
        "metric": "short-range pair interactions/s (FP32) + backward/forward time ratio",
        "value": rate,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "n_active": w.n_active,
                   "n_ghost": w.n - w.n_active, "cells": int(np.prod(sr.grid(w.problem))),
                   "r_s": w.problem.r_s, "eps": round(w.problem.eps, 6), "periodic": w.problem.periodic,
                   "leaf_depth": w.problem.leaf_depth,
                   "step": "bin + force + adjoint + float64 momentum", "parallelism": "none"},
        "pairs_forward": pairs_fwd,
        "pairs_adjoint": pairs_bwd,
        "forward_pairs_per_s": pairs_fwd / (kern["force"] * 1e-3),
        "bwd_fwd_ratio_kernel": round(kern["vjp"] / kern["force"], 3),
        "bwd_fwd_ratio_step": round(phase["vjp"] / (phase["bin"] + phase["force"]), 3),
        "phase_ms": {k: round(v, 3) for k, v in phase.items()},
        "roofline": roof(dominant),
        "roofline_forward": roof("force"),
        "roofline_adjoint": roof("vjp"),
        "peak_fp32_nonpacked": PEAK_FP32_NONPACKED,
    }
    if not args.no_batch:
        log("batched vs per-subvolume")
        result["batch"] = batch_comparison()
    if not args.no_blocks and not w.problem.periodic:
        log("overlapping data blocks")
        result["blocks"] = block_comparison(w, pos, mass, acc)
        result["blocks_force_ms_single_domain"] = round(phase["bin"] + phase["force"], 3)
    if not args.no_leaves:
        log("tree-leaf order on the extreme-clustering box")
        result["leaves"] = leaf_comparison(synth.get("clustered_2m_extreme"))
    if not args.no_pk:
        log("power spectrum")
        result["pk"] = pk_measure(cpu_sample=0 if args.no_cpu_baseline else 4_000_000)
    if not args.no_centres:
        log("most-bound-particle centres")
        result["centres"] = centres_measure(cpu_seconds=0.0 if args.no_cpu_baseline else 10.0)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w, g_np, args.cpu_seconds)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
