"""Adjoint parity: the HIP vector-Jacobian product against the float64 oracle
adjoint (RMS relative error <= 1e-4), the autograd wrapper, and central
finite differences of the float64 forward sum on local subproblems."""
import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

import oracle
import paper_1411_3396_amd as sr
from paper_1411_3396_amd import synth
from gpu_helpers import DEV, VJP_TOL, announce, gpu_vjp, to_dev

pytestmark = pytest.mark.gpu


def cases():
    return {
        "uniform_periodic": lambda: synth.uniform_box(30000, 31.0, 2),
        "clustered_periodic": lambda: synth.clustered_box(65536, 40.0, 61, 3),
        "slab_ghosts": lambda: synth.slab_with_ghosts(32, 3.0, 200, 4),
    }


@pytest.mark.parametrize("name", list(cases()))
def test_vjp_matches_oracle(name):
    w = cases()[name]()
    w.mass = np.random.default_rng(5).uniform(0.5, 2.0, w.n).astype(np.float32)
    g = synth.cotangent(w.n_active, 1)
    announce(f"vjp {name} n={w.n} n_active={w.n_active}")
    got = gpu_vjp(w, g)
    ref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g)
    err = oracle.rms_rel(got, ref)
    print(f"  vjp {name} rms_rel={err:.3e}", flush=True)
    assert np.all(np.isfinite(got)) and err <= VJP_TOL


def test_vjp_unsoftened():
    rng = np.random.default_rng(8)
    w = synth.uniform_box(1, 20.0, 0)
    w.pos = (rng.random((6000, 3)) * 20.0).astype(np.float32)
    w.mass = np.ones(6000, np.float32)
    w.n_active = 6000
    w.problem = synth.Problem.make((0, 0, 0), (20.0,) * 3, True, 3.0, 0.0, synth.filter_poly(3.0, 0.05))
    g = synth.cotangent(6000, 2)
    announce("vjp eps=0")
    got = gpu_vjp(w, g)
    ref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g)
    assert oracle.rms_rel(got, ref) <= VJP_TOL


def test_autograd_function_uses_the_vjp():
    w = synth.slab_with_ghosts(20, 3.0, 40, 7)
    pos = to_dev(w.pos).requires_grad_(True)
    mass = to_dev(w.mass)
    g = to_dev(synth.cotangent(w.n_active, 3))
    announce("autograd")
    acc = sr.sr_force(pos, mass, w.problem, w.n_active)
    (grad,) = torch.autograd.grad(acc, pos, g)
    direct = sr.force_vjp(to_dev(w.pos), mass, w.problem, g, w.n_active)
    assert torch.equal(grad, direct)
    ref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g.cpu().numpy())
    assert oracle.rms_rel(grad.cpu().numpy(), ref) <= VJP_TOL


def test_vjp_linear_in_cotangent():
    w = synth.uniform_box(20000, 27.0, 9)
    g = synth.cotangent(w.n, 4)
    a = gpu_vjp(w, g)
    b = gpu_vjp(w, 2.0 * g)
    assert np.array_equal((2.0 * a).view(np.uint32), b.view(np.uint32))


def local_fd(w, k, g, h):
    """Central difference of L = sum_i g_i . a_i with respect to x_k, in float64.

    Only pair terms with k change, so the loss is evaluated on a local
    subproblem: particles within 2 r_s + 2h of x_k (minimum image, shifted to
    an open domain), targets = k and its neighbours."""
    P = w.problem
    L = np.array(P.len, np.float64)
    x = w.pos.astype(np.float64)
    d = x - x[k]
    if P.periodic:
        d -= L * np.round(d / L)
    r = np.sqrt(np.sum(d * d, axis=1))
    sel = np.nonzero(r < 2 * P.r_s + 4 * h)[0]
    near = sel[r[sel] < P.r_s + 2 * h]
    act = near[near < w.n_active]
    order = np.concatenate([act, np.setdiff1d(sel, act)])
    xl = d[order] + 100.0
    ml = w.mass[order].astype(np.float64)
    gl = g[act].astype(np.float64)
    lp = synth.Problem.make((0, 0, 0), (200.0,) * 3, False, P.r_s, P.eps, P.poly)
    kk = int(np.nonzero(order == k)[0][0])
    out = np.zeros(3)
    for a in range(3):
        xp = xl.copy()
        xp[kk, a] += h
        xm = xl.copy()
        xm[kk, a] -= h
        ap, _ = oracle.force(xp, ml, len(act), lp)
        am, _ = oracle.force(xm, ml, len(act), lp)
        out[a] = np.sum(gl * (ap - am)) / (2 * h)
    return out, r[(r > 0) & (r < P.r_s + 4 * h)]


def test_vjp_against_finite_differences():
    w = synth.clustered_box(200000, 60.0, 200, 11)
    g = synth.cotangent(w.n_active, 1)
    idx = synth.sample_indices(w.n, 256, 2)
    announce("vjp vs finite differences")
    got = gpu_vjp(w, g)[idx]
    h = 1e-3
    fd = []
    keep = []
    for q, k in enumerate(idx):
        f1, rr = local_fd(w, int(k), g, h)
        if np.any(np.abs(rr - w.problem.r_s) < 2 * h):
            continue  # a pair would cross the cutoff
        f2, _ = local_fd(w, int(k), g, h / 2)
        fd.append((4 * f2 - f1) / 3)  # Richardson: error O(h^4)
        keep.append(q)
    fd = np.array(fd)
    err = oracle.rms_rel(got[keep], fd)
    print(f"  fd points={len(keep)} rms_rel={err:.3e}", flush=True)
    assert len(keep) >= 100 and err <= VJP_TOL


@pytest.mark.parametrize("eps,masses", [(0.01, "random"), (0.02, "random"), (0.01, "equal")])
def test_vjp_duplicated_positions_per_particle(eps, masses):
    # 400 particles placed exactly on others: the target's own entry must add
    # exactly zero (u is exactly antisymmetric), and a distinct particle at the
    # same position adds f(0) u, the derivative of its smooth softened force
    # term.  Checked per particle, not only in RMS: the own entry's rounding
    # would be amplified by f(0) ~ eps^-3 on every row.
    rng = np.random.default_rng(14)
    w = synth.uniform_box(30000, 31.0, 13)
    dst = rng.choice(w.n, 400, replace=False)
    src = rng.choice(np.setdiff1d(np.arange(w.n), dst), 400, replace=False)
    w.pos[dst] = w.pos[src]
    w.mass = (rng.uniform(0.5, 2.0, w.n) if masses == "random" else np.ones(w.n)).astype(np.float32)
    w.problem = synth.Problem.make((0, 0, 0), (31.0,) * 3, True, 3.0, eps, synth.filter_poly(3.0, eps))
    g = synth.cotangent(w.n, 6)
    announce(f"vjp duplicates eps={eps} masses={masses}")
    got = gpu_vjp(w, g)
    ref = oracle.vjp(w.pos, w.mass, w.n, w.problem, g)
    err = oracle.rms_rel(got, ref)
    row = np.linalg.norm(got - ref, axis=1)
    mag = np.linalg.norm(ref, axis=1)
    med = np.median(mag)
    worst = np.max(row / (mag + 0.1 * med))
    print(f"  rms_rel={err:.3e} worst row={worst:.3e} median row rel={np.median(row / mag):.3e}", flush=True)
    assert err <= VJP_TOL
    assert worst <= 1e-4
    # the forward sum is unchanged by the duplicates' zero separation
    a = sr.force(to_dev(w.pos), to_dev(w.mass), w.problem).cpu().numpy()
    aref, _ = oracle.force(w.pos, w.mass, w.n, w.problem)
    assert oracle.rms_rel(a, aref) <= 1e-5


def test_adjoint_pair_count_has_an_active_end():
    # the adjoint evaluates the ordered pairs with at least one active end:
    # all pairs of the domain minus those between two passive particles (both
    # counted by the oracle); the forward those with an active target
    w = synth.slab_with_ghosts(40, 3.0, 300, 2)
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    ws = sr.bin(pos, mass, w.problem, w.n_active)
    fwd = int(sr.count_pairs(ws, w.n, w.problem, w.n_active).item())
    adj = int(sr.count_pairs(ws, w.n, w.problem, w.n_active, adjoint=True).item())
    _, ref_fwd = oracle.force(w.pos, w.mass, w.n_active, w.problem)
    _, ref_all = oracle.force(w.pos, w.mass, w.n, w.problem)
    npas = w.n - w.n_active
    _, ref_pp = oracle.force(w.pos[w.n_active:], w.mass[w.n_active:], npas, w.problem)
    announce(f"pairs forward {fwd} ({ref_fwd}) adjoint {adj} ({ref_all - ref_pp}), passive-passive {ref_pp}")
    assert ref_pp > 0 and w.n_active < w.n
    assert abs(fwd - ref_fwd) <= 4
    assert abs(adj - (ref_all - ref_pp)) <= 4
    # the adjoint's gradients on the passive rows still match the oracle
    g = synth.cotangent(w.n_active, 9)
    got = sr.force_vjp(pos, mass, w.problem, to_dev(g), w.n_active, ws=ws, reuse_bins=True).cpu().numpy()
    ref = oracle.vjp(w.pos, w.mass, w.n_active, w.problem, g)
    assert oracle.rms_rel(got[w.n_active:], ref[w.n_active:]) <= VJP_TOL
    assert oracle.rms_rel(got, ref) <= VJP_TOL
