"""Shared helpers of the GPU tests (no test functions here)."""
import numpy as np
import torch

import oracle
import paper_1411_3396_amd as sr

DEV = "cuda:0"
FWD_TOL = 1e-5  # RMS relative force error against float64
VJP_TOL = 1e-4  # RMS relative gradient error against float64


def announce(msg: str) -> None:
    print(f"[gpu case] {msg}", flush=True)


def to_dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_force(w, **kw) -> np.ndarray:
    acc = sr.force(to_dev(w.pos), to_dev(w.mass), w.problem, w.n_active, **kw)
    torch.cuda.synchronize()
    return acc.cpu().numpy()


def gpu_vjp(w, g, **kw) -> np.ndarray:
    out = sr.force_vjp(to_dev(w.pos), to_dev(w.mass), w.problem, to_dev(g), w.n_active, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_force(w, targets=None):
    acc, _ = oracle.force(w.pos, w.mass, w.n_active, w.problem, targets)
    return acc


def assert_force_close(gpu, ref, tol=FWD_TOL, what=""):
    err = oracle.rms_rel(gpu, ref)
    print(f"  {what} rms_rel={err:.3e}", flush=True)
    assert np.all(np.isfinite(gpu)), what
    assert err <= tol, (what, err)
    scale = np.median(np.linalg.norm(ref, axis=1)) + 1e-30
    row = np.linalg.norm(gpu - ref, axis=1)
    assert np.all(row <= 1e-3 * (np.linalg.norm(ref, axis=1) + scale)), (what, row.max())
    return err
