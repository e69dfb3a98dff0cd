"""Power spectrum of the particle distribution, written out from its
definition in numpy float64 (test infrastructure only).

What it computes (paper Sec. 4.1: particles are deposited onto a grid with
cloud-in-cell assignment, a discrete Fourier transform gives delta(k),
P(k) = |delta(k)|^2 is averaged in bins of |k|, and the CIC smoothing is
compensated by dividing by the assignment's window function):

* deposit: grid points sit at integer multiples of the cell size h = box/ng;
  a particle at u = x/h (periodic, in [0, ng)) gives mass m (1 - f) to point
  floor(u) and m f to point floor(u) + 1 along each axis, f = u - floor(u),
  the product of the three axes' weights to each of the 8 points;
* delta(x) = rho(x) / mean(rho) - 1;  delta(k) = sum_x delta(x) exp(-i k.x)
  (unnormalised forward DFT);  P(k) = |delta(k)|^2 box^3 / ng^6, divided by
  the CIC window W(k)^2, W = prod_d sinc^2(pi n_d / ng), sinc(x) = sin(x)/x,
  n_d the integer mode index in (-ng/2, ng/2];
* bins: b = floor(|n| / dn) for |n| = sqrt(n_x^2 + n_y^2 + n_z^2) in units of
  the fundamental 2 pi / box; the k = 0 mode is left out; every mode of the
  full grid counts once.
"""
from __future__ import annotations

import numpy as np


def cic_deposit(pos, mass, ng: int, box: float) -> np.ndarray:
    """Mass on the ng^3 grid, float64, indexed [ix, iy, iz]."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    mass = np.asarray(mass, np.float64).reshape(-1)
    u = np.mod(pos / (box / ng), ng)
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    i0 %= ng  # u can round up to ng
    rho = np.zeros((ng, ng, ng), np.float64)
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1.0 - f[:, 0]
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1.0 - f[:, 1]
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                np.add.at(rho, ((i0[:, 0] + cx) % ng, (i0[:, 1] + cy) % ng, (i0[:, 2] + cz) % ng),
                          mass * wx * wy * wz)
    return rho


def mode_indices(ng: int) -> np.ndarray:
    """Integer mode index of each FFT frequency: 0, 1, ..., ng/2, -(ng/2 - 1), ..., -1."""
    n = np.fft.fftfreq(ng, d=1.0 / ng).round().astype(np.int64)
    if ng % 2 == 0:
        n[ng // 2] = ng // 2  # the Nyquist mode as +ng/2
    return n


def cic_window(ng: int) -> np.ndarray:
    """W(n) = prod_d sinc^2(pi n_d / ng) on the full grid of modes."""
    n = mode_indices(ng).astype(np.float64)
    s = np.ones(ng)
    nz = n != 0
    x = np.pi * n[nz] / ng
    s[nz] = (np.sin(x) / x) ** 2
    return s[:, None, None] * s[None, :, None] * s[None, None, :]


def power_spectrum(rho: np.ndarray, box: float, n_bins: int, dn: float = 1.0):
    """(P per bin, mean |k| per bin, modes per bin) from a mass grid.

    k is in units of the fundamental 2 pi / box times the bin's mean |n|; empty
    bins give P = 0 and |k| = 0."""
    ng = rho.shape[0]
    delta = rho / rho.mean() - 1.0
    dk = np.fft.fftn(delta)
    p = (np.abs(dk) ** 2) * box ** 3 / float(ng) ** 6 / cic_window(ng) ** 2
    n = mode_indices(ng).astype(np.float64)
    mag = np.sqrt(n[:, None, None] ** 2 + n[None, :, None] ** 2 + n[None, None, :] ** 2)
    b = np.floor(mag / dn).astype(np.int64)
    keep = (mag > 0) & (b < n_bins)
    cnt = np.bincount(b[keep], minlength=n_bins).astype(np.int64)
    psum = np.bincount(b[keep], weights=p[keep], minlength=n_bins)
    ksum = np.bincount(b[keep], weights=mag[keep], minlength=n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        pk = np.where(cnt > 0, psum / cnt, 0.0)
        km = np.where(cnt > 0, ksum / cnt, 0.0)
    return pk, km * (2.0 * np.pi / box), cnt
