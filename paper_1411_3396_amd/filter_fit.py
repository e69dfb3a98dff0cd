"""Project-owned fit of the short-range filter polynomial.

The method splits the gravitational force into a long-range part, solved on a
spectrally filtered particle-mesh grid, and a short-range remainder summed
directly over particle pairs (Sec. 2, "HACC and Accelerated Systems").  The
short-range pair kernel used here is

    f_SR(s) = (s + eps^2)^(-3/2) - sum_k c_k s^k ,   s = r^2 ,

i.e. the Plummer-softened Newtonian kernel minus a degree-5 polynomial in s
that stands for the part the grid already resolves.  The paper does not print
the filter or its coefficients (it defers the solver details to the HACC
method papers), so the coefficients are a run-time argument of the library and
of the oracle, and the values used for the synthetic workloads come from this
fit, not from HACC:

* target: the long-range kernel of a Gaussian force split,
  F_long(r)/r = r^-3 [erf(r/2sigma) - r/(sigma sqrt(pi)) exp(-r^2/4sigma^2)];
* least squares in s, weighted by r, over r in (0, r_s];
* one equality constraint, P(r_s^2) = (r_s^2 + eps^2)^(-3/2), so that the
  short-range kernel is continuous and vanishes at the cutoff.

Run as a script to regenerate ``filter_coeffs.json``.  The frozen file is an
input of the workloads; nothing here is evaluated on the force path.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

SIGMA = 0.6
DEGREE = 5
N_SAMPLES = 4000
_HERE = os.path.dirname(os.path.abspath(__file__))
COEFF_FILE = os.path.join(_HERE, "filter_coeffs.json")


def long_range_kernel(r: np.ndarray, sigma: float = SIGMA) -> np.ndarray:
    """F_long(r)/r for a unit point mass smoothed by a Gaussian of width sigma."""
    r = np.asarray(r, dtype=np.float64)
    x = r / (2.0 * sigma)
    out = np.empty_like(r)
    small = x < 0.5
    # series of erf(x) - 2x/sqrt(pi) exp(-x^2), divided by r^3 = 8 sigma^3 x^3
    xs = x[small]
    acc = np.zeros_like(xs)
    term_x = np.ones_like(xs)  # x^(2n-2)
    fact = 1.0
    for n in range(1, 16):
        fact *= n
        coef = (-1.0) ** (n + 1) * (2.0 * n) / (fact * (2.0 * n + 1.0))
        acc += coef * term_x
        term_x = term_x * xs * xs
    out[small] = (2.0 / math.sqrt(math.pi)) * acc / (8.0 * sigma ** 3)
    xl = x[~small]
    rl = r[~small]
    from scipy.special import erf

    out[~small] = (erf(xl) - (2.0 * xl / math.sqrt(math.pi)) * np.exp(-xl * xl)) / rl ** 3
    return out


def fit(r_s: float, eps: float, sigma: float = SIGMA) -> np.ndarray:
    """Return c_0..c_5 (float64) for cutoff r_s and Plummer length eps."""
    r = r_s * (np.arange(N_SAMPLES) + 0.5) / N_SAMPLES
    z = (r / r_s) ** 2  # scaled variable in [0, 1] for conditioning
    A = np.vander(z, DEGREE + 1, increasing=True)
    b = long_range_kernel(r, sigma)
    w = r
    AtW = A.T * w
    G = AtW @ A
    h = AtW @ b
    # equality constraint at z = 1
    a_c = np.ones(DEGREE + 1)
    d = (r_s * r_s + eps * eps) ** -1.5
    K = np.zeros((DEGREE + 2, DEGREE + 2))
    K[: DEGREE + 1, : DEGREE + 1] = G
    K[: DEGREE + 1, DEGREE + 1] = a_c
    K[DEGREE + 1, : DEGREE + 1] = a_c
    rhs = np.concatenate([h, [d]])
    sol = np.linalg.solve(K, rhs)
    gamma = sol[: DEGREE + 1]
    return np.array([gamma[k] / (r_s * r_s) ** k for k in range(DEGREE + 1)])


def key(r_s: float, eps: float) -> str:
    return f"rs={r_s:g},eps={eps:g}"


def load(r_s: float, eps: float) -> np.ndarray:
    """Frozen coefficients for (r_s, eps) as float64 (pass float32 to the solvers)."""
    with open(COEFF_FILE) as fh:
        table = json.load(fh)
    return np.array(table["coeffs"][key(r_s, eps)], dtype=np.float64)


def main() -> None:
    pairs = [(3.0, 0.05), (3.0, 0.02), (3.0, 0.01)]
    table = {
        "form": "f_SR(s) = (s+eps^2)^-1.5 - sum_k c[k] s^k, s = r^2, lengths in grid cells",
        "target": "Gaussian force split, long-range kernel, sigma=%g" % SIGMA,
        "constraint": "sum_k c[k] r_s^(2k) = (r_s^2+eps^2)^-1.5",
        "coeffs": {key(rs, e): [float(c) for c in fit(rs, e)] for rs, e in pairs},
    }
    with open(COEFF_FILE, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    print(json.dumps(table, indent=1))


if __name__ == "__main__":
    main()
