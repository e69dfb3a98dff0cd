"""Write oracle_values.json: oracle outputs on small fixed inputs, each next to
the closed form it must equal.  Calls only the oracle (and the seeded input
generators); rerun it after any deliberate change to the oracle's arithmetic.

Fixtures:
* short-range force (Sec. 2), Newtonian limit (no filter, no softening):
  a_0 = m_1 d / r^3 for two particles at several separations below r_s;
* most-bound particle (Sec. 2.2): the centre of a permuted 5x5x5 lattice;
* power spectrum (Sec. 4.1): a cosine density of amplitude A along x with
  mode 3 on a 16^3 grid, whose bin-3 power is 2 (A^2 box^3 / 4) / W^2 / modes.
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import pk  # noqa: E402
from paper_1411_3396_amd import synth  # noqa: E402


def force_cases():
    out = []
    prob = synth.Problem.make((0, 0, 0), (40.0, 40.0, 40.0), False, 3.0, 0.0, (0.0,) * 6)
    for r in (0.5, 1.0, 2.0, 2.9):
        pos = np.array([[10.0, 10.0, 10.0], [10.0 + r * 0.6, 10.0 + r * 0.8, 10.0]], np.float64)
        mass = np.array([1.0, 2.5])
        acc, pairs = oracle.force(pos, mass, 2, prob)
        d = pos[1] - pos[0]
        closed = (mass[1] * d / np.linalg.norm(d) ** 3).tolist()
        out.append({"r": r, "oracle_a0": acc[0].tolist(), "closed_form_a0": closed, "pairs": pairs})
    return out


def lattice_case():
    g = np.arange(5, dtype=float)
    pos = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T
    pos = pos[np.random.default_rng(0).permutation(len(pos))]
    phi = oracle.halo_potential(pos, np.ones(len(pos)), [0, len(pos)], 0.0)
    idx, val = oracle.most_bound(phi, [0, len(pos)])
    return {"most_bound_position": pos[idx[0]].tolist(), "phi_min": float(val[0]),
            "closed_form_position": [2.0, 2.0, 2.0]}


def plane_wave_case():
    ng, box, amp = 16, 50.0, 0.3
    x = np.arange(ng)
    rho = 1.0 + amp * np.cos(2 * np.pi * 3 * x / ng)[:, None, None] * np.ones((1, ng, ng))
    p, k, cnt = pk.power_spectrum(rho, box, n_bins=12)
    w = (math.sin(math.pi * 3 / ng) / (math.pi * 3 / ng)) ** 2
    closed = 2 * (amp ** 2 * box ** 3 / 4.0 / w ** 2) / int(cnt[3])
    return {"p_bin3": float(p[3]), "modes_bin3": int(cnt[3]), "closed_form_p_bin3": closed}


def main():
    data = {"force_newtonian_two_body": force_cases(), "lattice_most_bound": lattice_case(),
            "plane_wave_power": plane_wave_case()}
    with open(os.path.join(HERE, "oracle_values.json"), "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
