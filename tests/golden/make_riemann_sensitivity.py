"""Write tests/golden/riemann2000_sensitivity.json: how far the CPU oracle's
own FP64 result of the periodic double Riemann problem (Sec. IV.A states:
rho = 1, theta = theta0 | rho = 0.125, theta = 0.8 theta0; tau = 0.55) moves
after 2000 steps when its initial density is perturbed by 1e-16 relative,
for several seeded perturbations.  Interacting shocks amplify rounding, so
this is the scale of agreement that two correct FP64 implementations with
different rounding orders can reach there.  Only the oracle and the seeded
input recipe are called.

    python tests/golden/make_riemann_sensitivity.py   # ~2 min on 8 cores
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2409_05114_amd import workloads as wl  # noqa: E402

SHAPE = (2048, 1, 1)
TAU, STEPS, REL = 0.55, 2000, 1e-16
SEEDS = tuple(range(8))
OUT = os.path.join(HERE, "riemann2000_sensitivity.json")


def field_errors(a, b):
    """The parity tests' metric: max |a - b| / max |b| for rho and theta,
    the largest Euclidean velocity difference over max |u_b|."""
    ra, ua, ta = a
    rb, ub, tb = b
    du = np.sqrt(((ua - ub) ** 2).sum(0)).max()
    return {"rho": float(np.abs(ra - rb).max() / np.abs(rb).max()),
            "u": float(du / np.sqrt((ub ** 2).sum(0)).max()),
            "theta": float(np.abs(ta - tb).max() / np.abs(tb).max())}


def main():
    oracle.set_threads(os.cpu_count() or 1)
    fl = wl.double_riemann(SHAPE)
    (m0, _) = oracle.run(SHAPE, fl.rho, fl.u, fl.theta, TAU, STEPS)
    per_seed = []
    for seed in SEEDS:
        rng = np.random.default_rng(seed)
        rho = fl.rho * (1 + REL * rng.uniform(-1, 1, fl.rho.size))
        (m, _) = oracle.run(SHAPE, rho, fl.u, fl.theta, TAU, STEPS)
        per_seed.append(field_errors(m, m0))
        print(seed, per_seed[-1], flush=True)
    med = {k: float(np.median([e[k] for e in per_seed])) for k in per_seed[0]}
    rec = {"shape": SHAPE, "tau": TAU, "steps": STEPS, "perturbation": REL,
           "seeds": SEEDS, "per_seed": per_seed, "median": med}
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(OUT, med)


if __name__ == "__main__":
    main()
