"""Write tests/golden/tgv64_ma12_tau052.npz: the CPU oracle's FP64 fields of
the compressible Taylor-Green vortex (Sec. IV.C) on a full 64^3 grid at
Ma 1.2, tau = 0.52 -- the initial condition, relaxation time and run length
(1000 steps) of the 256^3 precision study, on a grid the oracle finishes in
minutes.  Only the oracle and the seeded input recipe are called.

Stored per checkpoint (steps 100, 200, 500 and 1000):
  * rho, u[3], theta at the sampled sites `sites_<n>`:
    - step 1000: every main site with x, y, z = 0 mod 4 (a 16^3 downsample)
      and every centre site with x, y, z = 0 mod 8;
    - steps 100, 200, 500: main and centre sites with x, y, z = 0 mod 8;
  * the full-grid maxima max|rho|, max|u| (Euclidean), max|theta| (the
    denominators of the relative error) and the domain totals (Eq. conslaws);
plus a SHA-256 of the input fields, so that a test can tell when the input
recipe has changed and the file must be written again.

    python tests/golden/make_tgv64_golden.py   # ~10 min on 8 cores
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2409_05114_amd import workloads as wl  # noqa: E402

SHAPE = (64, 64, 64)
MA, TAU = 1.2, 0.52
CHECKPOINTS = (100, 200, 500, 1000)
OUT = os.path.join(HERE, "tgv64_ma12_tau052.npz")


def input_fields():
    return wl.taylor_green(SHAPE, ma=MA)


def input_digest(fl):
    h = hashlib.sha256()
    for a in (fl.rho, fl.u, fl.theta):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def sample_sites(step):
    """Site indices (order ((sub nz + z) ny + y) nx + x) sampled at `step`."""
    nx, ny, nz = SHAPE
    out = []
    for sub in (0, 1):
        m = 4 if (step == CHECKPOINTS[-1] and sub == 0) else 8
        z, y, x = np.meshgrid(np.arange(0, nz, m), np.arange(0, ny, m),
                              np.arange(0, nx, m), indexing="ij")
        out.append((((sub * nz + z) * ny + y) * nx + x).reshape(-1))
    return np.concatenate(out).astype(np.int64)


def main():
    fl = input_fields()
    oracle.set_threads(os.cpu_count() or 1)
    f = oracle.init(SHAPE, fl.rho, fl.u, fl.theta)
    rec = {"shape": np.array(SHAPE), "ma": np.array(MA), "tau": np.array(TAU),
           "v0": np.array(fl.meta["v0"]),
           "checkpoints": np.array(CHECKPOINTS),
           "input_sha256": np.array(input_digest(fl))}
    done, t0 = 0, time.time()
    for n in CHECKPOINTS:
        oracle.step(SHAPE, f, TAU, n - done)
        done = n
        rho, u, th = oracle.moments(SHAPE, f)
        idx = sample_sites(n)
        rec[f"sites_{n}"] = idx
        rec[f"rho_{n}"] = rho[idx]
        rec[f"u_{n}"] = np.ascontiguousarray(u[:, idx])
        rec[f"theta_{n}"] = th[idx]
        rec[f"max_{n}"] = np.array([np.abs(rho).max(),
                                    np.sqrt((u ** 2).sum(0)).max(),
                                    np.abs(th).max()])
        rec[f"totals_{n}"] = oracle.totals(SHAPE, f)
        print(f"step {n}: max|u|/V0 = {rec[f'max_{n}'][1] / fl.meta['v0']:.3e}"
              f" ({time.time() - t0:.0f} s)", flush=True)
    rec["oracle_threads"] = np.array(oracle.get_threads())
    np.savez_compressed(OUT, **rec)
    print(OUT)


if __name__ == "__main__":
    main()
