"""FP64 parity over the precision study's whole run length: the compressible
Taylor-Green vortex (Sec. IV.C) at Ma 1.2, tau = 0.52, on a full 64^3 grid
for 1000 steps, compared with the CPU oracle's fields stored in
tests/golden/tgv64_ma12_tau052.npz (written by make_tgv64_golden.py beside
it, which calls only the oracle and the seeded input recipe).

Metric per checkpoint (100, 200, 500, 1000 steps), on the stored sites:
max |a - b| over the full-grid max |b| for rho and theta, and the largest
Euclidean velocity difference over the full-grid max |u| (the parity tests'
metric), required to be at most 1e-12.  At this grid size the vortex decays
viscously by orders of magnitude within 1000 steps, so late in the run the
current max |u| is far below the flow's scale V0 and a velocity difference
at the FP64 rounding level of V0 is a large fraction of it.  There the
velocity is compared against V0 (the normalisation of the flow) instead:
the metric against the current max |u| applies while that is at least
V0 / 100, and against V0 at every checkpoint.
"""
import hashlib
import os

import numpy as np
import pytest

from paper_2409_05114_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "tgv64_ma12_tau052.npz")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _golden():
    return np.load(GOLDEN, allow_pickle=False)


def test_tgv64_1000_steps_fp64_equals_oracle():
    from paper_2409_05114_amd import lbm81

    g = _golden()
    shape = tuple(int(v) for v in g["shape"])
    ma, tau, v0 = float(g["ma"]), float(g["tau"]), float(g["v0"])
    fl = wl.taylor_green(shape, ma=ma)
    h = hashlib.sha256()
    for a in (fl.rho, fl.u, fl.theta):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    assert h.hexdigest() == str(g["input_sha256"]), "input recipe changed"
    print(f"long parity: {shape} vortex Ma {ma}, tau {tau}, FP64", flush=True)
    sim = lbm81.Sim(shape, "f64")
    sim.init(fl.rho, fl.u, fl.theta)
    done = 0
    for n in (int(c) for c in g["checkpoints"]):
        sim.step(n - done, tau)
        done = n
        rho, u, th = (t.cpu().numpy() for t in sim.moments())
        idx = g[f"sites_{n}"]
        rmax, umax, tmax = g[f"max_{n}"]
        e_rho = np.abs(rho[idx] - g[f"rho_{n}"]).max() / rmax
        e_th = np.abs(th[idx] - g[f"theta_{n}"]).max() / tmax
        du = np.sqrt(((u[:, idx] - g[f"u_{n}"]) ** 2).sum(0)).max()
        tot, flags = sim.totals()
        print(f"step {n}: rho {e_rho:.2e}, theta {e_th:.2e}, u/V0 "
              f"{du / v0:.2e}, u/max|u| {du / umax:.2e} (max|u| = "
              f"{umax / v0:.2e} V0)", flush=True)
        assert flags == 0
        assert e_rho <= 1e-12 and e_th <= 1e-12
        assert du / v0 <= 1e-12
        if umax >= 1e-2 * v0:
            assert du / umax <= 1e-12
        # the totals of Eq. (conslaws) against the oracle's
        ref = g[f"totals_{n}"]
        assert abs(tot[0] - ref[0]) <= 1e-13 * ref[0]
        assert abs(tot[4] - ref[4]) <= 1e-13 * ref[4]
        assert np.abs(tot[1:4] - ref[1:4]).max() <= 1e-13 * ref[0] * wl.C_S
    sim.close()


# FP16: the 1e-3 target of the precision form.  FP32: 1e-4, ten times the
# FP32 error of the 256^3 vortex after 1000 steps (1.7e-5), so a regression
# shows.  BF16: 2e-2, which documents its miss of the target (8.8e-3 on the
# 256^3 vortex after 1000 steps).
BARS = {"f32": 1e-4, "f16": 1e-3, "bf16": 2e-2}


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_tgv64_1000_steps_low_precision_against_oracle(storage):
    """The precision form over the same 1000 steps, against the same stored
    oracle fields: FP16 within the 1e-3 target, FP32 within 1e-4, BF16
    within 2e-2 (its 8-bit mantissa misses 1e-3; the measured values are
    printed).  rho and theta at every checkpoint; the velocity against the
    current max |u| while that is at least V0 / 100 (100 and 200 steps) and
    against V0 at every checkpoint."""
    from paper_2409_05114_amd import lbm81

    g = _golden()
    shape = tuple(int(v) for v in g["shape"])
    ma, tau, v0 = float(g["ma"]), float(g["tau"]), float(g["v0"])
    fl = wl.taylor_green(shape, ma=ma)
    print(f"long precision: {shape} vortex, {storage}", flush=True)
    sim = lbm81.Sim(shape, storage)
    sim.init(fl.rho, fl.u, fl.theta)
    done = 0
    for n in (int(c) for c in g["checkpoints"]):
        sim.step(n - done, tau)
        done = n
        rho, u, th = (t.cpu().numpy() for t in sim.moments())
        idx = g[f"sites_{n}"]
        rmax, umax, tmax = g[f"max_{n}"]
        e_rho = np.abs(rho[idx] - g[f"rho_{n}"]).max() / rmax
        e_th = np.abs(th[idx] - g[f"theta_{n}"]).max() / tmax
        du = np.sqrt(((u[:, idx] - g[f"u_{n}"]) ** 2).sum(0)).max()
        print(f"{storage} step {n}: rho {e_rho:.2e}, theta {e_th:.2e}, u/V0 "
              f"{du / v0:.2e}, u/max|u| {du / umax:.2e}", flush=True)
        bar = BARS[storage]
        assert e_rho <= bar and e_th <= bar and du / v0 <= bar
        if umax >= 1e-2 * v0:
            assert du / umax <= bar
    assert sim.flags() == 0
    sim.close()
