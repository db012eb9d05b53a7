"""Compressible Taylor-Green vortex time series (Sec. IV.C): the mean kinetic
energy KE = <rho u.u / 2> and the mean enstrophy eps = <rho w.w / 2> of the
vortex over time, on an n^3 periodic box at a given Mach and Reynolds number,
advanced by the library's step kernels and measured by its diagnostics call.

Units follow Sec. IV.C: x^ = x / L with L = n / (2 pi) cells, V0 = Ma c_s,
Re = V0 L / nu, and nu = tau theta at theta = theta0 (Sec. II), so
tau = V0 L / (Re theta0).  Time is reported in convective units
t* = t V0 / L (t in steps).

Besides the two series the run reports the kinetic-energy budget: for a flow
whose density stays close to uniform (low Mach number) the energy decays as
dKE/dt = -2 nu eps, so the ratio (-dKE/dt) / (2 nu eps), with dKE/dt from
central differences of the series, is 1 up to compressibility, the time
differencing and the lattice's own dissipation error.  It needs no reference
data: it checks the viscosity the update delivers inside a turbulent flow.

    python -m paper_2409_05114_amd.tgv --n 512 --ma 0.1 --re 1600 --tmax 20

prints one JSON line per sample and a summary line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

from . import workloads as wl


def parameters(n, ma, re):
    """(L, V0, nu, tau, steps per convective time) of the vortex."""
    L = n / (2.0 * math.pi)
    v0 = ma * wl.C_S
    nu = v0 * L / re
    tau = nu / wl.THETA0
    return {"L": L, "V0": v0, "nu": nu, "tau": tau, "omega": 2.0 / (2.0 * tau + 1.0),
            "t_conv": L / v0}


def energy_budget(t, ke, eps, nu):
    """(-dKE/dt) / (2 nu eps) at the interior samples, dKE/dt by central
    differences in t (steps)."""
    out = []
    for k in range(1, len(t) - 1):
        d = -(ke[k + 1] - ke[k - 1]) / (t[k + 1] - t[k - 1])
        out.append(d / (2.0 * nu * eps[k]) if eps[k] > 0 else float("nan"))
    return out


def run(n=512, ma=0.1, re=1600.0, tmax=20.0, dt=0.25, storage="f32",
        collision="bgk", emit=print, warm_start=False):
    import torch
    from . import lbm81

    p = parameters(n, ma, re)
    every = max(1, int(round(dt * p["t_conv"])))
    nsteps = int(round(tmax * p["t_conv"]))
    emit(json.dumps({"event": "start", "n": n, "ma": ma, "re": re, "storage": storage,
                     "collision": collision, "warm_start": warm_start,
                     "steps": nsteps, "sample_every": every,
                     **p}))
    t0 = time.perf_counter()
    fl = wl.taylor_green((n, n, n), ma=ma)
    sim = lbm81.Sim((n, n, n), storage)
    sim.init(fl.rho, fl.u, fl.theta)
    del fl
    if collision != "bgk":
        sim.set_collision(collision)
    if warm_start and collision == "entropic":
        sim.set_warm_start()
    fields = torch.empty(4 * sim.n_sites, dtype=torch.float64, device=sim.device)
    emit(json.dumps({"event": "initialised", "seconds": round(time.perf_counter() - t0, 1)}))
    ts, kes, epss = [], [], []
    step_seconds = 0.0
    done = 0
    flagged = 0
    while True:
        ke, eps = sim.diagnostics(fields)
        fl_word = sim.flags()
        ts.append(done)
        kes.append(ke)
        epss.append(eps)
        emit(json.dumps({"step": done, "t": done / p["t_conv"], "ke": ke, "eps": eps,
                         "flags": fl_word}))
        if fl_word or not (math.isfinite(ke) and math.isfinite(eps)):
            flagged = fl_word or -1
            break
        if done >= nsteps:
            break
        k = min(every, nsteps - done)
        torch.cuda.synchronize()
        a = time.perf_counter()
        sim.step(k, p["tau"])
        torch.cuda.synchronize()
        step_seconds += time.perf_counter() - a
        done += k
    ratio = energy_budget(ts, kes, epss, p["nu"])
    kmax = max(range(len(epss)), key=lambda i: epss[i])
    summary = {"event": "summary", "steps_done": done, "flags": flagged,
               "mlups": 2 * n ** 3 * done / step_seconds / 1e6 if step_seconds else None,
               "ke0": kes[0], "ke_end": kes[-1], "eps_peak": epss[kmax],
               "t_eps_peak": ts[kmax] / p["t_conv"],
               "budget_ratio": ratio}
    emit(json.dumps(summary))
    sim.close()
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--ma", type=float, default=0.1)
    ap.add_argument("--re", type=float, default=1600.0)
    ap.add_argument("--tmax", type=float, default=20.0, help="convective times")
    ap.add_argument("--dt", type=float, default=0.25, help="sampling interval, convective times")
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16", "bf16"])
    ap.add_argument("--collision", default="bgk", choices=["bgk", "entropic"])
    ap.add_argument("--warm-start", action="store_true",
                    help="entropic collision: start each site's search from "
                         "its alpha of the previous step")
    ap.add_argument("--out", default=None, help="also append the JSON lines to this file")
    a = ap.parse_args(argv)
    fh = open(a.out, "a") if a.out else None

    def emit(line):
        print(line, flush=True)
        if fh:
            fh.write(line + "\n")
            fh.flush()

    s = run(a.n, a.ma, a.re, a.tmax, a.dt, a.storage, a.collision, emit,
            warm_start=a.warm_start)
    if fh:
        fh.close()
    return 0 if not s["flags"] else 1


if __name__ == "__main__":
    sys.exit(main())
