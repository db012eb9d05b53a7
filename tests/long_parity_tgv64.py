"""Long-run check of the FP64 GPU path against the CPU oracle: the
compressible Taylor-Green vortex of Sec. IV.C (Ma 1.2, tau = 0.52) on a full
64^3 grid for 1000 steps, the run length of the precision study, all fields
compared at every site.  It backs the use of the GPU FP64 run as the
reference of the 256^3 precision table.  About 4 minutes of oracle time on
16 threads, so it is a script, not part of the test suite:

    python tests/long_parity_tgv64.py [steps]

Prints per-field errors (the metric of the parity tests) every 100 steps,
with the velocity difference also against the initial velocity scale V0 and
the decay of max |u|, then one summary JSON line with the flags.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

from parity import field_errors  # noqa: E402

import oracle  # noqa: E402
from paper_2409_05114_amd import workloads as wl  # noqa: E402


def main():
    total = int(sys.argv[1]) if len(sys.argv) > 1 else 1000
    from paper_2409_05114_amd import lbm81
    shape, tau = (64, 64, 64), 0.52
    fl = wl.taylor_green(shape, ma=1.2)
    oracle.set_threads(min(16, os.cpu_count() or 1))
    f = oracle.init(shape, fl.rho, fl.u, fl.theta)
    sim = lbm81.Sim(shape, "f64")
    sim.init(fl.rho, fl.u, fl.theta)
    out, done, t0 = {}, 0, time.time()
    # compared (and printed) every 100 steps
    for target in sorted({10, *range(100, total + 1, 100), total}):
        if target > total or target <= done:
            continue
        oracle.step(shape, f, tau, target - done)
        sim.step(target - done, tau)
        done = target
        mo = oracle.moments(shape, f)
        rho, u, th = sim.moments()
        mg = (rho.cpu().numpy(), u.cpu().numpy(), th.cpu().numpy())
        out[target] = field_errors(mg, mo)
        # the vortex decays viscously, so the relative u error (against the
        # current max |u|) grows as the flow comes to rest; against the
        # initial velocity scale the difference stays at rounding level
        umax = float(np.sqrt((mo[1] ** 2).sum(0)).max())
        du = float(np.sqrt(((mg[1] - mo[1]) ** 2).sum(0)).max())
        out[target]["u_vs_v0"] = du / fl.meta["v0"]
        out[target]["max_u_over_v0"] = umax / fl.meta["v0"]
        print(json.dumps({"steps": target, "errors": out[target],
                          "elapsed_s": round(time.time() - t0, 1)}), flush=True)
    res = {"workload": "Taylor-Green 64^3, Ma 1.2, tau 0.52, FP64",
           "errors_by_steps": out, "flags": sim.flags(),
           "oracle_threads": oracle.get_threads()}
    sim.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
