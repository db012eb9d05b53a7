"""Benchmark of the RD3Q81 stream-collide hot path on one MI355X.

Workload (default): compressible Taylor-Green vortex on a 256^3 periodic box
(2 x 256^3 = 33.5M sites: cube corners and centres), Ma 1.2, tau = 0.52,
initialised to the entropic equilibrium; one "step" is one fused
stream-collide sweep of the whole grid (one kernel launch).  The FP64 path
is the headline `value`; the FP32 / FP16 / BF16 deviation-storage paths run
the same workload and are reported beside it with their error against the
FP64 run after the configured 1000 steps, on the 64^3 downsample (cube
corners with x, y, z = 0 mod 4); the FP64 GPU run stands in for the FP64
oracle there (the parity tests hold the two to 1e-12).

Timing: W untimed warm-up steps, then K steps bracketed by
torch.cuda.synchronize() and HIP events recorded on the stream the library
launches on; MLUPS = site updates per second / 1e6.  Roofline: algorithmic
HBM bytes per site update = 2 x 81 x sizeof(storage) (each population read
once and written once), divided by the average launch duration from the same
events.  cpu_baseline: the FP64 CPU oracle on a bounded sample of the same
workload (the same vortex on a 64^3 box, about 15 s of work), timed on this
host.

Serving: the first --serve-requests requests of a seeded Poisson request
stream (mean 20 arrivals/s; boxes of side 48..256, Ma 0.3..2, tau 0.51..0.9,
200..2000 steps, shear waves and vortices) are served in real time by the
continuous-batching server, once with FP32 and once with BF16 storage;
latency = completion - arrival, reported as p50 / p99 with the aggregate
throughput.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X nominal HBM3E bandwidth
METRIC = "MLUPS + % HBM peak, FP64 vs low-precision storage; p50/p99 solve latency"
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
# the sources of the step kernels and their launchers (the C ABI file holds
# no step kernel)
KERNEL_SOURCES = ["paper_2409_05114_amd/csrc/kernels.hpp",
                  "paper_2409_05114_amd/csrc/equilibrium.hpp",
                  "paper_2409_05114_amd/csrc/lattice.hpp",
                  "paper_2409_05114_amd/csrc/types.hpp",
                  "paper_2409_05114_amd/csrc/kernels_f64.hip",
                  "paper_2409_05114_amd/csrc/kernels_f32.hip",
                  "paper_2409_05114_amd/csrc/kernels_f16.hip",
                  "paper_2409_05114_amd/csrc/kernels_bf16.hip"]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_hash") != kernel_hash():
        return None
    e = t.get("per_launch_bytes", {}).get(storage)
    return e


WORKLOADS = {
    # name: (description, default storages, default steps, tau)
    "tgv256": ("compressible Taylor-Green vortex, 256^3 periodic cells "
               "(33554432 sites, corners + centres), Ma 1.2, tau 0.52, RD3Q81, "
               "in-place AA streaming", "f64,f32,f16,bf16", 1000, 0.52),
    "shear512": ("Mach-2 double shear layer, 512x512x256 periodic cells "
                 "(134217728 sites), tanh profile of 8 cells, 1e-3 velocity "
                 "perturbations, tau 0.52, RD3Q81, in-place AA streaming",
                 "f32", 500, 0.52),
}


def workload_fields(name, ma=None):
    from paper_2409_05114_amd import workloads as wl
    if name == "tgv256":
        return wl.taylor_green((256, 256, 256), ma=1.2 if ma is None else ma)
    return wl.shear_layer((512, 512, 256), ma=2.0)


# Run length of the precision study: the configured length of the 256^3
# Taylor-Green run (Sec. IV.C setting), whatever --steps times.
PRECISION_STEPS = 1000


def run_storage(storage, fields, tau, steps, warmup, keep_downsample,
                collision="bgk", warm_start=False, placement=1):
    import torch
    from paper_2409_05114_amd import lbm81

    sim = lbm81.Sim(fields.shape, storage, placement=placement)
    probe_ms, chosen = sim.placement_ms, sim.placement_choice
    sim.set_collision(collision)
    if warm_start and collision == "entropic":
        sim.set_warm_start()
    sim.init(fields.rho, fields.u, fields.theta)
    tot0, flags0 = sim.totals(check=False)  # (reading clears the flag word)
    sim.step(warmup, tau)
    torch.cuda.synchronize()
    stream = sim.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps, tau)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    tot, flags = sim.totals(check=False)
    flags |= flags0
    drift = {"mass": abs(tot[0] - tot0[0]) / abs(tot0[0]),
             "energy": abs(tot[4] - tot0[4]) / abs(tot0[4])}
    ds = None
    if keep_downsample:
        # the precision study compares the fields after PRECISION_STEPS
        # steps from the initial state: continue the timed run to that
        # length, or start again if it was longer
        done = warmup + steps
        if done > PRECISION_STEPS:
            sim.init(fields.rho, fields.u, fields.theta)
            done = 0
        sim.step(PRECISION_STEPS - done, tau)
        flags |= sim.flags()
        rho, u, th = sim.moments()
        nx, ny, nz = fields.shape
        r = rho.view(2, nz, ny, nx)[0, ::4, ::4, ::4].reshape(-1)
        # (cube corners with x, y, z = 0 mod 4)
        uu = u.view(3, 2, nz, ny, nx)[:, 0, ::4, ::4, ::4].reshape(3, -1)
        t = th.view(2, nz, ny, nx)[0, ::4, ::4, ::4].reshape(-1)
        ds = (r.cpu().numpy(), uu.cpu().numpy(), t.cpu().numpy())
        del rho, u, th
    sim.close()
    del sim
    torch.cuda.empty_cache()
    n = fields.n_sites
    per_launch_ms = ms / steps
    bytes_per_launch = 2 * 81 * STORAGE_BYTES[storage] * n
    gbs = bytes_per_launch / (per_launch_ms * 1e-3) / 1e9
    return {
        "storage": storage,
        "ms_per_step": per_launch_ms,
        "mlups": n * steps / (ms * 1e-3) / 1e6,
        "cell_mlups": n / 2 * steps / (ms * 1e-3) / 1e6,
        "gbs": gbs,
        "hbm_frac": gbs / HBM_PEAK_GBS,
        "bytes_per_launch": bytes_per_launch,
        "wall_s": wall,
        "flags": flags,
        "conservation_drift": drift,
        "mass_drift": None,
        "totals": tot.tolist(),
        # candidate population buffers timed by lbm_probe_placement (mean ms
        # of one pass of the step's memory pattern, in allocation order) and
        # the one kept; null for a plain allocation
        "placement": None if probe_ms is None else {
            "probe_ms": [round(v, 4) for v in probe_ms],
            "chosen": chosen,
            "first_vs_chosen": probe_ms[0] / probe_ms[chosen]},
    }, ds


def field_errors(a, b):
    ra, ua, ta = a
    rb, ub, tb = b
    du = np.sqrt(((ua - ub) ** 2).sum(0)).max()
    return {"rho": float(np.abs(ra - rb).max() / np.abs(rb).max()),
            "u": float(du / np.sqrt((ub ** 2).sum(0)).max()),
            "theta": float(np.abs(ta - tb).max() / np.abs(tb).max())}


def copy_probe(gib, reps=5):
    """A plain device-to-device copy of `gib` GiB (torch's copy kernel):
    known bytes for calibrating the byte counters, and a copy bandwidth."""
    import torch

    n = int(gib * 2 ** 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n,
            "ms": ms, "gbs": 2 * 8 * n / (ms * 1e-3) / 1e9}


def stream_probe(storage, gib=8.0, reps=10):
    """A second denominator: torch's in-place multiply of a `gib` GiB buffer
    of the storage's element type, i.e. every element read once and written
    once to the same place, as the in-place step does, with no pattern of its
    own.  GB/s."""
    import torch
    dt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16,
          "bf16": torch.bfloat16}[storage]
    n = int(gib * (1 << 30)) // STORAGE_BYTES[storage]
    a = torch.ones(n, dtype=dt, device="cuda")
    a.mul_(1.0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        a.mul_(1.0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a
    torch.cuda.empty_cache()
    return 2 * n * STORAGE_BYTES[storage] / (ms * 1e-3) / 1e9


def serve_bench(storage, n_requests, seed=0, rate=20.0, duration=60.0,
                policy="srpt", placement=1):
    """Real-time serving of the first n_requests (all if 0) of the seeded
    stream with `rate` arrivals/s over `duration` s."""
    import torch
    from paper_2409_05114_amd import workloads as wl
    from paper_2409_05114_amd.serve import Server, summarize

    reqs = wl.request_stream(rate=rate, duration=duration, seed=seed,
                             storage=storage)
    if n_requests:
        reqs = reqs[:n_requests]
    srv = Server(storage, realtime=True, policy=policy, placement=placement)

    def progress(rec, done, total):
        # one line per completed request (long runs report as they go)
        if done == total or done % max(1, total // 20) == 0:
            print(f"# serving {storage}: {done}/{total} requests done, "
                  f"latest {rec.rid} after {rec.latency:.1f} s", file=sys.stderr,
                  flush=True)

    recs = srv.run(reqs, progress=progress)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out = summarize(recs, srv.makespan)
    work = sum(r.sites * r.steps_done for r in recs)
    out.update({
        "storage": storage,
        "rate_per_s": rate,
        "arrival_window_s": reqs[-1].arrival,
        "site_updates": work,
        "max_resident": srv.max_resident,
        "policy": policy,
        "peak_hbm_bytes": srv.peak_used,
        "placement": placement,
    })
    return out


def batch_compare(storage, sides=(48, 64, 96, 128, 192, 256), tau=0.6,
                  reps=10):
    """The serving kernel against the plain step: for each box side, as many
    vortices of that side as make about 8M sites (at least one), stepped
    once through lbm_step_batch (one launch per step for all of them) and
    once one simulation at a time (lbm_step), two steps (one per parity)
    per repetition.  For sides up to 96 it first checks that 3 batched
    steps give bitwise the moments of 3 plain steps.  GLUPS = site updates
    per second / 1e9, timed with HIP events on the simulations' stream."""
    import torch
    from paper_2409_05114_amd import lbm81
    from paper_2409_05114_amd import workloads as wl

    dev = torch.device("cuda")

    def make(side, nsim):
        sims = []
        for k in range(nsim):
            rho, u, th = wl.device_fields("tgv", side, 1.0,
                                          (0.1 * k, 0.2, 0.3), dev)
            s = lbm81.Sim((side,) * 3, storage)
            s.init(rho, u, th)
            sims.append(s)
        return sims

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 2  # ms per step

    rows = []
    for side in sides:
        nsim = max(1, (8 << 20) // (2 * side ** 3))
        sims = make(side, nsim)
        sites = nsim * 2 * side ** 3
        equal = None
        if side <= 96:
            twins = make(side, nsim)
            lbm81.lbm_step_batch(twins, 3, [tau] * nsim)
            for s in sims:
                s.step(3, tau)
            equal = all(torch.equal(a, b) for s, t in zip(sims, twins)
                        for a, b in zip(s.moments(), t.moments()))
            for t in twins:
                t.close()

        def plain():
            for s in sims:
                s.step(2, tau)

        def batched():
            lbm81.lbm_step_batch(sims, 2, [tau] * nsim)

        tp, tb = timed(plain), timed(batched)
        rows.append({"storage": storage, "side": side, "sims": nsim,
                     "sites": sites, "plain_glups": sites / tp / 1e6,
                     "batch_glups": sites / tb / 1e6,
                     "batched_equals_plain": equal})
        print(f"# batch {storage} {side}^3 x {nsim}: plain "
              f"{rows[-1]['plain_glups']:.2f}, batched "
              f"{rows[-1]['batch_glups']:.2f} GLUPS, bitwise equal: {equal}",
              file=sys.stderr, flush=True)
        for s in sims:
            s.close()
        del sims
        torch.cuda.empty_cache()
    return rows


def cpu_baseline(seconds_target=15.0):
    import oracle
    from paper_2409_05114_amd import workloads as wl

    # every CPU this process may run on (its affinity mask; where nproc and a
    # cgroup quota also apply they are reported beside it)
    host_cpus = len(os.sched_getaffinity(0))
    oracle.set_threads(host_cpus)
    side = 64
    shape = (side, side, side)
    fl = wl.taylor_green(shape, ma=1.2)
    f = oracle.init(shape, fl.rho, fl.u, fl.theta)
    t0 = time.perf_counter()
    oracle.step(shape, f, 0.52, 1)
    one = time.perf_counter() - t0
    steps = max(1, min(500, int(seconds_target / max(one, 1e-3))))
    t0 = time.perf_counter()
    oracle.step(shape, f, 0.52, steps)
    dt = time.perf_counter() - t0
    n = 2 * side ** 3
    return {"value": n * steps / dt / 1e6, "unit": "MLUPS",
            "cores": oracle.get_threads(), "host_cpus": host_cpus,
            "nproc": os.cpu_count(), "kind": "oracle",
            "sample": f"Taylor-Green Ma 1.2, tau 0.52 on {side}^3 cells "
                      f"({n} sites), {steps} FP64 steps after 1 warm-up "
                      f"step, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="tgv256", choices=sorted(WORKLOADS),
                    help="tgv256: the headline benchmark; shear512: the "
                         "512x512x256 shear-layer roofline study")
    ap.add_argument("--ma", type=float, default=None,
                    help="Mach number of the tgv256 vortex (default 1.2, the "
                         "headline); the series step applies at low Mach")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--storages", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--collision", default="bgk",
                    choices=["bgk", "entropic", "series"],
                    help="bgk: the headline (alpha = 2); entropic: alpha from "
                         "the entropy condition at every site (ALU-bound); "
                         "series: BGK towards the series equilibrium where "
                         "it is positive")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="entropic collision: start every search cold "
                         "(default: from the alpha each site had in the "
                         "previous step, lbm_set_warm_start)")
    ap.add_argument("--placement", type=int, default=32,
                    help="candidate population buffers per storage: the "
                         "fastest under lbm_probe_placement is kept (1: the "
                         "first allocation, unprobed)")
    ap.add_argument("--serve-placement", type=int, default=1,
                    help="served requests of side >= 128 get the fastest of "
                         "this many candidate buffers (1: no probing)")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests of the serving stream to serve per storage "
                         "(0: skip the serving measurement)")
    ap.add_argument("--serve-storages", default="f32,bf16")
    ap.add_argument("--serve-rate", type=float, default=20.0,
                    help="mean arrivals per second of the serving stream")
    ap.add_argument("--serve-duration", type=float, default=60.0,
                    help="seconds of arrivals of the serving stream")
    ap.add_argument("--serve-policy", default="srpt", choices=["srpt", "share"],
                    help="srpt: each tick advances the simulations with the "
                         "least remaining work (enough to fill the GPU); "
                         "share: all resident simulations every tick")
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the serving measurement")
    ap.add_argument("--batch-compare", default=None, metavar="STORAGES",
                    help="only compare the batched (serving) step with the "
                         "plain one per box side for these storages")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only time a plain device copy of this many GiB "
                         "(calibration of the rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.ma is not None and args.workload != "tgv256":
        ap.error("--ma applies to the tgv256 workload")
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                          "the multi-GPU path is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2409_05114_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.copy_gib > 0:
        print(json.dumps(copy_probe(args.copy_gib)), flush=True)
        return
    if args.batch_compare:
        rows = []
        for st in [s for s in args.batch_compare.split(",") if s]:
            rows += batch_compare(st)
        print(json.dumps({"batch_compare": rows}), flush=True)
        return
    if args.serve_only:
        out = {}
        for st in [s for s in args.serve_storages.split(",") if s]:
            out[st] = serve_bench(st, args.serve_requests, rate=args.serve_rate,
                                  duration=args.serve_duration,
                                  policy=args.serve_policy,
                                  placement=args.serve_placement)
            print(f"# serving {st}: {json.dumps(out[st])}", file=sys.stderr,
                  flush=True)
        print(json.dumps({"serving": out}), flush=True)
        return
    desc, def_storages, def_steps, tau = WORKLOADS[args.workload]
    args.steps = args.steps if args.steps is not None else def_steps
    fields = workload_fields(args.workload, args.ma)
    if args.ma is not None:
        desc = desc.replace("Ma 1.2", f"Ma {args.ma:g}")
    shape = fields.shape
    n_sites = 2 * shape[0] * shape[1] * shape[2]
    storages = [s for s in (args.storages or def_storages).split(",") if s]
    results, ds = {}, {}
    for st in storages:
        r, d = run_storage(st, fields, tau, args.steps, args.warmup,
                           keep_downsample=args.workload == "tgv256",
                           collision=args.collision,
                           warm_start=not args.no_warm_start,
                           placement=args.placement)
        results[st] = r
        ds[st] = d
        print(f"# {st}: {r['mlups']:.1f} MLUPS, {r['gbs']:.1f} GB/s "
              f"({100 * r['hbm_frac']:.1f}% of 8 TB/s), "
              f"{r['ms_per_step']:.3f} ms/step, flags={r['flags']}",
              file=sys.stderr, flush=True)
    if "f64" in ds and ds["f64"] is not None:
        for st in storages:
            if st != "f64" and ds[st] is not None:
                err = field_errors(ds[st], ds["f64"])
                err.update({
                    "steps": PRECISION_STEPS,
                    "sites": "cube corners with x, y, z = 0 mod 4 (64^3)",
                    "reference": "the FP64 GPU run of the same workload, "
                                 "which stands in for the FP64 oracle: it "
                                 "equals the oracle within 1e-12 per step "
                                 "and over 1000 steps of the 64^3 vortex "
                                 "(GPU parity tests)"})
                results[st]["error_vs_f64_64cubed"] = err
                results[st]["speedup_vs_f64"] = (results[st]["mlups"] /
                                                 results["f64"]["mlups"])
    head = results.get("f64") or results[storages[0]]
    main_st = head["storage"]
    bgk = args.collision in ("bgk", "series")  # bound by HBM
    traffic = (measured_traffic(main_st)
               if args.workload == "tgv256" and args.collision == "bgk"
               and args.ma is None else None)
    stream_gbs = stream_probe(main_st)
    line = {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_st,
        "data": "synthetic",
        "config": {
            "workload": desc,
            "grid": list(shape), "sites": n_sites, "tau": tau,
            "storage": main_st, "mlups_counts": "site updates",
            "collision": args.collision,
            "warm_start": args.collision == "entropic" and not args.no_warm_start,
            "placement": (f"the fastest of up to {args.placement} population "
                          "buffers under lbm_probe_placement"
                          if args.placement > 1 else "first allocation"),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": head["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": head["hbm_frac"],
            "traffic": traffic,
            "stream_gbs": stream_gbs,
            "frac_of_stream": head["gbs"] / stream_gbs,
        } if bgk else {
            # the entropic step is bound by the vector ALU; its HBM rate
            # is given for comparison with the BGK step
            "bound": "alu",
            "hbm_achieved": head["gbs"],
            "hbm_peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "hbm_frac": head["hbm_frac"],
        },
        "storages": results,
    }
    if args.serve_requests > 0:
        serving = {"sample": f"a burst: the first {args.serve_requests} "
                             "requests of the seeded Poisson stream "
                             f"({args.serve_rate:g} arrivals/s, seed 0), "
                             "served in real time; `arrival_window_s` is "
                             "when the last of them arrives.  The whole "
                             f"{args.serve_duration:g}-s stream offers far "
                             "more work than one GPU serves in that time "
                             "(--serve-requests 0 serves all of it)"}
        for st in [s for s in args.serve_storages.split(",") if s]:
            r = serve_bench(st, args.serve_requests, rate=args.serve_rate,
                            duration=args.serve_duration,
                            policy=args.serve_policy,
                            placement=args.serve_placement)
            serving[st] = r
            print(f"# serving {st}: p50 {r['p50_latency_s']:.2f} s, "
                  f"p99 {r['p99_latency_s']:.2f} s, "
                  f"{r['aggregate_mlups']:.0f} MLUPS aggregate, "
                  f"{r['requests']} requests, flags={r['flags']}",
                  file=sys.stderr, flush=True)
        line["serving"] = serving
        first = serving.get("f32") or next(
            v for k, v in serving.items() if k != "sample")
        line["p50_latency_s"] = first["p50_latency_s"]
        line["p99_latency_s"] = first["p99_latency_s"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
