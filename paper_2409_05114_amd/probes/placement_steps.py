"""Placement against step time: for each storage form, allocate simulations
of the 256^3 Taylor-Green vortex (Ma 1.2) one after another until device
memory runs short, and print for each buffer the placement probe's time
(lbm_probe_placement, one pass of the step's memory pattern) beside the
times of one even step, one odd step and the mean of ten steps (tau 0.52).

    python -m paper_2409_05114_amd.probes.placement_steps --storages f64,f16

A measurement program beside the library: it shows whether the probe ranks
buffers as the step kernels do.  One JSON line per buffer on stdout.
"""
import argparse
import ctypes
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--storages", default="f64,f16,bf16")
    ap.add_argument("--max", type=int, default=48,
                    help="at most this many buffers per storage form")
    ap.add_argument("--reserve-gib", type=float, default=8.0,
                    help="device memory left free beside the buffers")
    args = ap.parse_args()

    import torch
    from paper_2409_05114_amd import lbm81
    from paper_2409_05114_amd import workloads as wl

    torch.cuda.set_device(0)
    shape = (256, 256, 256)
    fields = wl.taylor_green(shape, ma=1.2)
    lib = lbm81.library()
    tau = 0.52
    for st in [s for s in args.storages.split(",") if s]:
        pb = lbm81.lbm_population_bytes(*shape, st)
        sims = []
        while len(sims) < args.max:
            if torch.cuda.mem_get_info()[0] < pb + args.reserve_gib * 2 ** 30:
                break
            s = lbm81.Sim(shape, st)
            s.init(fields.rho, fields.u, fields.theta)
            sims.append(s)
        torch.cuda.synchronize()
        for k, s in enumerate(sims):
            ms = ctypes.c_float()
            if lib.lbm_probe_placement(s.handle, 3, ctypes.byref(ms)) != 0:
                raise RuntimeError(lbm81.library().lbm_last_error())
            s.step(2, tau)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record(s.stream)
            s.step(1, tau)
            ev[1].record(s.stream)
            s.step(1, tau)
            ev[2].record(s.stream)
            s.step(8, tau)
            ev[3].record(s.stream)
            torch.cuda.synchronize()
            print(json.dumps({
                "storage": st, "buffer": k,
                "address_gib": round(s.populations.data_ptr() / 2 ** 30, 2),
                "probe_ms": round(ms.value, 4),
                "even_ms": round(ev[0].elapsed_time(ev[1]), 4),
                "odd_ms": round(ev[1].elapsed_time(ev[2]), 4),
                "mean10_ms": round(ev[0].elapsed_time(ev[3]) / 10, 4)}),
                flush=True)
        for s in sims:
            s.close()
        del sims
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
