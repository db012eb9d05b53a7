"""The serving scheduler's selection (paper_2409_05114_amd.serve.schedule),
on the CPU: each tick advances the resident simulations with the least
remaining work until the launch is full, never starves one beyond the skip
bound, and with processor sharing advances all."""
from paper_2409_05114_amd.serve import schedule


def test_least_remaining_work_first_until_full():
    # (remaining work, sites, ticks skipped, id)
    jobs = [(900, 10, 0, 0), (100, 10, 0, 1), (500, 10, 0, 2), (100, 10, 0, 3)]
    assert schedule(jobs, "srpt", sat_sites=20) == [1, 3]
    assert schedule(jobs, "srpt", sat_sites=25) == [1, 3, 2]
    assert sorted(schedule(jobs, "srpt", sat_sites=10 ** 9)) == [0, 1, 2, 3]


def test_share_advances_everything():
    jobs = [(900, 10, 0, 0), (100, 10, 0, 1)]
    assert schedule(jobs, "share", sat_sites=1) == [0, 1]


def test_a_starved_job_joins_the_next_launch():
    jobs = [(900, 10, 64, 0), (100, 10, 0, 1), (200, 10, 0, 2)]
    got = schedule(jobs, "srpt", sat_sites=20, max_skip=64)
    assert got[0] == 0 and got == [0, 1]


def test_every_job_progresses_within_the_bound():
    """Simulated ticks: a long job among a steady supply of short ones is
    advanced at least once every max_skip + 1 ticks."""
    max_skip = 8
    long_job = [10 ** 6, 100, 0, 0]
    shorts = []
    advanced_at = []
    nid = 1
    for tick in range(200):
        while len(shorts) < 3:  # short jobs keep arriving
            shorts.append([50, 100, 0, nid])
            nid += 1
        jobs = [tuple(long_job)] + [tuple(j) for j in shorts]
        pick = schedule(jobs, "srpt", sat_sites=100, max_skip=max_skip)
        allj = [long_job] + shorts
        for k, j in enumerate(allj):
            j[2] = 0 if k in pick else j[2] + 1
            if k in pick:
                j[0] -= 25
        if 0 in pick:
            advanced_at.append(tick)
        shorts = [j for j in shorts if j[0] > 0]
    gaps = [b - a for a, b in zip([-1] + advanced_at, advanced_at)]
    assert advanced_at and max(gaps) <= max_skip + 1


def test_every_request_of_the_stream_starts_realizable():
    """Every request of the seeded serving stream (20 arrivals/s for 60 s)
    starts from a realizable state: density at least a quarter of rho0 and
    positive temperature, so no simulation is flagged at initialisation.
    The fields are evaluated at the request's Mach number and phases on a
    coarser box; the vortex's minimum density on any grid is at least its
    minimum over the continuous box, p0 - (3/8) rho0 V0^2 over theta0, which
    the densest sampling here (x^ = y^ = z^ = pi/2 on a 16^3 box with zero
    phase) reaches exactly."""
    import dataclasses

    import numpy as np

    from paper_2409_05114_amd import workloads as wl

    reqs = wl.request_stream(rate=20.0, duration=60.0, seed=0)
    assert len(reqs) > 1000
    assert max(r.ma for r in reqs) > 1.9
    for r in reqs:
        fl = dataclasses.replace(r, side=16).fields()
        assert fl.rho.min() >= wl.SERVE_TGV_RHO_MIN * (1 - 1e-12), r
        assert fl.theta.min() > 0 and np.isfinite(fl.u).all()
    # the bound is reached: a Mach-2 vortex with zero phase
    fl = wl.taylor_green((16, 16, 16), ma=2.0, p0=wl.serve_tgv_p0(2.0))
    assert abs(fl.rho.min() - wl.SERVE_TGV_RHO_MIN) < 1e-12
    # p0 = rho0 theta0 (the benchmark vortex) wherever that keeps the bound
    assert wl.serve_tgv_p0(1.0) == wl.THETA0


def test_served_fields_on_device_equal_the_host_recipe():
    """Request.fields_on_device (built with torch, here on the CPU) equals
    Request.fields for a vortex above Ma 1.26 and for a shear wave."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2409_05114_amd import workloads as wl

    reqs = wl.request_stream(rate=20.0, duration=60.0, seed=0)
    tgv = next(r for r in reqs if r.kind == "tgv" and r.ma > 1.5)
    shear = next(r for r in reqs if r.kind == "shear")
    for r in (tgv, shear):
        r = dataclasses.replace(r, side=12)
        fl = r.fields()
        rho, u, th = r.fields_on_device(torch.device("cpu"))
        np.testing.assert_allclose(rho.numpy(), fl.rho, rtol=1e-13, atol=0)
        np.testing.assert_allclose(u.numpy(), fl.u, rtol=0, atol=1e-13)
        np.testing.assert_allclose(th.numpy(), fl.theta, rtol=0, atol=0)
