"""Serving form: continuous batching of independent simulations.

Every served result must equal the same request run alone with lbm_step
(bitwise: the batched launch does exactly the per-site work of the plain
step), admission must respect the memory budget while requests that arrive
later join simulations already on the device, and a request that can never
fit must be refused loudly.
"""
import numpy as np
import pytest

from paper_2409_05114_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _requests(storage):
    # mixed sides (row segments of 16..96 lanes), Mach numbers, taus, steps
    spec = [(16, 0.3, 0.6, 40, "shear"), (24, 1.2, 0.52, 25, "tgv"),
            (32, 2.0, 0.9, 33, "shear"), (48, 0.8, 0.55, 18, "tgv"),
            (16, 0.8, 0.51, 57, "tgv"), (64, 0.5, 0.7, 12, "shear"),
            (20, 1.0, 0.8, 29, "tgv")]
    out = []
    for k, (n, ma, tau, steps, kind) in enumerate(spec):
        out.append(wl.Request(rid=k, arrival=0.0, side=n, ma=ma, tau=tau,
                              steps=steps, kind=kind,
                              phase=(0.1 * k, 0.2 * k, 0.3 * k),
                              storage=storage))
    return out


def _alone(req, storage):
    import torch
    from paper_2409_05114_amd import lbm81
    sim = lbm81.Sim((req.side,) * 3, storage)
    rho, u, th = req.fields_on_device(sim.device)
    sim.init(rho, u, th)
    sim.step(req.steps, req.tau)
    out = tuple(t.cpu().numpy() for t in sim.moments())
    torch.cuda.synchronize()
    sim.close()
    return out


@pytest.mark.parametrize("storage", ["f32", "bf16", "f64"])
@pytest.mark.parametrize("placement", [1, 3], ids=["plain", "probed"])
def test_served_results_equal_alone(storage, placement):
    """probed: requests of side >= 32 are admitted into the fastest of three
    candidate buffers (lbm_probe_placement); the results do not change."""
    from paper_2409_05114_amd.serve import Server
    reqs = _requests(storage)
    srv = Server(storage, keep_results=True, realtime=False,
                 placement=placement, placement_min_side=32)
    # a budget that holds the largest request plus a few small ones, so that
    # requests queue and are admitted while others are running
    srv.budget = srv.footprint(64) + 2 * srv.footprint(24)
    recs = srv.run(reqs)
    assert len(recs) == len(reqs)
    assert srv.peak_used <= srv.budget
    assert srv.max_resident >= 2
    for r, q in zip(recs, reqs):
        assert r.flags == 0
        alone = _alone(q, storage)
        for a, b in zip(r.result, alone):
            assert np.array_equal(a, b), (q.rid, q.side)


def test_requests_arriving_later_join_the_running_batch():
    from paper_2409_05114_amd.serve import Server
    reqs = [_requests("f32")[5]] + _requests("f32")[:3]
    # staggered arrivals in real time; the first (64^3, 3000 steps) is still
    # running when the others arrive
    for k, q in enumerate(reqs):
        q.arrival = 0.05 * k
        q.steps = 3000 if k == 0 else 300
    srv = Server("f32", keep_results=False, realtime=True)
    recs = srv.run(reqs)
    assert all(r.done > r.admitted >= r.arrival for r in recs)
    assert srv.max_resident >= 2


class _UnrealizableVortex(wl.Request):
    """A Taylor-Green vortex at Mach 1.6 with the benchmark's background
    pressure p0 = rho0 theta0 instead of the served one: its pressure, and so
    its density, is negative at the vortex centres."""

    def fields_on_device(self, device):
        import torch
        fl = wl.taylor_green((self.side,) * 3, ma=self.ma, phase=self.phase)
        assert fl.rho.min() < 0
        return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(device)
                     for a in (fl.rho, fl.u, fl.theta))


def test_failed_request_is_evicted_and_the_others_are_unchanged():
    """A request whose initial state the lattice cannot represent (negative
    density at the vortex centres) raises the unrealizable flag at
    initialisation; the server evicts it after its first tick, long before
    its steps are done, and every other result still equals its run alone
    bit for bit."""
    from paper_2409_05114_amd.serve import Server, summarize
    reqs = _requests("f32")[:4]
    bad = _UnrealizableVortex(rid=len(reqs), arrival=0.0, side=24, ma=1.6,
                              tau=0.6, steps=2000, kind="tgv",
                              phase=(0.0, 0.0, 0.0), storage="f32")
    reqs = reqs[:2] + [bad] + reqs[2:]
    srv = Server("f32", keep_results=True, realtime=False)
    recs = srv.run(reqs)
    by_id = {r.rid: r for r in recs}
    rb = by_id[bad.rid]
    assert rb.failed and rb.flags & 0x1 and rb.result is None
    assert rb.steps_done < bad.steps
    for q in reqs:
        if q.rid == bad.rid:
            continue
        r = by_id[q.rid]
        assert not r.failed and r.flags == 0 and r.steps_done == q.steps
        for a, b in zip(r.result, _alone(q, "f32")):
            assert np.array_equal(a, b), q.rid
    s = summarize(recs, srv.makespan)
    assert s["evicted_requests"] == [bad.rid]


def test_flags_of_a_request_that_ends_before_its_poll_is_read_are_kept():
    """A flagged request short enough (20 steps: two ticks) to complete
    before the poll that cleared its device flag word has been read still
    reports the flag."""
    from paper_2409_05114_amd.serve import Server
    bad = _UnrealizableVortex(rid=0, arrival=0.0, side=16, ma=1.6, tau=0.6,
                              steps=20, kind="tgv", phase=(0.0, 0.0, 0.0),
                              storage="f32")
    recs = Server("f32", realtime=False).run([bad])
    assert recs[0].flags & 0x1, recs[0]


def test_shortest_remaining_work_finishes_first():
    """Default scheduling: a short request admitted together with a long one
    is advanced first and completes first, while processor sharing
    ("share") advances both every tick (equal step counts: they finish in
    the same tick).  Results are the same either way."""
    from paper_2409_05114_amd.serve import Server
    reqs = _requests("f32")
    big, small = reqs[5], reqs[0]  # 64^3 and 16^3 boxes
    big.steps, small.steps = 400, 400
    out = {}
    for policy in ("srpt", "share"):
        srv = Server("f32", keep_results=True, realtime=False, policy=policy)
        # a saturation floor below the long request's size, so that the two
        # do not share the launch (real floors hold millions of sites)
        srv.sat_sites = 2 * small.side ** 3
        recs = {r.rid: r for r in srv.run([big, small])}
        out[policy] = recs
    assert out["srpt"][small.rid].done < out["srpt"][big.rid].done
    for rid in (big.rid, small.rid):
        for a, b in zip(out["srpt"][rid].result, out["share"][rid].result):
            assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        Server("f32", policy="fifo")


def test_request_too_large_for_the_budget_is_refused():
    from paper_2409_05114_amd.serve import Server
    srv = Server("f32", realtime=False)
    srv.budget = srv.footprint(16)
    with pytest.raises(RuntimeError):
        srv.run(_requests("f32")[1:2])
