"""Continuous-batching server for independent RD3Q81 simulations.

Requests (periodic boxes of different sizes, Mach numbers, relaxation times
and step counts) arrive over time.  The server keeps every admitted
simulation's populations resident in HBM, admits queued requests first come
first served as soon as their memory footprint fits the budget, and advances
resident simulations together: every tick issues batched stream-collide
launches (lbm_step_batch: one kernel per streaming parity over all the
simulations it advances, one workgroup per tile) over the simulations with the least
remaining work, enough of them to fill the device (or, with policy "share",
over all of them), so small and large simulations share the device and short
requests are not held behind long ones.  A simulation that has taken its steps
gets its moments read back and its memory freed, which lets the next request
in.  Latency = completion - arrival; queue wait = admission - arrival.

All device work is enqueued on one HIP stream; the host loop runs at most a
few ticks ahead of the device (events), and never synchronises on a
simulation other than to detect completions.

Failure handling: after every tick the device flag words of the resident
simulations (unrealizable or non-finite state, Newton cap, non-positive
population) are gathered and copied to the host asynchronously, one launch
per batch of simulations (lbm_flags_batch); a simulation whose word is nonzero is
evicted at once -- it leaves the batch, its memory is released, and its
record carries the flags and the steps it took -- while the others continue
untouched (each simulation owns its populations and its flag word).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm81

STEPS_PER_TICK_MAX = 16
TICKS_AHEAD = 3
# Scheduling ("srpt"): each tick advances the resident simulations with the
# least remaining work (steps left x sites), as many as it takes for the
# launch to hold SAT_SITES sites -- enough to keep the GPU busy (a 128^3 box,
# 4.2M sites, alone already steps at ~97 % of the largest grids' rate).
# "share": every resident simulation every tick (processor sharing).
SAT_SITES = 1 << 23
# Starvation bound of "srpt": a resident simulation left out of this many
# consecutive ticks joins the next launch whatever its remaining work.
MAX_SKIP = 64


def schedule(jobs, policy="srpt", sat_sites=SAT_SITES, max_skip=MAX_SKIP):
    """Indices of the jobs to advance this tick.  jobs: sequence of
    (remaining work, sites, ticks skipped, id).  "share": all of them;
    "srpt": those skipped max_skip times, then the least remaining work
    first (ties by id) until the chosen ones hold sat_sites sites."""
    if policy == "share":
        return list(range(len(jobs)))
    chosen = [k for k, j in enumerate(jobs) if j[2] >= max_skip]
    sites = sum(jobs[k][1] for k in chosen)
    for k in sorted(range(len(jobs)), key=lambda k: (jobs[k][0], jobs[k][3])):
        if sites >= sat_sites:
            break
        if k not in chosen:
            chosen.append(k)
            sites += jobs[k][1]
    return chosen
# flag polls: one pinned row per tick (a slot per resident simulation),
# reused after POLL_SLOTS ticks (more than the ticks in flight, so a row is
# read before it is reused)
POLL_SLOTS = TICKS_AHEAD + 2


@dataclass
class Record:
    rid: int
    side: int
    steps: int
    sites: int
    arrival: float
    admitted: float = float("nan")
    done: float = float("nan")
    flags: int = 0
    result: tuple | None = None
    failed: bool = False  # evicted on a device flag before its last step
    steps_done: int = 0

    @property
    def latency(self):
        return self.done - self.arrival

    @property
    def queue_wait(self):
        return self.admitted - self.arrival


@dataclass
class _Job:
    req: object
    rec: Record
    sim: lbm81.Sim
    left: int
    out: tuple | None = None
    event: object | None = None
    flag_host: object | None = None
    skipped: int = 0  # consecutive ticks left out (scheduling)


class Server:
    """storage: population storage of every simulation ("f32", "bf16", ...);
    memory_bytes: HBM budget for resident simulations (default 85 % of the
    device memory free at construction, counting what torch's caching
    allocator holds unused); keep_results: copy each result's
    moments (rho, u, theta) to the host in its Record; placement: a request
    with a side of at least placement_min_side gets the fastest of up to
    `placement` candidate population buffers (lbm81.Sim(placement=...)),
    probed when it is admitted (the probe waits for the work queued on the
    server's stream)."""

    def __init__(self, storage="f32", memory_bytes=None, keep_results=False,
                 device=None, realtime=True, policy="srpt", placement=1,
                 placement_min_side=128):
        import torch

        self.torch = torch
        self.storage = storage
        self.device = torch.device(device or "cuda:0")
        free, _ = torch.cuda.mem_get_info(self.device)
        # memory torch's caching allocator holds but does not use is free for
        # the server's own allocations, which go through that allocator
        free += (torch.cuda.memory_reserved(self.device)
                 - torch.cuda.memory_allocated(self.device))
        self.budget = int(memory_bytes if memory_bytes is not None else 0.85 * free)
        self.keep = keep_results
        self.realtime = realtime
        if policy not in ("srpt", "share"):
            raise ValueError(f"unknown scheduling policy {policy!r}")
        self.policy = policy
        self.placement = int(placement)
        self.placement_min_side = int(placement_min_side)
        self.sat_sites = SAT_SITES
        self.stream = torch.cuda.current_stream(self.device)
        self.used = 0
        self.peak_used = 0
        self.max_resident = 0
        self.launch_steps = 0
        self._polls = None

    def footprint(self, side):
        """Bytes a request holds while resident: populations, workspace and
        the FP64 moment outputs (the initial fields use the same room)."""
        n = 2 * side ** 3
        return (lbm81.lbm_population_bytes(side, side, side, self.storage)
                + lbm81.lbm_workspace_bytes(side, side, side) + 5 * 8 * n)

    def _admit(self, req, now):
        k = self.placement if req.side >= self.placement_min_side else 1
        sim = lbm81.Sim((req.side,) * 3, self.storage, stream=self.stream,
                        device=self.device, placement=k)
        rho, u, th = req.fields_on_device(self.device)
        sim.init(rho, u, th)
        rec = Record(req.rid, req.side, req.steps, req.sites, req.arrival,
                     admitted=now)
        self.used += self.footprint(req.side)
        self.peak_used = max(self.peak_used, self.used)
        return _Job(req, rec, sim, req.steps)

    def _poll_row(self, slot, n):
        """Pinned int32 row of at least n slots for tick slot `slot` (the
        pool grows by whole batches; rows of a replaced pool stay alive
        while the ticks that hold them are in flight)."""
        torch = self.torch
        cap = 0 if self._polls is None else self._polls.shape[1]
        if n > cap:
            cap = max(n, 2 * cap, lbm81.BATCH_MAX)
            cap = -(-cap // lbm81.BATCH_MAX) * lbm81.BATCH_MAX
            self._polls = torch.zeros((POLL_SLOTS, cap), dtype=torch.int32,
                                      pin_memory=True)
        return self._polls[slot]

    def _schedule(self, active):
        """The resident simulations to advance this tick (`schedule`)."""
        picked = schedule([(j.left * j.req.sites, j.req.sites, j.skipped,
                            j.rec.rid) for j in active],
                          self.policy, self.sat_sites)
        for j in active:
            j.skipped += 1
        run_now = [active[k] for k in picked]
        for j in run_now:
            j.skipped = 0
        return run_now

    def _finish(self, j, evicted):
        """Queue the read-back (unless evicted) and the final flag copy of
        job j; its memory is released once the stream has passed them."""
        torch = self.torch
        j.out = None if evicted else j.sim.moments()
        j.rec.failed = evicted
        j.rec.steps_done = j.req.steps - j.left
        j.flag_host = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        j.sim.flags_async(j.flag_host)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        j.event = ev

    def run(self, requests, progress=None):
        """Serve `requests` (sorted by arrival, seconds from the start) and
        return one Record per request.  In real-time mode arrivals follow the
        wall clock; otherwise every request is available at time 0.
        progress: optional callable(record, done, total), called as each
        request completes or is evicted."""
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        active, finishing, records = [], [], []
        ticks = collections.deque()
        tick_no = 0
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if self.realtime else \
            (lambda: float("inf"))
        while pending or queue or active or finishing:
            now = clock()
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admission: first come first served while the footprint fits
            while queue and self.used + self.footprint(queue[0].side) <= self.budget:
                req = queue.popleft()
                active.append(self._admit(req, time.perf_counter() - t0))
            if queue and not active and not finishing:
                raise RuntimeError(
                    f"request {queue[0].rid} (side {queue[0].side}) does not "
                    f"fit the memory budget of {self.budget} bytes")
            self.max_resident = max(self.max_resident, len(active))
            if active:
                # advance each scheduled simulation by its own count, the
                # steps it still needs capped per tick; those that need
                # fewer drop out of the later launches of the tick
                run_now = self._schedule(active)
                ks = [min(STEPS_PER_TICK_MAX, j.left) for j in run_now]
                for c in range(0, len(run_now), lbm81.BATCH_MAX):
                    chunk = run_now[c:c + lbm81.BATCH_MAX]
                    lbm81.lbm_step_batch([j.sim for j in chunk],
                                         ks[c:c + lbm81.BATCH_MAX],
                                         [j.req.tau for j in chunk],
                                         stream=self.stream)
                self.launch_steps += max(ks)
                for j, k in zip(run_now, ks):
                    j.left -= k
                done = [j for j in active if j.left == 0]
                active = [j for j in active if j.left > 0]
                for j in done:
                    self._finish(j, evicted=False)
                    finishing.append(j)
                # poll the flag word of every simulation still running, one
                # gather per batch of simulations (lbm_flags_batch)
                row = self._poll_row(tick_no % POLL_SLOTS, len(active))
                for c in range(0, len(active), lbm81.BATCH_MAX):
                    lbm81.lbm_flags_batch(
                        [j.sim for j in active[c:c + lbm81.BATCH_MAX]],
                        row[c:c + lbm81.BATCH_MAX], stream=self.stream)
                ev = torch.cuda.Event()
                ev.record(self.stream)
                ticks.append((ev, row, list(active)))
                tick_no += 1
                while len(ticks) > TICKS_AHEAD:
                    ev, row, polled = ticks.popleft()
                    ev.synchronize()
                    bad = set()
                    for k, j in enumerate(polled):
                        f = int(row[k])
                        if f:
                            # (the poll cleared the device word: the record
                            # keeps the bits even if the job has finished)
                            j.rec.flags |= f
                            if j.sim is not None and j.event is None:
                                bad.add(id(j))
                    if bad:
                        # evict: out of the batch at once, memory released
                        # once the stream has passed the queued work
                        for j in [j for j in active if id(j) in bad]:
                            self._finish(j, evicted=True)
                            finishing.append(j)
                        active = [j for j in active if id(j) not in bad]
            # completions
            still = []
            for j in finishing:
                if j.event.query():
                    j.rec.done = time.perf_counter() - t0
                    j.rec.flags |= int(j.flag_host[0])
                    if self.keep and j.out is not None:
                        j.rec.result = tuple(t.cpu().numpy() for t in j.out)
                    j.sim.close()
                    j.sim = None
                    j.out = None
                    self.used -= self.footprint(j.req.side)
                    records.append(j.rec)
                    if progress is not None:
                        progress(j.rec, len(records), len(requests))
                else:
                    still.append(j)
            finishing = still
            if not active and finishing:
                finishing[0].event.synchronize()
            elif not active and not finishing and not queue and pending:
                # idle until the next arrival
                time.sleep(max(0.0, min(0.01, pending[0].arrival - clock())))
        self.makespan = time.perf_counter() - t0
        # flag polls still unread (the device words they cleared)
        while ticks:
            ev, row, polled = ticks.popleft()
            ev.synchronize()
            for k, j in enumerate(polled):
                j.rec.flags |= int(row[k])
        return sorted(records, key=lambda r: r.rid)


def summarize(records, makespan):
    """Latency and queue-wait percentiles over the requests that completed
    (evicted ones are listed apart); throughput over all steps taken."""
    ok = [r for r in records if not r.failed] or records
    lat = np.array([r.latency for r in ok])
    wait = np.array([r.queue_wait for r in ok])
    work = sum(r.sites * r.steps_done for r in records)
    return {
        "requests": len(records),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "p50_queue_wait_s": float(np.percentile(wait, 50)),
        "p99_queue_wait_s": float(np.percentile(wait, 99)),
        "makespan_s": makespan,
        "aggregate_mlups": work / makespan / 1e6,
        "flags": int(np.bitwise_or.reduce([r.flags for r in records]))
        if records else 0,
        "flagged_requests": [r.rid for r in records if r.flags],
        "evicted_requests": [r.rid for r in records if r.failed],
    }
