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
