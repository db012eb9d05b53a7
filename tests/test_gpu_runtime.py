"""GPU tests of the library's runtime behaviour through the C ABI: error
paths forced from the host, device flags, batched stepping (serving) and
checkpoint / resume."""
import ctypes

import numpy as np
import pytest

from paper_2409_05114_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lbm():
    from paper_2409_05114_amd import lbm81
    return lbm81


def test_bad_tau_and_steps_are_rejected():
    lbm81 = _lbm()
    sim = lbm81.Sim((8, 8, 8), "f64")
    fl = wl.uniform((8, 8, 8))
    sim.init(fl.rho, fl.u, fl.theta)
    for tau in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(lbm81.LbmError):
            sim.step(1, tau)
    with pytest.raises(lbm81.LbmError):
        sim.step(-1, 0.8)
    assert sim.step_count == 0
    sim.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_unrealizable_input_is_flagged(storage):
    lbm81 = _lbm()
    fl = wl.uniform((8, 8, 8))
    fl.theta[5] = -0.1
    fl.rho[17] = 0.0
    sim = lbm81.Sim(fl.shape, storage)
    sim.init(fl.rho, fl.u, fl.theta)
    with pytest.raises(lbm81.LbmError) as ei:
        sim.totals()
    assert ei.value.status == -4
    # the flag word was cleared by the read
    assert sim.flags() == 0
    sim.close()


def test_nonfinite_population_is_flagged_and_kept():
    """A NaN written into one population from the host: the site is flagged
    and not collided; far-away sites are untouched by it."""
    lbm81 = _lbm()
    import torch
    shape = (64, 8, 8)
    fl = wl.uniform(shape, rho=1.0, u=(0.05, 0.0, 0.0))
    sim = lbm81.Sim(shape, "f64")
    sim.init(fl.rho, fl.u, fl.theta)
    ref = lbm81.Sim(shape, "f64")
    ref.init(fl.rho, fl.u, fl.theta)
    pops = sim.populations.view(torch.float64).view(81, -1)
    pops[0, 0] = float("nan")
    sim.step(1, 0.8)
    ref.step(1, 0.8)
    assert sim.flags() & lbm81.FLAG_NONFINITE
    a = sim.populations_f64()
    b = ref.populations_f64()
    far = torch.arange(a.shape[1], device=a.device)
    x = far % 64
    mask = (x > 10) & (x < 50)
    assert torch.equal(a[:, mask], b[:, mask])
    sim.close()
    ref.close()


def test_newton_cap_is_flagged_for_extreme_states():
    """A state far outside the lattice's range (Ma 6, cold) cannot be
    matched; the solve stops at its cap and the flag is raised."""
    lbm81 = _lbm()
    fl = wl.uniform((8, 8, 8), rho=1.0, u=(6.0 * wl.C_S, 0.0, 0.0),
                    theta=0.2 * wl.THETA0)
    sim = lbm81.Sim(fl.shape, "f64")
    sim.init(fl.rho, fl.u, fl.theta)
    f = sim.flags()
    assert f & (lbm81.FLAG_NEWTON | lbm81.FLAG_UNREALIZABLE)
    sim.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_batched_step_equals_individual_steps(storage):
    """Serving: one batched launch per step over simulations of different
    sizes, taus and parities gives bitwise the same populations as stepping
    each simulation alone."""
    lbm81 = _lbm()
    import torch
    cases = [((64, 8, 8), 0.6, 0), ((48, 12, 8), 0.8, 1), ((64, 4, 16), 0.52, 3),
             ((128, 6, 4), 0.7, 1), ((256, 4, 5), 0.55, 0), ((512, 4, 4), 0.6, 1)]
    sims, alone, taus = [], [], []
    for k, (shape, tau, pre) in enumerate(cases):
        fl = wl.taylor_green(shape, ma=0.8 + 0.2 * k)
        a = lbm81.Sim(shape, storage)
        b = lbm81.Sim(shape, storage)
        for s in (a, b):
            s.init(fl.rho, fl.u, fl.theta)
            s.step(pre, tau)  # different parities at batch time
        sims.append(a)
        alone.append(b)
        taus.append(tau)
    row_only = [sims[0], sims[2]]
    for _ in range(5):
        lbm81.lbm_step_batch(sims, 1, taus)
    for s, t in zip(alone, taus):
        s.step(5, t)
    torch.cuda.synchronize()
    for a, b in zip(sims, alone):
        assert a.step_count == b.step_count
        assert torch.equal(a.populations, b.populations)
    # and a batch of row-aligned grids only (wavefront-uniform addressing)
    for _ in range(3):
        lbm81.lbm_step_batch(row_only, 1, [taus[0], taus[2]])
    for s, t in zip([alone[0], alone[2]], [taus[0], taus[2]]):
        s.step(3, t)
    torch.cuda.synchronize()
    for a, b in zip(row_only, [alone[0], alone[2]]):
        assert torch.equal(a.populations, b.populations)
    for s in sims + alone:
        s.close()


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_batched_step_counts_per_simulation(storage):
    """lbm_step_batch advances each simulation by its own step count (some
    zero); those that finish drop out of the later launches.  Every result
    and step counter equals the same simulation stepped alone."""
    lbm81 = _lbm()
    import torch
    cases = [((64, 8, 8), 0.6, 0, 5), ((48, 12, 8), 0.8, 1, 0),
             ((64, 4, 16), 0.52, 3, 2), ((128, 6, 4), 0.7, 1, 7),
             ((40, 5, 6), 0.55, 0, 1)]
    sims, alone = [], []
    for k, (shape, tau, pre, n) in enumerate(cases):
        fl = wl.taylor_green(shape, ma=0.7 + 0.2 * k)
        a, b = lbm81.Sim(shape, storage), lbm81.Sim(shape, storage)
        for s in (a, b):
            s.init(fl.rho, fl.u, fl.theta)
            s.step(pre, tau)
        sims.append(a)
        alone.append(b)
    lbm81.lbm_step_batch(sims, [c[3] for c in cases], [c[1] for c in cases])
    for b, c in zip(alone, cases):
        b.step(c[3], c[1])
    torch.cuda.synchronize()
    for a, b, c in zip(sims, alone, cases):
        assert a.step_count == b.step_count == c[2] + c[3]
        assert torch.equal(a.populations, b.populations)
    with pytest.raises(lbm81.LbmError):
        lbm81.lbm_step_batch(sims[:2], [1, -1], [0.6, 0.8])
    with pytest.raises(ValueError):
        lbm81.lbm_step_batch(sims[:2], [1], [0.6, 0.8])
    for s in sims + alone:
        s.close()


def test_batch_orders_against_the_simulations_streams():
    """Simulations created on their own streams and stepped in a batch on a
    third stream: the batch waits for their queued init, and their later
    read-back waits for the batch (events), with no host synchronisation
    in between."""
    lbm81 = _lbm()
    import torch
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    shapes = [(64, 8, 8), (48, 6, 10)]
    fields = [wl.taylor_green(sh, ma=1.0) for sh in shapes]
    ref = []
    for sh, fl in zip(shapes, fields):
        r = lbm81.Sim(sh, "f64")
        r.init(fl.rho, fl.u, fl.theta)
        r.step(4, 0.6)
        ref.append(r)
    torch.cuda.synchronize()
    sims = [lbm81.Sim(sh, "f64", stream=st)
            for sh, st in zip(shapes, (s1, s2))]
    for s, fl in zip(sims, fields):
        s.init(fl.rho, fl.u, fl.theta)
    lbm81.lbm_step_batch(sims, [4, 4], [0.6, 0.6], stream=s3)
    outs = [s.moments() for s in sims]
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        for a, b in zip(o, r.moments()):
            assert torch.equal(a, b)
    for s in sims + ref:
        s.close()


def _xy_fields(shape):
    """Smooth fields that depend on x and y only."""
    x, y, _ = wl.positions(shape)
    nx, ny = shape[0], shape[1]
    kx, ky = 2 * np.pi * x / nx, 2 * np.pi * y / ny
    rho = 1.0 + 0.1 * np.sin(kx) * np.cos(ky)
    ux = 0.4 * wl.C_S * np.sin(ky)
    uy = 0.3 * wl.C_S * np.cos(kx)
    uz = 0.25 * wl.C_S * np.sin(kx + ky)
    theta = wl.THETA0 * (1.0 + 0.1 * np.cos(kx))
    return wl._pack(shape, rho, ux, uy, uz, theta)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_row_exchange_matches_plain_odd_step(storage):
    """With 16-bit storage the odd step of a grid whose workgroups cover
    whole rows, here (64, 5, 4), routes its loads and stores through the LDS
    row exchange; (64, 5, 5) takes the plain path.  The problem does not
    depend on z, so both grids must hold the same values bit for bit, in
    every z-plane, after odd and even steps."""
    lbm81 = _lbm()
    import torch
    a_shape, b_shape = (64, 5, 4), (64, 5, 5)
    a = lbm81.Sim(a_shape, storage)
    b = lbm81.Sim(b_shape, storage)
    fa, fb = _xy_fields(a_shape), _xy_fields(b_shape)
    a.init(fa.rho, fa.u, fa.theta)
    b.init(fb.rho, fb.u, fb.theta)
    for n in (1, 1, 1, 4):
        a.step(n, 0.55)
        b.step(n, 0.55)
        pa = a.populations_f64().view(81, 2, 4, 5, 64)
        pb = b.populations_f64().view(81, 2, 5, 5, 64)
        for z in range(4):
            assert torch.equal(pa[:, :, z], pb[:, :, 0]), (a.step_count, z)
        assert torch.equal(pb[:, :, 4], pb[:, :, 0])
    assert a.flags() == 0 and b.flags() == 0
    a.close()
    b.close()


@pytest.mark.parametrize("tau", [0.5, 0.9])
def test_populations_stay_positive_for_omega_at_most_one(tau):
    """omega = 2/(2 tau + 1) <= 1: the GPU update keeps every population
    positive from a rough random state, and raises no flag."""
    lbm81 = _lbm()
    shape = (64, 6, 5)
    fl = wl.random_state(shape, seed=13, ma_max=1.5)
    sim = lbm81.Sim(shape, "f64")
    sim.init(fl.rho, fl.u, fl.theta)
    for _ in range(3):
        sim.step(7, tau)
        assert float(sim.populations_f64().min()) > 0
    assert sim.flags() == 0
    sim.close()


def test_batch_rejects_mixed_storage_and_duplicates():
    lbm81 = _lbm()
    a = lbm81.Sim((8, 8, 8), "f64")
    b = lbm81.Sim((8, 8, 8), "f32")
    with pytest.raises(lbm81.LbmError):
        lbm81.lbm_step_batch([a, b], 1, [0.8, 0.8])
    with pytest.raises(lbm81.LbmError):
        lbm81.lbm_step_batch([a, a], 1, [0.8, 0.8])
    c = lbm81.Sim((2, 8, 8), "f64")
    with pytest.raises(lbm81.LbmError):
        lbm81.lbm_step_batch([c], 1, [0.8])
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_checkpoint_resume_is_bitwise(storage):
    lbm81 = _lbm()
    import torch
    shape = (64, 8, 8)
    fl = wl.taylor_green(shape, ma=1.2)
    a = lbm81.Sim(shape, storage)
    a.init(fl.rho, fl.u, fl.theta)
    a.step(7, 0.55)
    ck = a.checkpoint()
    a.step(6, 0.55)
    b = lbm81.Sim(shape, storage)
    b.restore(ck)
    assert b.step_count == 7
    b.step(6, 0.55)
    torch.cuda.synchronize()
    assert torch.equal(a.populations, b.populations)
    ra, ua, ta = a.moments()
    rb, ub, tb = b.moments()
    assert torch.equal(ra, rb) and torch.equal(ua, ub) and torch.equal(ta, tb)
    a.close()
    b.close()


def test_explicit_stream():
    """Work is enqueued on the stream given at creation."""
    lbm81 = _lbm()
    import torch
    s = torch.cuda.Stream()
    shape = (64, 4, 4)
    fl = wl.taylor_green(shape, ma=1.0)
    a = lbm81.Sim(shape, "f64", stream=s)
    b = lbm81.Sim(shape, "f64")
    a.init(fl.rho, fl.u, fl.theta)
    b.init(fl.rho, fl.u, fl.theta)
    a.step(4, 0.6)
    b.step(4, 0.6)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(a.populations, b.populations)
    a.close()
    b.close()


def test_flags_batch_gathers_and_clears_every_flag_word():
    """lbm_flags_batch returns each simulation's flag word (here: two whose
    initial state is unrealizable, three clean ones) and clears them, like
    lbm_flags_async on each; simulations on another stream are ordered."""
    lbm81 = _lbm()
    import torch
    side = torch.cuda.Stream()
    sims, expect = [], []
    for k in range(5):
        shape = (8 + 4 * k, 6, 5)
        fl = wl.taylor_green(shape, ma=0.5)
        if k in (1, 3):
            fl.rho[7] = -1.0  # unrealizable: LBM_FLAG_UNREALIZABLE at init
        s = lbm81.Sim(shape, "f64", stream=side if k == 4 else None)
        s.init(fl.rho, fl.u, fl.theta)
        sims.append(s)
        expect.append(lbm81.FLAG_UNREALIZABLE if k in (1, 3) else 0)
    host = torch.full((8,), -1, dtype=torch.int32, pin_memory=True)
    lbm81.lbm_flags_batch(sims, host)
    torch.cuda.synchronize()
    assert host[:5].tolist() == expect
    assert host[5:].tolist() == [-1, -1, -1]  # nothing written past n
    for s in sims:
        assert s.flags(clear=False) == 0  # cleared on the device
    with pytest.raises(ValueError):
        lbm81.lbm_flags_batch(sims, host[:3])
    for s in sims:
        s.close()
