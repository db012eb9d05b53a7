"""Placement probe (lbm_probe_placement) and placement-probed allocation
(Sim(placement=k)).

The probe reads every population and writes it back: the buffer must hold
the same bytes afterwards, at either streaming parity and in every
addressing mode, and a simulation created in the buffer the probe picked
must step exactly as one in a plain allocation.
"""
import ctypes

import numpy as np
import pytest

from paper_2409_05114_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _probe(sim, reps):
    from paper_2409_05114_amd import lbm81
    ms = ctypes.c_float(-1.0)
    st = lbm81.library().lbm_probe_placement(sim.handle, reps, ctypes.byref(ms))
    return st, ms.value


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(64, 8, 4), (72, 5, 4), (3, 4, 5)],
                         ids=["row", "row-ragged", "small"])
@pytest.mark.parametrize("nsteps", [0, 3])
def test_probe_leaves_the_populations_unchanged(storage, shape, nsteps):
    import torch
    from paper_2409_05114_amd import lbm81
    fl = wl.random_state(shape, seed=5, ma_max=1.0)
    sim = lbm81.Sim(shape, storage)
    ref = lbm81.Sim(shape, storage)
    for s in (sim, ref):
        s.init(fl.rho, fl.u, fl.theta)
        s.step(nsteps, 0.6)
    torch.cuda.synchronize()
    before = sim.populations.clone()
    print(f"probe {storage} {shape} after {nsteps} steps", flush=True)
    st, ms = _probe(sim, 2)
    assert st == lbm81.LBM_OK
    assert ms > 0.0
    assert torch.equal(before, sim.populations)
    # and the run goes on as one never probed
    sim.step(2, 0.6)
    ref.step(2, 0.6)
    for a, b in zip(sim.moments(), ref.moments()):
        assert torch.equal(a, b)
    sim.close()
    ref.close()


def test_probe_rejects_bad_repetitions():
    from paper_2409_05114_amd import lbm81
    sim = lbm81.Sim((8, 4, 4), "f32")
    for reps in (0, -1, 1001):
        st, ms = _probe(sim, reps)
        assert st == -1  # LBM_E_ARG
        assert ms == 0.0
    sim.close()


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_placed_simulation_steps_as_a_plain_one(storage):
    from paper_2409_05114_amd import lbm81
    shape = (64, 16, 8)
    fl = wl.taylor_green(shape, ma=1.2)
    placed = lbm81.Sim(shape, storage, placement=3)
    plain = lbm81.Sim(shape, storage)
    assert len(placed.placement_ms) == 3
    assert all(v > 0 for v in placed.placement_ms)
    assert placed.placement_choice == int(np.argmin(placed.placement_ms))
    assert plain.placement_ms is None
    for s in (placed, plain):
        s.init(fl.rho, fl.u, fl.theta)
        s.step(7, 0.52)
    for a, b in zip(placed.moments(), plain.moments()):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    placed.close()
    plain.close()
