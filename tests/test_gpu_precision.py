"""Precision form: FP32 / FP16 / BF16 deviation storage with FP32 compute,
against the FP64 CPU oracle on the same seeded inputs.

Error metric as in the FP64 parity tests (max-norm relative per field).
Bars, per storage: FP32 1e-5, FP16 1e-3 (the target), BF16 1e-2 -- BF16's
8-bit mantissa misses the 1e-3 target on these transonic flows, which the
measured values here document.
"""
import numpy as np
import pytest

from paper_2409_05114_amd import workloads as wl

from parity import field_errors, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

BARS = {"f32": 1e-5, "f16": 1e-3, "bf16": 1e-2}


@pytest.fixture(scope="module", autouse=True)
def _setup(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle_mod.set_threads(16)


@pytest.fixture(scope="module")
def tgv_reference():
    # 64^3 for 60 steps: the vortex keeps about a third of its velocity
    # (on 32^3 it would decay by 1e-6 within 200 steps, and the velocity
    # metric would measure rounding of a vanishing field)
    fl = wl.taylor_green((64, 64, 64), ma=1.2)
    mo, _ = oracle_run(fl, 60, 0.52)
    return fl, mo


@pytest.fixture(scope="module")
def shear_reference():
    fl = wl.shear_layer((64, 64, 32), ma=2.0, delta=4.0)
    mo, _ = oracle_run(fl, 100, 0.52)
    return fl, mo


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_taylor_green_ma12_low_precision(storage, tgv_reference, record_property):
    fl, mo = tgv_reference
    m, _, _, flags = gpu_run(fl, 60, 0.52, storage=storage)
    assert flags == 0
    e = field_errors(m, mo)
    record_property("errors", e)
    print(storage, e)
    assert max(e.values()) < BARS[storage], e


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_shear_layer_ma2_low_precision(storage, shear_reference, record_property):
    fl, mo = shear_reference
    m, _, _, flags = gpu_run(fl, 100, 0.52, storage=storage)
    assert flags == 0
    e = field_errors(m, mo)
    record_property("errors", e)
    print(storage, e)
    assert max(e.values()) < BARS[storage], e


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_low_precision_conserves_mass(storage):
    """Mass drift of the deviation forms over 100 steps: FP32 arithmetic
    gives ~1e-8 per step; BF16 rounding of smooth fields is correlated
    between sites and drifts by ~1e-4 (round-to-nearest-even, no stochastic
    rounding)."""
    from paper_2409_05114_amd import lbm81
    fl = wl.taylor_green((64, 32, 32), ma=1.2)
    sim = lbm81.Sim(fl.shape, storage)
    sim.init(fl.rho, fl.u, fl.theta)
    t0, _ = sim.totals()
    sim.step(100, 0.52)
    t1, flags = sim.totals()
    sim.close()
    assert flags == 0
    drift = abs(t1[0] - t0[0]) / t0[0]
    print(storage, "mass drift", drift)
    assert drift < {"f32": 1e-5, "f16": 1e-5, "bf16": 1e-3}[storage]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(4, 4, 4), (64, 4, 4), (8, 4, 6), (72, 6, 4)],
                         ids=["row-4", "rowx-4", "row-small", "row-ragged"])
def test_small_sides_low_precision(storage, shape):
    """Sides of 4 (the smallest row-mode side), where links of length 3 and
    4 wrap the whole period, and a ragged row, in each storage form: a
    rough random state against the oracle after an even, an odd and an even
    step, to the storage bars (the 16-bit forms' one-sided wraps and, at
    (64, 4, 4), the row exchange)."""
    fl = wl.random_state(shape, seed=31, ma_max=0.8)
    mo, _ = oracle_run(fl, 3, 0.6)
    m, _, _, flags = gpu_run(fl, 3, 0.6, storage=storage)
    assert flags == 0
    e = field_errors(m, mo)
    print(storage, shape, e)
    assert max(e.values()) < BARS[storage], e
