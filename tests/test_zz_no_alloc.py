"""lbm_create_static (the entry point for callers that cannot allocate device
memory) against lbm_create with a caller workspace, through the C ABI: the
same kernels run, so populations, moments, totals, flags and diagnostics are
bitwise equal.  Two calls in a row, the second on a smaller grid; the first
leaves a raised flag in the shared static workspace, which creating the
second simulation must clear."""
import numpy as np
import pytest

from paper_2409_05114_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(shape, storage, fields, steps, tau, static):
    import torch
    from paper_2409_05114_amd import lbm81
    print(f"no-alloc case: shape {shape}, storage {storage}, steps {steps}, "
          f"static {static}", flush=True)
    sim = lbm81.Sim(shape, storage, static_workspace=static)
    assert (sim.workspace is None) == static
    sim.init(fields.rho, fields.u, fields.theta)
    sim.step(steps, tau)
    out = {"moments": [t.clone() for t in sim.moments()]}
    torch.cuda.synchronize()
    out["populations"] = sim.populations.clone()
    return sim, out


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_static_workspace_equals_caller_workspace(storage):
    import torch

    # call 1: a vortex with one unrealizable site (the init flags it and
    # gives it the rest weights); the flag is left unread in the scratch
    big, tau = (40, 20, 16), 0.55
    f1 = wl.taylor_green(big, ma=1.1)
    f1.rho[123] = -1.0
    ref, r = _run(big, storage, f1, 5, tau, static=False)
    sim, s = _run(big, storage, f1, 5, tau, static=True)
    assert torch.equal(r["populations"], s["populations"])
    for a, b in zip(r["moments"], s["moments"]):
        assert torch.equal(a, b)
    assert sim.flags(clear=False) == ref.flags(clear=False) != 0
    sim.close()
    ref.close()

    # call 2: a smaller realizable grid; creating it cleared the flag word
    small = (12, 8, 6)
    f2 = wl.shear_wave(small, amp_ma=0.5, noise=1e-3, seed=4)
    ref, r = _run(small, storage, f2, 7, 0.6, static=False)
    sim, s = _run(small, storage, f2, 7, 0.6, static=True)
    assert torch.equal(r["populations"], s["populations"])
    for a, b in zip(r["moments"], s["moments"]):
        assert torch.equal(a, b)
    tr, fr = ref.totals()
    ts, fs = sim.totals()
    assert fr == fs == 0
    assert np.array_equal(tr, ts)
    dr, ds = ref.diagnostics(), sim.diagnostics()
    assert dr == ds
    sim.close()
    ref.close()
