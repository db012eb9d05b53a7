"""Pins of the oracle's entropic collision (Sec. II, Eq. delH): alpha is the
positive root of H[f + alpha (f_eq - f)] = H[f] with the convex entropy
H[g] = sum_i g_i (ln(g_i / w_i) - 1) whose constrained minimiser is f_eq.

The oracle evaluates the entropy difference in a rearranged form (second
order in the deviation, see entropic_alpha in the oracle).  These checks do
not use that form: the defining equation is evaluated directly at 40 digits,
the near-equilibrium limit alpha -> 2 (the trapezoidal BGK of
Eq. discretelbm) follows from H being quadratic there, the discrete H
theorem H[f*] <= H[f] for beta <= 1 follows from convexity, the positivity
bound is checked on the populations, alpha is invariant under scaling of
f, and the entropic update conserves mass, momentum and energy.
"""
import mpmath as mp
import numpy as np
import pytest

from paper_2409_05114_amd import workloads as wl


@pytest.fixture(scope="module")
def basis(oracle_mod):
    c, w, th0 = oracle_mod.lattice()
    P = np.stack([np.ones(81), c[:, 0], c[:, 1], c[:, 2], (c ** 2).sum(1)])
    return c, w, th0, P


def _state(oracle_mod, basis, eps, seed=0, rho=1.1, u=(0.3, -0.2, 0.1),
           th=0.9):
    """f = f_eq - eps d with d free of the five conserved moments, scaled
    so that the largest |d_i / f_eq,i| is 1 (eps < 1 keeps f positive)."""
    c, w, th0, P = basis
    feq = oracle_mod.equilibrium(rho, np.array(u), th * th0)
    rng = np.random.default_rng(seed)
    d = rng.normal(size=81) * feq
    d = d - P.T @ np.linalg.lstsq(P.T, d, rcond=None)[0]
    d /= np.abs(d / feq).max()
    return feq - eps * d, feq


def _H(g, w):
    # g ln(g / w) - g, with 0 ln 0 = 0
    return mp.fsum(mp.mpf(gi) * (mp.log(mp.mpf(gi) / mp.mpf(wi)) - 1)
                   if gi != 0 else mp.mpf(0) for gi, wi in zip(g, w))


@pytest.mark.parametrize("eps", [0.9, 0.5, 0.1, 1e-2, 1e-3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_alpha_solves_the_entropy_condition(oracle_mod, basis, eps, seed):
    c, w, th0, P = basis
    f, feq = _state(oracle_mod, basis, eps, seed)
    a, it = oracle_mod.entropic_alpha(f, feq)
    assert a > 0 and 0 < it < 20
    mp.mp.dps = 40
    D = feq - f
    scale = float(mp.fsum(mp.mpf(fi) * (mp.mpf(di) / mp.mpf(fi)) ** 2
                          for fi, di in zip(f, D)))
    dH = float(_H(f + a * D, w) - _H(f, w))
    # f and f_eq are FP64 numbers, so their conserved moments agree to
    # ~1e-17: that bounds how well the defining equation can hold
    assert abs(dH) < 1e-9 * scale + 1e-16, (dH, scale)
    # and alpha is the positive root: H dips below H[f] before it
    assert float(_H(f + 0.5 * a * D, w) - _H(f, w)) < 0


def test_alpha_tends_to_two_near_equilibrium(oracle_mod, basis):
    dev = []
    for eps in (1e-2, 1e-3, 1e-4, 1e-5):
        f, feq = _state(oracle_mod, basis, eps, seed=3)
        a, _ = oracle_mod.entropic_alpha(f, feq)
        dev.append(abs(2.0 - a))
    dev = np.array(dev)
    # first order in the deviation (the cubic term of H): a factor 10 per
    # decade
    r = dev[:-1] / dev[1:]
    assert np.all(np.abs(r - 10.0) < 0.5), r


@pytest.mark.parametrize("beta", [0.25, 0.5, 0.9, 1.0])
def test_discrete_h_theorem(oracle_mod, basis, beta):
    c, w, th0, P = basis
    mp.mp.dps = 40
    for seed in range(3):
        f, feq = _state(oracle_mod, basis, 0.5, seed)
        a, _ = oracle_mod.entropic_alpha(f, feq)
        dH = float(_H(f + a * beta * (feq - f), w) - _H(f, w))
        if beta < 1.0:
            assert dH < 0.0
        else:
            assert abs(dH) < 1e-16


def test_positivity_bound_when_no_root(oracle_mod, basis):
    # deviation concentrated on one direction: the line f + alpha (f_eq - f)
    # leaves the positive orthant before H comes back up
    c, w, th0, P = basis
    feq = oracle_mod.equilibrium(1.0, np.zeros(3), th0)
    d = np.zeros(81)
    d[80] = 1.0
    d = d - P.T @ np.linalg.lstsq(P.T, d, rcond=None)[0]
    # population 80 at 6 times its equilibrium value, the others moved to
    # keep the moments
    f = feq + 5.0 * feq[80] / d[80] * d
    assert np.all(f > 0)
    a, it = oracle_mod.entropic_alpha(f, feq)
    g = f + a * (feq - f)
    assert g.min() >= -1e-16 * f.max()
    assert g.min() < 1e-12 * f.max()   # the bound is active
    mp.mp.dps = 40
    assert float(_H(g, w) - _H(f, w)) <= 0.0


def test_alpha_is_invariant_under_scaling(oracle_mod, basis):
    f, feq = _state(oracle_mod, basis, 0.3, seed=4)
    a, _ = oracle_mod.entropic_alpha(f, feq)
    for s in (0.25, 3.0):
        b, _ = oracle_mod.entropic_alpha(s * f, s * feq)
        assert abs(a - b) < 1e-14


def test_entropic_collision_conserves(oracle_mod):
    shape = (6, 5, 4)
    fl = wl.random_state(shape, seed=5, ma_max=1.2)
    f = oracle_mod.init(shape, fl.rho, fl.u, fl.theta)
    oracle_mod.step(shape, f, 0.6, 3, entropic=True)   # off equilibrium
    t0 = oracle_mod.totals(shape, f)
    g = f.copy()
    oracle_mod.step(shape, g, 0.6, 1, mode="collide", entropic=True)
    t1 = oracle_mod.totals(shape, g)
    assert np.allclose(t1, t0, rtol=0, atol=1e-13 * abs(t0[0]))
    assert not np.array_equal(f, g)


def test_entropic_step_is_bgk_near_equilibrium(oracle_mod):
    # a weak shear wave stays close to equilibrium: alpha = 2 + O(Kn)
    shape = (16, 16, 4)
    fl = wl.shear_wave(shape, amp_ma=0.01, noise=0.0)
    f = oracle_mod.init(shape, fl.rho, fl.u, fl.theta)
    g = f.copy()
    oracle_mod.step(shape, f, 0.8, 5)
    oracle_mod.step(shape, g, 0.8, 5, entropic=True)
    assert np.abs(f - g).max() < 1e-7 * np.abs(f).max()
