"""Pins of the oracle's series equilibrium (Sec. III; Appendix B: the quartic
weights of Eq. zeroveleqseries and the velocity expansion to third order)
and of its series step (the series where it is positive, Newton elsewhere).

What fixes it, independently of the oracle's code:
  - the series is built so that its mass, momentum and energy moments are
    those of the fluid, order by order; with the R-bar corrections they hold
    exactly, so they must hold to rounding at any Mach number and
    temperature (a dropped or mis-signed term of f2 or f3 breaks energy or
    momentum);
  - it approaches the exact entropic equilibrium as O(u^4) at theta0 and as
    O(eta^5) at rest (the next orders of the expansion);
  - it goes negative somewhere at Mach numbers of about one half (Appendix B
    remark); the step must then take the Newton solution instead."""
import numpy as np
import pytest

import oracle

C_S = None


def _cs(th0):
    return np.sqrt(5.0 * th0 / 3.0)


DIRS = [np.array(d, dtype=float) / np.linalg.norm(d)
        for d in ((1, 0, 0), (1, 0.6, -0.3), (0.2, -1, 0.7), (1, 1, 1))]


@pytest.mark.parametrize("rho", [1.0, 0.7, 1.9])
@pytest.mark.parametrize("ma,eta", [(0.05, 0.0), (0.2, 0.1), (0.4, -0.2),
                                    (0.7, 0.3), (1.0, -0.4)])
def test_series_conserves_exactly(rho, ma, eta):
    c, w, th0 = oracle.lattice()
    theta = (1 + eta) * th0
    c2 = (c ** 2).sum(1)
    for d in DIRS:
        u = ma * _cs(th0) * d
        f, _ = oracle.series_equilibrium(rho, u, theta)
        assert abs(f.sum() - rho) <= 4e-15 * rho
        assert np.abs(c.T @ f - rho * u).max() <= 4e-15 * rho
        e = (f * c2).sum()
        assert abs(e - rho * (u @ u + 3 * theta)) <= 4e-15 * e


def test_series_scales_with_density():
    """The R-bar moments are per unit density, so f~ is linear in rho."""
    _, _, th0 = oracle.lattice()
    u = (0.1, -0.05, 0.02)
    f1, _ = oracle.series_equilibrium(1.0, u, 1.1 * th0)
    f3, _ = oracle.series_equilibrium(3.0, u, 1.1 * th0)
    assert np.abs(f3 - 3 * f1).max() <= 1e-15 * np.abs(f3).max()


def test_series_is_fourth_order_in_velocity():
    c, w, th0 = oracle.lattice()
    d = DIRS[1]
    errs = []
    for ma in (0.2, 0.1, 0.05, 0.025):
        u = ma * _cs(th0) * d
        fs, _ = oracle.series_equilibrium(1.0, u, th0)
        fe = oracle.equilibrium(1.0, u, th0)
        errs.append(np.abs(fs - fe).max() / w.max())
    for a, b in zip(errs, errs[1:]):
        assert 13 < a / b < 19, errs


def test_series_is_fifth_order_in_temperature_at_rest():
    c, w, th0 = oracle.lattice()
    errs = []
    for eta in (0.2, 0.1, 0.05):
        fs, _ = oracle.series_equilibrium(1.0, (0, 0, 0), (1 + eta) * th0)
        fe = oracle.equilibrium(1.0, (0, 0, 0), (1 + eta) * th0)
        errs.append(np.abs(fs - fe).max() / w.max())
    for a, b in zip(errs, errs[1:]):
        assert 24 < a / b < 40, errs


def test_series_at_rest_and_theta0_is_the_weights():
    c, w, th0 = oracle.lattice()
    fs, pos = oracle.series_equilibrium(1.3, (0, 0, 0), th0)
    assert pos
    assert np.abs(fs - 1.3 * w).max() <= 1e-16


def test_series_positivity_flag():
    c, w, th0 = oracle.lattice()
    f, pos = oracle.series_equilibrium(1.0, 0.1 * _cs(th0) * DIRS[1], th0)
    assert pos and f.min() > 0
    f, pos = oracle.series_equilibrium(1.0, 0.6 * _cs(th0) * DIRS[0], th0)
    assert not pos and f.min() <= 0


def _uniform(shape, ma, th):
    ns = oracle.n_sites(shape)
    c, w, th0 = oracle.lattice()
    u = np.zeros((3, ns))
    u[0] = ma * _cs(th0)
    return np.ones(ns), u, np.full(ns, th)


def test_series_step_uses_series_where_positive_and_newton_elsewhere():
    """Collide-only steps: a low-Mach site relaxes towards the series, a
    Mach-0.6 site (series negative) exactly as the BGK step."""
    shape = (2, 1, 1)
    c, w, th0 = oracle.lattice()
    ns = oracle.n_sites(shape)
    rng = np.random.default_rng(3)
    rho, u, th = _uniform(shape, 0.1, th0)
    u[0, 2:] = 0.6 * _cs(th0)  # sub-lattice 1: Mach 0.6
    f0 = oracle.init(shape, rho, u, th)
    f0 *= 1 + 0.02 * rng.uniform(-1, 1, f0.shape)
    assert oracle.series_fallbacks(shape, f0) == 2
    tau = 0.6
    om = 2 / (2 * tau + 1)
    fs = oracle.step(shape, f0.copy(), tau, 1, mode="collide", series=True)
    fb = oracle.step(shape, f0.copy(), tau, 1, mode="collide")
    mr, mu, mt = oracle.moments(shape, f0)
    for s in range(ns):
        eq, pos = oracle.series_equilibrium(mr[s], mu[:, s], mt[s])
        if s < 2:
            assert pos
            assert np.abs(fs[s] - (f0[s] + om * (eq - f0[s]))).max() <= 1e-16
        else:
            assert not pos
            assert np.array_equal(fs[s], fb[s])


def test_series_step_conserves():
    shape = (4, 3, 2)
    c, w, th0 = oracle.lattice()
    rho, u, th = _uniform(shape, 0.15, 1.05 * th0)
    rng = np.random.default_rng(5)
    u[1] = 0.05 * _cs(th0) * rng.uniform(-1, 1, u.shape[1])
    rho = rho * (1 + 0.01 * rng.uniform(-1, 1, rho.shape))
    f = oracle.init(shape, rho, u, th)
    t0 = oracle.totals(shape, f)
    oracle.step(shape, f, 0.55, 6, series=True)
    t1 = oracle.totals(shape, f)
    assert np.abs(t1 - t0).max() <= 1e-12 * np.abs(t0).max()
