"""Host logic of the Taylor-Green time-series driver (Sec. IV.C): the
conversion of (n, Ma, Re) into lattice parameters and the kinetic-energy
budget estimator.  No GPU."""
import math

import numpy as np

from paper_2409_05114_amd import tgv
from paper_2409_05114_amd import workloads as wl


def test_parameters_follow_the_definitions():
    # Re = V0 L / nu with L = n / (2 pi), V0 = Ma c_s, nu = tau theta0
    for n, ma, re in [(512, 0.1, 1600.0), (512, 1.0, 400.0), (64, 0.5, 100.0)]:
        p = tgv.parameters(n, ma, re)
        L = n / (2 * math.pi)
        assert math.isclose(p["L"], L)
        assert math.isclose(p["V0"], ma * math.sqrt(5.0 / 3.0 * wl.THETA0))
        assert math.isclose(p["V0"] * p["L"] / (p["tau"] * wl.THETA0), re)
        assert math.isclose(p["omega"], 2.0 / (2.0 * p["tau"] + 1.0))
        assert math.isclose(p["t_conv"] * p["V0"], L)


def test_energy_budget_is_one_for_viscous_decay():
    """A single Fourier mode decaying viscously, KE = KE0 exp(-2 nu k^2 t),
    has eps = k^2 KE (enstrophy of a shear wave u = U sin(k y): w = -U k
    cos(k y), so <w^2>/2 = k^2 <u^2>/2); the estimator returns 1 up to the
    central difference's O(dt^2) error."""
    nu, k, ke0 = 0.01, 2 * math.pi / 64, 1e-3
    t = np.arange(0, 4000, 50.0)
    ke = ke0 * np.exp(-2 * nu * k * k * t)
    eps = k * k * ke
    r = tgv.energy_budget(list(t), list(ke), list(eps), nu)
    assert len(r) == len(t) - 2
    rate = 2 * nu * k * k * 50.0
    # central difference of exp: sinh(h)/h with h = rate
    expected = math.sinh(rate) / rate
    np.testing.assert_allclose(r, expected, rtol=1e-12)
    assert abs(expected - 1) < 1e-4


def test_energy_budget_detects_extra_dissipation():
    nu, k = 0.01, 0.1
    t = np.arange(0, 1000, 10.0)
    ke = np.exp(-2 * 1.3 * nu * k * k * t)  # 30 % faster than 2 nu eps
    eps = k * k * ke
    r = tgv.energy_budget(list(t), list(ke), list(eps), nu)
    np.testing.assert_allclose(r, 1.3, rtol=1e-3)
