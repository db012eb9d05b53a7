"""Pins of the oracle's Taylor-Green diagnostics (Sec. IV.C): mean kinetic
energy <rho u.u/2> and mean enstrophy <rho w.w/2>, w = curl u, with every
derivative a central difference over one cell on the same sub-lattice.

For fields built from sines of wavenumber k = 2 pi / N the discrete sums are
known in closed form: the mean of sin^2 over a full period of N >= 3 points
is exactly 1/2 (also on the sub-lattice shifted by half a cell), and the
central difference of sin(k x + phi) is sin(k) cos(k x + phi).  The
Taylor-Green velocity field of Sec. IV.C at constant density therefore has
KE = V0^2 / 8 and eps = (3/8) V0^2 sin^2(k); its curl adds the two terms of
w_z constructively, so a sign or axis slip in the curl changes eps.
"""
import numpy as np
import pytest

from paper_2409_05114_amd import workloads as wl


def _tgv_unit_density(n, v0, phase=(0.0, 0.0, 0.0)):
    fl = wl.taylor_green((n, n, n), ma=v0 / wl.C_S, phase=phase)
    return np.ones_like(fl.rho), fl.u


@pytest.mark.parametrize("n", [8, 16, 20])
def test_taylor_green_closed_form(oracle_mod, n):
    v0 = 0.37
    rho, u = _tgv_unit_density(n, v0, phase=(0.3, -0.7, 1.1))
    ke, eps = oracle_mod.diagnostics((n, n, n), rho, u)
    k = 2 * np.pi / n
    assert abs(ke - v0 ** 2 / 8) < 1e-14 * v0 ** 2
    assert abs(eps - 3.0 / 8.0 * v0 ** 2 * np.sin(k) ** 2) < 1e-14 * v0 ** 2


def test_shear_waves_along_each_axis(oracle_mod):
    # u_a = A sin(k x_b) for every ordered pair a != b: KE = A^2 / 4,
    # eps = A^2 sin^2(k) / 4 (one curl component, mean cos^2 = 1/2)
    n, amp = 12, 0.2
    shape = (n, n, n)
    pos = wl.positions(shape)
    k = 2 * np.pi / n
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            u = np.zeros((3, pos[0].size))
            u[a] = amp * np.sin(k * pos[b] + 0.4)
            ke, eps = oracle_mod.diagnostics(shape, np.ones(pos[0].size), u)
            assert abs(ke - amp ** 2 / 4) < 1e-15, (a, b)
            assert abs(eps - amp ** 2 * np.sin(k) ** 2 / 4) < 1e-15, (a, b)


def test_uniform_flow_has_no_enstrophy_and_density_weights(oracle_mod):
    shape = (6, 5, 7)
    ns = 2 * 6 * 5 * 7
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.5, 1.5, ns)
    u = np.tile(np.array([0.1, -0.2, 0.3])[:, None], (1, ns))
    ke, eps = oracle_mod.diagnostics(shape, rho, u)
    assert eps == 0.0
    assert abs(ke - 0.5 * rho.mean() * 0.14) < 1e-15


def test_mixed_field_is_not_a_sum_of_axis_terms(oracle_mod):
    # a rotation-like periodic field: u = (sin y, sin z, sin x) (k = 2 pi/N)
    # has w = -(cos z, cos x, cos y) sin(k): eps = 3 sin^2(k) / 4 * A^2 / 2
    n, amp = 10, 0.3
    shape = (n, n, n)
    x, y, z = wl.positions(shape)
    k = 2 * np.pi / n
    u = amp * np.array([np.sin(k * y), np.sin(k * z), np.sin(k * x)])
    ke, eps = oracle_mod.diagnostics(shape, np.ones(x.size), u)
    assert abs(ke - 3 * amp ** 2 / 4) < 1e-15
    assert abs(eps - 3 * amp ** 2 * np.sin(k) ** 2 / 4) < 1e-15
