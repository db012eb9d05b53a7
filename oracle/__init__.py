"""FP64 CPU oracle for the RD3Q81 lattice Boltzmann update (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark -- never by the GPU library or its Python
binding.  The C source (lbm81_oracle.c) is an independent, plain restatement of
the method of Atif et al., arXiv:2409.05114 (lattice: Table "tab:weights";
moments: Eq. conslaws; equilibrium: Sec. III; update: Eq. discretelbm).

Arrays use the site order ((sub * nz + z) * ny + y) * nx + x, sub 0 = cube
corners, sub 1 = cube centres; u is [3][site]; populations are [site][81] in
the oracle's own velocity order (see ``lattice()``).
"""
import ctypes
import os

import numpy as np

from . import build as _build

Q = 81
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        lib.lbo_lattice.argtypes = [dp, dp, dp]
        lib.lbo_equilibrium.argtypes = [ctypes.c_double] * 5 + [dp, dp]
        lib.lbo_init.argtypes = [i, i, i, dp, dp, dp, dp]
        lib.lbo_step.argtypes = [i, i, i, ctypes.c_double, i, i, dp, dp]
        lib.lbo_step_entropic.argtypes = [i, i, i, ctypes.c_double, i, i, dp, dp]
        lib.lbo_step_series.argtypes = [i, i, i, ctypes.c_double, i, i, dp, dp]
        lib.lbo_series_equilibrium.argtypes = [ctypes.c_double] * 5 + [dp]
        lib.lbo_series_fallbacks.argtypes = [i, i, i, dp]
        lib.lbo_series_fallbacks.restype = ctypes.c_longlong
        lib.lbo_entropic_alpha.argtypes = [dp, dp, dp]
        lib.lbo_entropy.argtypes = [dp]
        lib.lbo_entropy.restype = ctypes.c_double
        lib.lbo_moments.argtypes = [i, i, i, dp, dp, dp, dp]
        lib.lbo_totals.argtypes = [i, i, i, dp, dp]
        lib.lbo_diagnostics.argtypes = [i, i, i, dp, dp, dp]
        lib.lbo_stream_target.argtypes = [i, i, i, ctypes.c_longlong, i]
        lib.lbo_stream_target.restype = ctypes.c_longlong
        lib.lbo_set_threads.argtypes = [i]
        lib.lbo_get_threads.restype = i
        _lib = lib
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc < 0:
        raise OracleError(f"{what}: oracle returned {rc}")
    return rc


def set_threads(n: int) -> None:
    _load().lbo_set_threads(int(n))


def get_threads() -> int:
    return int(_load().lbo_get_threads())


def lattice():
    """(c[81,3], w[81], theta0) of the oracle's lattice."""
    c = np.zeros((Q, 3))
    w = np.zeros(Q)
    t = np.zeros(1)
    _check(_load().lbo_lattice(_p(c), _p(w), _p(t)), "lattice")
    return c, w, float(t[0])


def equilibrium(rho, u, theta, return_multipliers=False):
    """Entropic equilibrium f_eq[81] at one point; optionally the multipliers
    (mu, zeta_x, zeta_y, zeta_z, gamma) per unit density and the Newton
    iteration count."""
    f = np.zeros(Q)
    lam = np.zeros(5)
    it = _check(_load().lbo_equilibrium(float(rho), float(u[0]), float(u[1]),
                                         float(u[2]), float(theta), _p(f),
                                         _p(lam)), "equilibrium")
    if return_multipliers:
        return f, lam, it
    return f


def n_sites(shape):
    nx, ny, nz = shape
    return 2 * nx * ny * nz


def init(shape, rho, u, theta):
    """Populations [sites, 81] set to f_eq of the given fields."""
    nx, ny, nz = shape
    ns = n_sites(shape)
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(ns)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, ns)
    theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(ns)
    f = np.zeros((ns, Q))
    _check(_load().lbo_init(nx, ny, nz, _p(rho), _p(u), _p(theta), _p(f)),
           "init")
    return f


def step(shape, f, tau, nsteps, mode="full", entropic=False, series=False):
    """Advance populations in place. mode: 'full', 'stream' or 'collide';
    entropic: alpha from the entropy condition (Eq. delH) instead of 2;
    series: the series equilibrium (Appendix B) at sites where it is
    positive, the Newton solution elsewhere."""
    nx, ny, nz = shape
    m = {"full": 0, "stream": 1, "collide": 2}[mode]
    scratch = np.empty_like(f)
    assert not (entropic and series)
    fn = (_load().lbo_step_entropic if entropic else
          _load().lbo_step_series if series else _load().lbo_step)
    _check(fn(nx, ny, nz, float(tau), int(nsteps), m, _p(f), _p(scratch)),
           "step")
    return f


def series_equilibrium(rho, u, theta):
    """(f~[81], positive) of one point: the series form of the equilibrium
    (Sec. III; Appendix B, Eq. zeroveleqseries and the third-order term),
    and whether all 81 values are positive."""
    f = np.zeros(Q)
    r = _check(_load().lbo_series_equilibrium(float(rho), float(u[0]),
                                               float(u[1]), float(u[2]),
                                               float(theta), _p(f)),
               "series_equilibrium")
    return f, bool(r)


def series_fallbacks(shape, f):
    """Sites of f where a series step falls back to the Newton solution."""
    nx, ny, nz = shape
    f = np.ascontiguousarray(f, dtype=np.float64)
    return int(_check(_load().lbo_series_fallbacks(nx, ny, nz, _p(f)),
                      "series_fallbacks"))


def entropic_alpha(f, feq):
    """(alpha, iterations) of one site: the positive root of
    H[f + alpha (feq - f)] = H[f] (Eq. delH), capped by positivity."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    feq = np.ascontiguousarray(feq, dtype=np.float64)
    a = np.zeros(1)
    it = _check(_load().lbo_entropic_alpha(_p(f), _p(feq), _p(a)),
                "entropic_alpha")
    return float(a[0]), it


def entropy(f):
    """H[f] = sum f (ln(f / w) - 1) of one site's 81 populations."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    return float(_load().lbo_entropy(_p(f)))


def moments(shape, f):
    """(rho[sites], u[3, sites], theta[sites])."""
    nx, ny, nz = shape
    ns = n_sites(shape)
    rho = np.zeros(ns)
    u = np.zeros((3, ns))
    th = np.zeros(ns)
    _check(_load().lbo_moments(nx, ny, nz, _p(f), _p(rho), _p(u), _p(th)),
           "moments")
    return rho, u, th


def totals(shape, f):
    """[sum rho, sum rho u_x, sum rho u_y, sum rho u_z, sum energy moment]."""
    nx, ny, nz = shape
    out = np.zeros(5)
    _check(_load().lbo_totals(nx, ny, nz, _p(f), _p(out)), "totals")
    return out


def diagnostics(shape, rho, u):
    """(mean kinetic energy, mean enstrophy) of the fields rho[sites],
    u[3, sites] (Sec. IV.C; curl by central differences on each
    sub-lattice, see lbo_diagnostics)."""
    nx, ny, nz = shape
    out = np.zeros(2)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    _check(_load().lbo_diagnostics(nx, ny, nz, _p(rho), _p(u), _p(out)),
           "diagnostics")
    return float(out[0]), float(out[1])


def stream_target(shape, site, i):
    nx, ny, nz = shape
    return int(_load().lbo_stream_target(nx, ny, nz, int(site), int(i)))


def run(shape, rho, u, theta, tau, nsteps, entropic=False, series=False):
    """init + nsteps full updates; returns (rho, u, theta) and populations."""
    f = init(shape, rho, u, theta)
    if nsteps:
        step(shape, f, tau, nsteps, entropic=entropic, series=series)
    return moments(shape, f), f
