"""Seeded synthetic initial fields (rho, u, theta) for the RD3Q81 workloads.

This module holds input recipes only -- no part of the lattice Boltzmann method
(no lattice, equilibrium, collision or streaming).  Both the GPU library and
the CPU oracle are fed the arrays it returns, so the two sides see bit-identical
inputs.

Conventions shared with both sides (interface, not arithmetic):
  * lattice units, dx = dt = 1;
  * theta0 is the base temperature printed with the RD3Q81 weight table
    (Table "tab:weights");
  * sound speed c_s = sqrt(gamma theta0) with gamma = 5/3 (Sec. IV.C,
    Taylor-Green vortex), so Ma = |u| / c_s;
  * a grid of nx x ny x nz cubic cells holds 2 nx ny nz sites: cube corners
    (sub 0) at (x, y, z) and cube centres (sub 1) at (x+1/2, y+1/2, z+1/2);
  * field arrays are float64, site order ((sub * nz + z) * ny + y) * nx + x,
    rho and theta shaped [sites], u shaped [3, sites].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

THETA0 = 0.821035006329447750282591763
GAMMA = 5.0 / 3.0
C_S = math.sqrt(GAMMA * THETA0)


@dataclass
class Fields:
    shape: tuple  # (nx, ny, nz) cells
    rho: np.ndarray
    u: np.ndarray
    theta: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_sites(self) -> int:
        nx, ny, nz = self.shape
        return 2 * nx * ny * nz


def positions(shape, dtype=np.float64):
    """Physical coordinates (x, y, z) of every site, each shaped [sites]."""
    nx, ny, nz = shape
    sub = np.arange(2, dtype=dtype).reshape(2, 1, 1, 1) * 0.5
    z = np.arange(nz, dtype=dtype).reshape(1, nz, 1, 1) + sub
    y = np.arange(ny, dtype=dtype).reshape(1, 1, ny, 1) + sub
    x = np.arange(nx, dtype=dtype).reshape(1, 1, 1, nx) + sub
    full = (2, nz, ny, nx)
    return (np.broadcast_to(x, full).reshape(-1),
            np.broadcast_to(y, full).reshape(-1),
            np.broadcast_to(z, full).reshape(-1))


def _pack(shape, rho, ux, uy, uz, theta, **meta):
    ns = 2 * shape[0] * shape[1] * shape[2]
    u = np.empty((3, ns))
    u[0] = ux
    u[1] = uy
    u[2] = uz
    return Fields(tuple(shape), np.ascontiguousarray(rho, dtype=np.float64),
                  u, np.ascontiguousarray(theta, dtype=np.float64), meta)


def uniform(shape, rho=1.0, u=(0.0, 0.0, 0.0), theta=THETA0):
    ns = 2 * shape[0] * shape[1] * shape[2]
    return _pack(shape, np.full(ns, rho), u[0], u[1], u[2],
                 np.full(ns, theta), kind="uniform")


def shear_wave(shape=(32, 32, 32), amp_ma=0.1, noise=1e-4, seed=0,
               phase=0.0):
    """Transverse shear wave u_x = amp_ma c_s sin(2 pi y / ny + phase),
    rho = 1 + noise U(-1, 1) (seeded), theta = theta0.  The noise is drawn in
    site order."""
    x, y, z = positions(shape)
    ns = x.size
    rng = np.random.default_rng(seed)
    rho = 1.0 + noise * rng.uniform(-1.0, 1.0, ns) if noise else np.ones(ns)
    ux = amp_ma * C_S * np.sin(2.0 * np.pi * y / shape[1] + phase)
    return _pack(shape, rho, ux, 0.0, 0.0, np.full(ns, THETA0),
                 kind="shear_wave", amp=amp_ma * C_S, k=2 * np.pi / shape[1])


def sound_wave(shape=(64, 1, 1), amp=1e-4):
    """Standing isentropic acoustic wave of a monatomic gas:
    rho = 1 + amp s, theta = theta0 (1 + (gamma - 1) amp s), u = 0, with
    s = sin(2 pi x / nx)."""
    x, y, z = positions(shape)
    s = np.sin(2.0 * np.pi * x / shape[0])
    return _pack(shape, 1.0 + amp * s, 0.0, 0.0, 0.0,
                 THETA0 * (1.0 + (GAMMA - 1.0) * amp * s),
                 kind="sound_wave", amp=amp, k=2 * np.pi / shape[0])


def double_riemann(shape=(2048, 4, 4), rho_l=1.0, theta_l=THETA0,
                   rho_r=0.125, theta_r=0.8 * THETA0):
    """Periodic double Riemann problem along x: sites with x-position < nx/2
    hold the left state, the rest the right state; u = 0.  With periodic
    wrap there are two interfaces, at nx/2 and at 0."""
    x, y, z = positions(shape)
    left = x < shape[0] / 2.0
    rho = np.where(left, rho_l, rho_r)
    theta = np.where(left, theta_l, theta_r)
    return _pack(shape, rho, 0.0, 0.0, 0.0, theta, kind="double_riemann")


# Smallest initial density of a served vortex, as a fraction of rho0.
SERVE_TGV_RHO_MIN = 0.25


def serve_tgv_p0(ma, rho0=1.0):
    """Background pressure p0 of a served Taylor-Green vortex.  Sec. IV.C
    leaves p0 open.  Its pressure field p0 + rho0 V0^2 / 16 (cos 2x^ +
    cos 2y^)(cos 2z^ + 2) falls to p0 - (3/8) rho0 V0^2, so p0 = rho0 theta0
    (the benchmark's reading) leaves a negative density beyond Ma 1.26.  The
    served vortices take p0 = rho0 theta0 while that keeps the density at or
    above SERVE_TGV_RHO_MIN rho0 (Ma up to 1.095), and above that the p0 that
    keeps it exactly there: p0 = (3/8) rho0 V0^2 + SERVE_TGV_RHO_MIN rho0
    theta0 (continuous in Ma; 2.75 rho0 theta0 at Ma 2)."""
    v0 = ma * C_S
    return max(rho0 * THETA0,
               0.375 * rho0 * v0 * v0 + SERVE_TGV_RHO_MIN * rho0 * THETA0)


def taylor_green(shape=(256, 256, 256), ma=1.2, rho0=1.0, phase=(0.0, 0.0, 0.0),
                 p0=None):
    """Compressible Taylor-Green vortex of Sec. IV.C on a periodic box:
    u1 = V0 sin x^ cos y^ cos z^, u2 = -V0 cos x^ sin y^ cos z^, u3 = 0,
    p = p0 + rho0 V0^2 / 16 (cos 2x^ + cos 2y^)(cos 2z^ + 2), with
    x^ = x / L, L = n / (2 pi) so the box is one period; V0 = Ma c_s;
    theta = theta0 uniform and rho = p / theta0 with p0 = rho0 theta0 unless
    given (serve_tgv_p0 for the served vortices)."""
    nx, ny, nz = shape
    x, y, z = positions(shape)
    v0 = ma * C_S
    xh = 2.0 * np.pi * x / nx + phase[0]
    yh = 2.0 * np.pi * y / ny + phase[1]
    zh = 2.0 * np.pi * z / nz + phase[2]
    ux = v0 * np.sin(xh) * np.cos(yh) * np.cos(zh)
    uy = -v0 * np.cos(xh) * np.sin(yh) * np.cos(zh)
    p0 = rho0 * THETA0 if p0 is None else p0
    p = p0 + rho0 * v0 * v0 / 16.0 * (np.cos(2 * xh) + np.cos(2 * yh)) * \
        (np.cos(2 * zh) + 2.0)
    return _pack(shape, p / THETA0, ux, uy, 0.0, np.full(x.size, THETA0),
                 kind="taylor_green", ma=ma, v0=v0, p0=p0)


def shear_layer(shape=(512, 512, 256), ma=2.0, delta=8.0, pert=1e-3, seed=0):
    """Periodic double shear layer: u_x = U [tanh((y - ny/4)/delta) -
    tanh((y - 3 ny/4)/delta) - 1] with U = Ma c_s, so the two streams move at
    +-U; rho = 1, theta = theta0; seeded perturbations pert c_s U(-1, 1) added
    to all three velocity components (drawn component by component in site
    order)."""
    nx, ny, nz = shape
    x, y, z = positions(shape)
    ns = x.size
    U = ma * C_S
    ux = U * (np.tanh((y - ny / 4.0) / delta) -
              np.tanh((y - 3.0 * ny / 4.0) / delta) - 1.0)
    rng = np.random.default_rng(seed)
    amp = pert * C_S
    ux = ux + amp * rng.uniform(-1.0, 1.0, ns)
    uy = amp * rng.uniform(-1.0, 1.0, ns)
    uz = amp * rng.uniform(-1.0, 1.0, ns)
    return _pack(shape, np.ones(ns), ux, uy, uz, np.full(ns, THETA0),
                 kind="shear_layer", ma=ma)


def random_state(shape, seed=0, ma_max=1.0, rho_range=(0.5, 1.5),
                 theta_range=(0.7, 1.4)):
    """Independent random (rho, u, theta) per site: a stress test with no
    smoothness.  |u| <= ma_max c_s; theta in theta_range x theta0."""
    ns = 2 * shape[0] * shape[1] * shape[2]
    rng = np.random.default_rng(seed)
    rho = rng.uniform(*rho_range, ns)
    d = rng.normal(size=(3, ns))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    u = d * rng.uniform(0.0, ma_max * C_S, ns)
    theta = THETA0 * rng.uniform(*theta_range, ns)
    return _pack(shape, rho, u[0], u[1], u[2], theta, kind="random")


# ------------------------------------------------------------ serving traffic

SERVE_SIDES = (48, 64, 96, 128, 192, 256)


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the stream
    side: int
    ma: float
    tau: float
    steps: int
    kind: str  # "shear" or "tgv"
    phase: tuple
    storage: str

    def fields(self) -> Fields:
        n = self.side
        if self.kind == "shear":
            return shear_wave((n, n, n), amp_ma=self.ma, noise=0.0,
                              phase=self.phase[0])
        return taylor_green((n, n, n), ma=self.ma, phase=self.phase,
                            p0=serve_tgv_p0(self.ma))

    def fields_on_device(self, device):
        """The same initial fields generated directly in device memory
        (torch, FP64): (rho[S], u[3, S], theta[S])."""
        return device_fields(self.kind, self.side, self.ma, self.phase, device)

    @property
    def sites(self) -> int:
        return 2 * self.side ** 3


def device_fields(kind, n, ma, phase, device):
    """Shear-wave or Taylor-Green initial fields of an n^3 box built with
    torch on `device` (FP64), same formulas as Request.fields (the vortex
    with the served background pressure serve_tgv_p0)."""
    import torch

    t = torch.float64
    sub = torch.arange(2, dtype=t, device=device).view(2, 1, 1, 1) * 0.5
    ar = torch.arange(n, dtype=t, device=device)
    z = (ar.view(1, n, 1, 1) + sub).expand(2, n, n, n).reshape(-1)
    y = (ar.view(1, 1, n, 1) + sub).expand(2, n, n, n).reshape(-1)
    x = (ar.view(1, 1, 1, n) + sub).expand(2, n, n, n).reshape(-1)
    S = x.numel()
    u = torch.zeros((3, S), dtype=t, device=device)
    theta = torch.full((S,), THETA0, dtype=t, device=device)
    if kind == "shear":
        rho = torch.ones(S, dtype=t, device=device)
        u[0] = ma * C_S * torch.sin(2.0 * math.pi * y / n + phase[0])
        return rho, u, theta
    v0 = ma * C_S
    xh = 2.0 * math.pi * x / n + phase[0]
    yh = 2.0 * math.pi * y / n + phase[1]
    zh = 2.0 * math.pi * z / n + phase[2]
    u[0] = v0 * torch.sin(xh) * torch.cos(yh) * torch.cos(zh)
    u[1] = -v0 * torch.cos(xh) * torch.sin(yh) * torch.cos(zh)
    p = serve_tgv_p0(ma) + v0 * v0 / 16.0 * \
        (torch.cos(2 * xh) + torch.cos(2 * yh)) * (torch.cos(2 * zh) + 2.0)
    return p / THETA0, u, theta


def request_stream(rate=20.0, duration=60.0, seed=0, sides=SERVE_SIDES,
                   ma_range=(0.3, 2.0), tau_range=(0.51, 0.9),
                   steps_range=(200, 2000), storage="f32"):
    """Poisson arrivals of independent periodic-box simulations: side drawn
    uniformly from ``sides``, Ma ~ U(ma_range), tau ~ U(tau_range), steps
    uniform on the integer range, half shear waves with a random phase and
    half Taylor-Green vortices with random phase shifts."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        kind = "shear" if rng.uniform() < 0.5 else "tgv"
        out.append(Request(
            rid=len(out), arrival=t, side=int(rng.choice(sides)),
            ma=float(rng.uniform(*ma_range)), tau=float(rng.uniform(*tau_range)),
            steps=int(rng.integers(steps_range[0], steps_range[1] + 1)),
            kind=kind, phase=tuple(float(p) for p in rng.uniform(0, 2 * np.pi, 3)),
            storage=storage))
    return out
