"""Helpers shared by the GPU parity tests: run the same seeded fields
through the HIP library (via its C ABI binding) and through the CPU oracle,
and compare.

Error metric (per field, over all compared sites): max |a - b| / max |b| for
rho and theta, and max |u_a - u_b| / max |u_b| with |.| the Euclidean norm of
the velocity vector (u crosses zero, so a pointwise relative error is
meaningless).
"""
import numpy as np

import oracle


def lib_to_oracle_perm():
    """perm[i] = oracle direction index of library direction i."""
    from paper_2409_05114_amd import lbm81
    c, _ = lbm81.lbm_velocities()
    co, _, _ = oracle.lattice()
    where = {tuple((2 * v).astype(int)): j for j, v in enumerate(co)}
    return np.array([where[tuple((2 * v).astype(int))] for v in c])


def field_errors(a, b):
    """a, b = (rho, u[3, n], theta) numpy arrays; returns dict of errors."""
    ra, ua, ta = a
    rb, ub, tb = b
    du = np.sqrt(((ua - ub) ** 2).sum(0))
    nu = np.sqrt((ub ** 2).sum(0))
    umax = nu.max()
    return {
        "rho": float(np.abs(ra - rb).max() / np.abs(rb).max()),
        "u": float(du.max() / umax) if umax > 0 else float(du.max()),
        "theta": float(np.abs(ta - tb).max() / np.abs(tb).max()),
    }


def population_error(f_gpu_lib_order, f_oracle):
    """f_gpu [81, n] (library order), f_oracle [n, 81] -> max rel error."""
    perm = lib_to_oracle_perm()
    fo = f_oracle[:, perm].T  # [81, n] in library order
    return float(np.abs(f_gpu_lib_order - fo).max() / np.abs(fo).max())


def gpu_run(fields, nsteps, tau, storage="f64", populations=False):
    from paper_2409_05114_amd import lbm81
    sim = lbm81.Sim(fields.shape, storage)
    sim.init(fields.rho, fields.u, fields.theta)
    if nsteps:
        sim.step(nsteps, tau)
    rho, u, th = sim.moments()
    out = (rho.cpu().numpy(), u.cpu().numpy(), th.cpu().numpy())
    pops = sim.populations_f64().cpu().numpy() if populations else None
    tot, flags = sim.totals(check=False)
    sim.close()
    return out, pops, tot, flags


def oracle_run(fields, nsteps, tau, shape=None, entropic=False, series=False):
    shape = shape or fields.shape
    (rho, u, th), f = oracle.run(shape, fields.rho, fields.u, fields.theta,
                                 tau, nsteps, entropic=entropic, series=series)
    return (rho, u, th), f


def window(fields_full, shape, centre, radius):
    """Fields of a periodic window of (2 radius + 1)^3 cells around cell
    `centre` of the full periodic grid, in the window's own site order."""
    nx, ny, nz = shape
    w = 2 * radius + 1
    cx, cy, cz = centre
    xs = (np.arange(w) + cx - radius) % nx
    ys = (np.arange(w) + cy - radius) % ny
    zs = (np.arange(w) + cz - radius) % nz
    sub = np.arange(2).reshape(2, 1, 1, 1)
    z = zs.reshape(1, w, 1, 1)
    y = ys.reshape(1, 1, w, 1)
    x = xs.reshape(1, 1, 1, w)
    idx = (((sub * nz + z) * ny + y) * nx + x).reshape(-1)
    from paper_2409_05114_amd.workloads import Fields
    return Fields((w, w, w), fields_full.rho[idx],
                  np.ascontiguousarray(fields_full.u[:, idx]),
                  fields_full.theta[idx]), idx


def window_centre_sites(radius):
    """Site indices (window order) of the two sites of the centre cell."""
    w = 2 * radius + 1
    c = ((radius * w) + radius) * w + radius
    return np.array([c, w ** 3 + c])
