"""The library's in-place (AA) streaming scheme, checked on the CPU from its
own direction table (lbm_velocities, a host-only call of the C ABI):

  even step: the thread of site s reads slot i at s and writes slot opp(i)
             at s;
  odd step:  it reads slot opp(i) at s - c_i and writes slot i at s + c_i,
             where a half-integer c_i moves between the cube corners and
             the cube centres (Sec. I replica grid).

Race freedom: in each step every thread writes exactly the 81 addresses it
read, and no two threads write the same address, so a launch needs no
synchronisation beyond the kernel boundary.  Semantics: an even step and an
odd step with the collision left out move the populations exactly as two
streaming steps of the oracle.  The GPU kernels' own address arithmetic is
checked bit for bit against the oracle by the GPU parity tests; this test
pins the scheme they implement, on grids down to 1x1x1 where every link
wraps onto the site itself."""
import numpy as np
import pytest

import oracle
from parity import lib_to_oracle_perm

SHAPES = [(1, 1, 1), (2, 3, 1), (5, 4, 3), (3, 2, 5), (8, 8, 2)]


def _lattice():
    from paper_2409_05114_amd import lbm81
    c, _ = lbm81.lbm_velocities()
    c2 = np.rint(2 * c).astype(int)
    opp = np.array([next(j for j in range(len(c2)) if (c2[j] == -c2[i]).all())
                    for i in range(len(c2))])
    return c2, opp


def _sites(shape):
    """(sub, x, y, z) of every site in the site order [sub][z][y][x]."""
    nx, ny, nz = shape
    sub, z, y, x = np.meshgrid(np.arange(2), np.arange(nz), np.arange(ny),
                               np.arange(nx), indexing="ij")
    return sub.ravel(), x.ravel(), y.ravel(), z.ravel()


def _shift(shape, c2):
    """Index of the site reached from every site by the doubled velocity c2
    (positions doubled: 2 x + sub on each axis, periodic)."""
    nx, ny, nz = shape
    sub, x, y, z = _sites(shape)
    p = [2 * x + sub + c2[0], 2 * y + sub + c2[1], 2 * z + sub + c2[2]]
    nsub = p[0] % 2
    assert all(((q % 2) == nsub).all() for q in p)
    xn = ((p[0] - nsub) // 2) % nx
    yn = ((p[1] - nsub) // 2) % ny
    zn = ((p[2] - nsub) // 2) % nz
    return ((nsub * nz + zn) * ny + yn) * nx + xn


def _odd_maps(shape, c2, opp):
    q = len(c2)
    fwd = np.stack([_shift(shape, c2[i]) for i in range(q)], axis=1)
    back = np.stack([_shift(shape, -c2[i]) for i in range(q)], axis=1)
    slots = np.arange(q)
    reads = back * q + opp[slots][None, :]  # slot opp(i) at s - c_i
    writes = fwd * q + slots[None, :]  # slot i at s + c_i
    return reads, writes


@pytest.mark.parametrize("shape", SHAPES)
def test_odd_step_writes_what_it_read_and_nothing_twice(shape):
    c2, opp = _lattice()
    assert (opp[opp] == np.arange(len(c2))).all()
    reads, writes = _odd_maps(shape, c2, opp)
    ns = 2 * shape[0] * shape[1] * shape[2]
    # per thread: the same 81 addresses read and written
    assert (np.sort(reads, axis=1) == np.sort(writes, axis=1)).all()
    # across threads: every address written exactly once
    assert np.array_equal(np.sort(writes.ravel()), np.arange(ns * len(c2)))


@pytest.mark.parametrize("shape", SHAPES)
def test_even_then_odd_step_streams_like_the_oracle(shape):
    c2, opp = _lattice()
    q = len(c2)
    ns = 2 * shape[0] * shape[1] * shape[2]
    rng = np.random.default_rng(7)
    p = rng.uniform(0.5, 1.5, (ns, q))  # slot i at s holds f_i(s)
    # even step, collision left out: f_i(s) goes to slot opp(i) at s
    buf = np.empty_like(p)
    buf[:, opp] = p
    # odd step: read slot opp(i) at s - c_i, write slot i at s + c_i
    reads, writes = _odd_maps(shape, c2, opp)
    vals = buf.ravel()[reads]
    out = np.empty(ns * q)
    out[writes.ravel()] = vals.ravel()
    out = out.reshape(ns, q)
    # the oracle: two push-streaming steps, in its own direction order
    perm = lib_to_oracle_perm()
    fo = np.empty((ns, q))
    fo[:, perm] = p
    oracle.step(shape, fo, 0.8, 2, mode="stream")
    assert np.array_equal(out, fo[:, perm])
