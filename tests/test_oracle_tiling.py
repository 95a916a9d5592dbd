"""Pins of the oracle's large-sample forms (Sec. 1 patch composition, Sec. 4.6
periodic display): the tiled field against the literal sum of Eq. 10 at
points in later periods; composition of identical patches against tiling;
a uniform sample composed of patches against the closed-form plane wave."""
import numpy as np

import workloads as W
from oracle import cwt


def _prob(seed, n_in=1.45 + 0.02j):
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((2, 6, 7)) + 0.03j * rng.random((2, 6, 7))
    n[:, 2:4, 2:5] = n_in
    return W.Problem(n=n.astype(complex), px=0.3, py=0.32, pz=0.21, lam=1.0, U=5, V=3,
                     n_top=1.0, n_bot=1.3 + 0.0j, plane_wave=W.PlaneWave(1, 0, 0.9, 0.2j))


def test_tiled_field_is_eq10_at_later_periods():
    prob = _prob(1)
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    grid = W.Grid(fx=7, fy=6, fz=4, z_begin=-0.2, z_end=prob.thickness + 0.3)
    E = cwt.tiled(st, sol, grid, 3, 2)
    assert E.shape == (3, 4, 12, 21)
    rng = np.random.default_rng(4)
    zs = grid.z_planes()
    for _ in range(12):
        f, g, j = rng.integers(21), rng.integers(12), rng.integers(4)
        x = f * prob.X / grid.fx   # absolute position, beyond the first period for f >= fx
        y = g * prob.Y / grid.fy
        want = cwt.field_at_points(st, sol, [x], [y], [zs[j]])[:, 0]
        assert np.abs(E[:, j, g, f] - want).max() <= 1e-12 * np.abs(want).max()


def test_identical_patches_compose_to_the_periodic_field():
    prob = _prob(2)
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    grid = W.Grid(fx=7, fy=6, fz=3, z_begin=0.0, z_end=prob.thickness)
    comp = cwt.compose([(st, sol)] * 6, 3, 2, grid)
    assert np.array_equal(comp, cwt.tiled(st, sol, grid, 3, 2))


def test_uniform_patches_give_the_plane_wave():
    """Every patch uniform (n = n_top = n_bot): the composed field is the
    incident plane wave exp(i k (s_x x + s_z z)) over the whole mosaic."""
    n0 = 1.0
    probs = []
    for pxv in (0.3, 0.3):
        probs.append(W.Problem(n=np.full((2, 5, 5), n0, dtype=complex), px=pxv, py=0.3,
                               pz=0.2, lam=1.0, U=3, V=3, n_top=n0, n_bot=n0 + 0.0j,
                               plane_wave=W.PlaneWave(1, 0, 1.0, 0.0)))
    parts = []
    for pr in probs * 2:
        st = cwt.setup(pr)
        parts.append((st, cwt.solve(st)))
    grid = W.Grid(fx=5, fy=5, fz=3, z_begin=-0.1, z_end=0.5)
    E = cwt.compose(parts, 2, 2, grid)
    X = 5 * 0.3
    sx = 1.0 / X
    sz = np.sqrt(1 - sx * sx)
    k = 2 * np.pi
    x = np.arange(10) * X / 5
    z = np.array(grid.z_planes())
    want = np.exp(1j * k * (sx * x[None, None, :] + sz * z[:, None, None]))
    want = np.broadcast_to(want, (3, 10, 10))  # [fz, y, x]
    # E_x carries the unit amplitude; E_z = -(s_x / s_z) E_x by transversality
    assert np.abs(E[0] - want).max() <= 1e-12
    assert np.abs(E[2] + sx / sz * want).max() <= 1e-12
    assert np.abs(E[1]).max() <= 1e-12
