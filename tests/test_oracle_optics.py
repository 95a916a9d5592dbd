"""Pins of the oracle's objective image (cwt.objective_pass, cwt.image):
closed forms of an ideal objective's coherent transfer function acting on the
plane-wave spectrum (Sec. 1), independent of the HIP library."""
import numpy as np

import workloads as W
from oracle import cwt


def _lossy_problem(seed=6, U=5, V=3):
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((3, 6, 8)) + 0.04j * rng.random((3, 6, 8))
    return W.Problem(n=n.astype(complex), px=0.31, py=0.27, pz=0.19, lam=1.0, U=U, V=V,
                     n_top=1.0, n_bot=1.45 + 0.01j,
                     plane_wave=W.PlaneWave(1, -1, 0.8, 0.3 - 0.2j))


def _grid(prob):
    return W.Grid(fx=9, fy=7, fz=7, z_begin=-0.3, z_end=prob.thickness + 0.3)


def test_wide_objective_passes_the_whole_field():
    prob = _lossy_problem()
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    grid = _grid(prob)
    na = 1.01 * np.sqrt(np.max(st.sx ** 2 + st.sy ** 2))
    E, I = cwt.image(st, sol, grid, na)
    np.testing.assert_array_equal(E, cwt.synthesize(st, sol, grid))
    assert np.all(I > 0)


def test_narrow_objective_keeps_only_the_axial_wave():
    # below the smallest nonzero direction sine only the (0, 0) mode passes:
    # the image of every plane is then uniform, p(m0, z), with intensity
    # |p_x|^2 + |p_y|^2 + |p_z|^2 of that mode
    prob = _lossy_problem()
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    grid = _grid(prob)
    r = np.sqrt(st.sx ** 2 + st.sy ** 2)
    E, I = cwt.image(st, sol, grid, 0.5 * np.min(r[r > 0]))
    m0 = (st.V // 2) * st.U + st.U // 2
    assert r[m0] == 0.0
    for j, z in enumerate(grid.z_planes()):
        p0 = cwt.plane_coefficients(st, sol, z)[:, m0]
        for c in range(3):
            np.testing.assert_allclose(E[c, j], np.full((grid.fy, grid.fx), p0[c]),
                                       rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(I[j], np.sum(np.abs(p0) ** 2), rtol=1e-12)


def test_objective_on_a_plane_wave_in_a_uniform_medium():
    # a tilted plane wave through a uniform medium: an objective wider than
    # its direction sine images it unchanged, with the uniform intensity
    # |E_x|^2 + |E_y|^2 + |E_z|^2 of a transverse plane wave; a narrower one
    # passes nothing
    X, ns, lam = 2.5, 1.4, 1.0
    n = np.full((2, 6, 6), complex(ns))
    prob = W.Problem(n=n, px=X / 6, py=X / 6, pz=0.3, lam=lam, U=5, V=5, n_top=ns, n_bot=ns,
                     plane_wave=W.PlaneWave(1, 0, 0.0, 1.0))
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    grid = W.Grid(fx=8, fy=6, fz=5, z_begin=-0.2, z_end=0.8)
    sx = lam / X
    sz = np.sqrt(ns ** 2 - sx ** 2)
    E, I = cwt.image(st, sol, grid, 1.05 * sx)
    pw = np.array([0.0, 1.0, 0.0])  # E_y polarisation: transverse to s = (sx, 0, sz)
    xs = np.arange(grid.fx) * X / grid.fx
    for j, z in enumerate(grid.z_planes()):
        want = pw[:, None, None] * np.exp(1j * 2 * np.pi / lam * (sx * xs[None, :] + sz * z))
        want = np.broadcast_to(want, (3, grid.fy, grid.fx))
        np.testing.assert_allclose(E[:, j], want, atol=1e-12)
    np.testing.assert_allclose(I, 1.0, rtol=1e-12)
    E0, I0 = cwt.image(st, sol, grid, 0.95 * sx)
    assert np.abs(E0).max() < 1e-14 and np.abs(I0).max() < 1e-28


def test_transfer_function_of_ones_and_of_the_objective():
    prob = _lossy_problem(seed=7)
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    grid = _grid(prob)
    E1, _ = cwt.filtered(st, sol, grid, np.ones(st.M))
    np.testing.assert_array_equal(E1, cwt.synthesize(st, sol, grid))
    Eo, Io = cwt.filtered(st, sol, grid, cwt.objective_pass(st, 0.7))
    Ei, Ii = cwt.image(st, sol, grid, 0.7)
    np.testing.assert_array_equal(Eo, Ei)
    np.testing.assert_array_equal(Io, Ii)


def test_propagation_transfer_function_moves_the_transmitted_field():
    # below the sample every mode is a plane wave exp(i k s_z (z - zL)) of the
    # bottom medium: the transfer function exp(i k s_z dz) applied at z must
    # give the field at z + dz
    prob = _lossy_problem(seed=8)
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    T = prob.thickness
    dz = 0.23
    near = W.Grid(fx=9, fy=7, fz=4, z_begin=T + 0.05, z_end=T + 0.45)
    far = W.Grid(fx=9, fy=7, fz=4, z_begin=T + 0.05 + dz, z_end=T + 0.45 + dz)
    H = np.exp(1j * st.k * st.sz_bot * dz)
    E, I = cwt.filtered(st, sol, near, H)
    want = cwt.synthesize(st, sol, far)
    np.testing.assert_allclose(E, want, rtol=1e-11, atol=1e-13 * np.abs(want).max())
