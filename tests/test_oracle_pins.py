"""Pins of the FP64 oracle against closed forms, textbook results, invariants
and brute force. None of these compares the oracle with itself."""
import numpy as np
import pytest

import workloads as W
from oracle import cwt


def _uniform_problem(n_layers, ns, n_top, n_bot, U, V, X, thickness, pw,
                     lam=1.0, nxy=6):
    n = np.full((n_layers, nxy, nxy), complex(ns))
    return W.Problem(n=n, px=X / nxy, py=X / nxy, pz=thickness / n_layers,
                     lam=lam, U=U, V=V, n_top=n_top, n_bot=n_bot, plane_wave=pw)


def _same_multiset(a, b, atol):
    """Match two lists of complex numbers one to one (greedy nearest)."""
    a = list(np.asarray(a))
    for x in np.asarray(b):
        j = int(np.argmin(np.abs(np.asarray(a) - x)))
        assert abs(a[j] - x) < atol, (a[j], x)
        a.pop(j)


def _airy(r12, r23, t12, t23, beta):
    den = 1 + r12 * r23 * np.exp(2j * beta)
    return (r12 + r23 * np.exp(2j * beta)) / den, t12 * t23 * np.exp(1j * beta) / den


# ---------------------------------------------------------------- spectra
def test_band_coefficients_equal_direct_sum_with_wrap():
    rng = np.random.default_rng(11)
    f = rng.standard_normal((4, 5)) + 1j * rng.standard_normal((4, 5))
    # U = V = 5: the band (9 x 9) is wider than the 5 x 4 grid, so it wraps
    for U, V in ((3, 3), (5, 5), (3, 5)):
        np.testing.assert_allclose(cwt.band_coefficients(f, U, V),
                                   cwt.band_coefficients_direct(f, U, V),
                                   rtol=0, atol=1e-13)


def test_toeplitz_product_is_circular_convolution_on_the_grid():
    # (eps * E) sampled on the voxel grid has DFT coefficients Phi @ e at every
    # in-band frequency when E is band-limited: the convolution theorem.
    rng = np.random.default_rng(3)
    ny, nx, U, V = 7, 9, 5, 3
    eps = rng.uniform(1, 3, (ny, nx)) + 1j * rng.uniform(0, .2, (ny, nx))
    u, v = cwt.mode_indices(U, V)
    e = rng.standard_normal(U * V) + 1j * rng.standard_normal(U * V)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    E = sum(e[m] * np.exp(2j * np.pi * (u[m] * i / nx + v[m] * j / ny))
            for m in range(U * V))
    prod = np.fft.fft2(eps * E) / (nx * ny)
    want = prod[v % ny, u % nx]
    Phi = cwt.toeplitz_from_band(cwt.band_coefficients(eps, U, V), u, v, U, V)
    np.testing.assert_allclose(Phi @ e, want, rtol=0, atol=1e-12)


def test_homogeneous_layer_spectra_are_delta():
    f = np.full((6, 8), 2.25 + 0.1j)
    c = cwt.band_coefficients(f, 3, 5)
    assert abs(c[4, 2] - (2.25 + 0.1j)) < 1e-15
    c[4, 2] = 0
    assert np.abs(c).max() < 1e-15


# ---------------------------------------------------------------- D and modes
@pytest.mark.parametrize("n_layer", [1.5, 1.3 + 0.05j])
def test_homogeneous_eigenvalues_are_plus_minus_sz(n_layer):
    U = V = 5
    X = 1.7            # some modes evanescent (|s| up to 1.66)
    u, v = cwt.mode_indices(U, V)
    sx, sy = cwt.spatial_frequencies(u, v, X, X, 1.0)
    eps = np.full((6, 6), complex(n_layer) ** 2)
    Phi = cwt.toeplitz_from_band(cwt.band_coefficients(eps, U, V), u, v, U, V)
    Psi = cwt.toeplitz_from_band(cwt.band_coefficients(1 / eps, U, V), u, v, U, V)
    md = cwt.layer_modes(cwt.property_matrix(Phi, Psi, sx, sy))
    sz = cwt.s_z(n_layer, sx, sy)
    _same_multiset(md.gamma, np.concatenate([sz, sz, -sz, -sz]), 1e-12)
    # forward modes are exactly the +s_z branch
    _same_multiset(md.gamma[md.forward], np.concatenate([sz, sz]), 1e-12)


def test_eigenmodes_are_transverse_in_homogeneous_layer():
    # With p_z = Psi (S_y b_x - S_x b_y), each eigenmode satisfies s . p = 0
    # for s = (s_x, s_y, gamma): Gauss's law in the layer.
    U = V = 3
    u, v = cwt.mode_indices(U, V)
    sx, sy = cwt.spatial_frequencies(u, v, 2.1, 1.9, 1.0)
    n = 1.45 + 0.02j
    eps = np.full((4, 4), n ** 2)
    Phi = cwt.toeplitz_from_band(cwt.band_coefficients(eps, U, V), u, v, U, V)
    Psi = cwt.toeplitz_from_band(cwt.band_coefficients(1 / eps, U, V), u, v, U, V)
    md = cwt.layer_modes(cwt.property_matrix(Phi, Psi, sx, sy))
    M = U * V
    for q in range(4 * M):
        col = md.Q[:, q]
        px, py, bx, by = col[:M], col[M:2 * M], col[2 * M:3 * M], col[3 * M:]
        pz = Psi @ (sy * bx - sx * by)
        div = sx * px + sy * py + md.gamma[q] * pz
        assert np.abs(div).max() < 1e-12 * np.abs(col).max()


# ---------------------------------------------------------------- slabs
@pytest.mark.parametrize("ns", [1.5, 1.4 + 0.05j])
def test_slab_normal_incidence_matches_airy(ns):
    n1, n3, T = 1.0, 1.2 + 0.01j, 0.37
    prob = _uniform_problem(3, ns, n1, n3, 1, 1, 1.0, T, W.PlaneWave(0, 0, 1, 0))
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    k = 2 * np.pi
    r, t = _airy((n1 - ns) / (n1 + ns), (ns - n3) / (ns + n3),
                 2 * n1 / (n1 + ns), 2 * ns / (ns + n3), k * ns * T)
    assert abs(sol.p_ref[0] - r) < 1e-12
    assert abs(sol.p_trn[0] - t) < 1e-12
    if np.isreal(ns) and np.isreal(n3):
        assert abs(abs(r) ** 2 + (n3.real / n1) * abs(t) ** 2 - 1) < 1e-12


def _oblique_setup(ns, n1=1.0, n3=1.33, T=0.61, X=2.3, pw=None):
    prob = _uniform_problem(2, ns, n1, n3, 3, 3, X, T, pw)
    st = cwt.setup(prob)
    return prob, st, cwt.solve(st)


@pytest.mark.parametrize("ns", [1.6, 1.5 + 0.03j])
def test_slab_oblique_te_matches_fresnel_airy(ns):
    n1, n3 = 1.0, 1.33
    prob, st, sol = _oblique_setup(ns, pw=W.PlaneWave(1, 0, 0.0, 1.0))
    m = int(np.nonzero((st.u == 1) & (st.v == 0))[0][0])
    M = st.M
    s = st.sx[m]
    s1, s2, s3 = (cwt.s_z(n, s, 0.0) for n in (n1, ns, n3))
    r, t = _airy((s1 - s2) / (s1 + s2), (s2 - s3) / (s2 + s3),
                 2 * s1 / (s1 + s2), 2 * s2 / (s2 + s3), 2 * np.pi * s2 * 0.61)
    assert abs(sol.p_ref[M + m] - r) < 1e-12
    assert abs(sol.p_trn[M + m] - t) < 1e-12
    # all other modes stay dark
    other = np.ones(3 * M, bool)
    other[[m, M + m, 2 * M + m]] = False
    assert np.abs(sol.p_ref[other]).max() < 1e-12
    assert np.abs(sol.p_trn[other]).max() < 1e-12


@pytest.mark.parametrize("ns", [1.6, 1.5 + 0.03j])
def test_slab_oblique_tm_matches_fresnel_airy(ns):
    n1, n3 = 1.0, 1.33
    prob, st, sol = _oblique_setup(ns, pw=W.PlaneWave(1, 0, 1.0, 0.0))
    m = int(np.nonzero((st.u == 1) & (st.v == 0))[0][0])
    M = st.M
    s = st.sx[m]
    e1, e2, e3 = n1 ** 2, ns ** 2, n3 ** 2
    s1, s2, s3 = (cwt.s_z(n, s, 0.0) for n in (n1, ns, n3))

    def rr(ea, sa, eb, sb):
        return (eb * sa - ea * sb) / (eb * sa + ea * sb)

    r12, r23 = rr(e1, s1, e2, s2), rr(e2, s2, e3, s3)
    r, t = _airy(r12, r23, 1 + r12, 1 + r23, 2 * np.pi * s2 * 0.61)
    p_inc = st.p_inc.reshape(3, M)[:, m]
    p_ref = sol.p_ref.reshape(3, M)[:, m]
    p_trn = sol.p_trn.reshape(3, M)[:, m]
    hy_inc = s1 * p_inc[0] - s * p_inc[2]
    hy_ref = -s1 * p_ref[0] - s * p_ref[2]
    hy_trn = s3 * p_trn[0] - s * p_trn[2]
    assert abs(hy_ref / hy_inc - r) < 1e-12
    assert abs(hy_trn / hy_inc - t) < 1e-12


def _characteristic_matrix_rt(n_layers, d, n0, nsub, lam=1.0):
    """Thin-film stack at normal incidence by the characteristic-matrix method
    (Born & Wolf, Principles of Optics, Sec. 1.6)."""
    k = 2 * np.pi / lam
    Mt = np.eye(2, dtype=complex)
    for n in n_layers:
        b = k * n * d
        Mt = Mt @ np.array([[np.cos(b), -1j * np.sin(b) / n],
                            [-1j * n * np.sin(b), np.cos(b)]])
    Bc = Mt @ np.array([1.0, nsub])
    den = n0 * Bc[0] + Bc[1]
    return (n0 * Bc[0] - Bc[1]) / den, 2 * n0 / den


def test_single_frequency_reduces_to_thin_film_stack():
    # M = 1: each layer acts as a film of index sqrt(mean(n^2)) (Phi = phi_0).
    rng = np.random.default_rng(5)
    n = 1.3 + 0.3 * rng.random((5, 8, 8)) + 0.02j * rng.random((5, 8, 8))
    prob = W.Problem(n=n, px=0.2, py=0.2, pz=0.13, lam=1.0, U=1, V=1, n_top=1.0,
                     n_bot=1.5 + 0j)
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    neff = [np.sqrt(np.mean(n[l] ** 2)) for l in range(5)]
    r, t = _characteristic_matrix_rt(neff, 0.13, 1.0, 1.5)
    assert abs(sol.p_ref[0] - r) < 1e-12
    assert abs(sol.p_trn[0] - t) < 1e-12


# ---------------------------------------------------------------- uniform medium
def test_uniform_medium_propagates_incident_field_exactly():
    n = 1.33
    prob = _uniform_problem(3, n, n, n, 5, 3, 2.2, 0.9, W.PlaneWave(0, 0, 1, 0))
    rng = np.random.default_rng(8)
    prob.inc_ex = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    prob.inc_ey = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    assert np.abs(sol.p_ref).max() < 1e-12
    prop = np.tile(np.exp(1j * st.k * st.sz_top * 0.9), 3)
    np.testing.assert_allclose(sol.p_trn, st.p_inc * prop, atol=1e-12)
    # interior field at random points = brute-force sum of incident plane waves
    pts = rng.random((3, 20)) * np.array([[2.2], [2.2], [0.9]])
    E = cwt.field_at_points(st, sol, *pts)
    pin = st.p_inc.reshape(3, st.M)
    for q in range(20):
        x, y, z = pts[:, q]
        ph = np.exp(1j * st.k * (st.sx * x + st.sy * y + st.sz_top * z))
        np.testing.assert_allclose(E[:, q], pin @ ph, atol=1e-11)


# ---------------------------------------------------------------- energy, Gauss
def _random_problem(seed, lossless, U=5, nz=3, nxy=8, X=4.0, n_bot=1.0):
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((nz, nxy, nxy))
    if not lossless:
        n = n + 0.05j * rng.random((nz, nxy, nxy))
    return W.Problem(n=n.astype(complex), px=X / nxy, py=X / nxy, pz=0.21,
                     lam=1.0, U=U, V=U, n_top=1.0, n_bot=complex(n_bot),
                     plane_wave=W.PlaneWave(1, -1, 0.7, 0.4j))


def _fluxes(st, sol):
    M = st.M
    pin = st.p_inc.reshape(3, M)
    pre = sol.p_ref.reshape(3, M)
    ptr = sol.p_trn.reshape(3, M)
    bin_ = cwt.h_coefficients(pin, st.sx, st.sy, st.sz_top)
    bre = cwt.h_coefficients(pre, st.sx, st.sy, -st.sz_top)
    btr = cwt.h_coefficients(ptr, st.sx, st.sy, st.sz_bot)
    top = cwt.z_flux(pin + pre, bin_ + bre)
    return (cwt.z_flux(pin, bin_), -cwt.z_flux(pre, bre), cwt.z_flux(ptr, btr), top)


def test_energy_conserved_for_lossless_sample():
    st = cwt.setup(_random_problem(1, True, n_bot=1.5))
    sol = cwt.solve(st)
    inc, ref, trn, top = _fluxes(st, sol)
    assert inc > 0 and ref > 0 and trn > 0
    assert abs(inc - ref - trn) < 1e-12 * inc
    assert abs(top - trn) < 1e-12 * inc


def test_energy_absorbed_by_lossy_sample():
    st = cwt.setup(_random_problem(2, False))
    sol = cwt.solve(st)
    inc, ref, trn, _ = _fluxes(st, sol)
    assert inc - ref - trn > 1e-4 * inc


def test_exterior_waves_are_transverse():
    st = cwt.setup(_random_problem(3, False))
    sol = cwt.solve(st)
    M = st.M
    pre = sol.p_ref.reshape(3, M)
    ptr = sol.p_trn.reshape(3, M)
    assert np.abs(st.sx * pre[0] + st.sy * pre[1] - st.sz_top * pre[2]).max() < 1e-13
    assert np.abs(st.sx * ptr[0] + st.sy * ptr[1] + st.sz_bot * ptr[2]).max() < 1e-13
    # E . H = 0 for each plane wave (Sec. 2.1)
    b = cwt.h_coefficients(ptr, st.sx, st.sy, st.sz_bot)
    assert np.abs(np.sum(ptr * b, axis=0)).max() < 1e-13


# ---------------------------------------------------------------- structure
def test_layer_split_invariance():
    prob = _random_problem(4, False, nz=3)
    n2 = np.repeat(prob.n, 2, axis=0)
    prob2 = W.Problem(n=n2, px=prob.px, py=prob.py, pz=prob.pz / 2, lam=1.0,
                      U=prob.U, V=prob.V, n_top=1.0, n_bot=prob.n_bot,
                      plane_wave=prob.plane_wave)
    grid = W.Grid(fx=8, fy=8, fz=6, z_begin=-0.1, z_end=prob.thickness + 0.1)
    st1, sol1, E1 = cwt.simulate(prob, grid)
    st2, sol2, E2 = cwt.simulate(prob2, grid)
    np.testing.assert_allclose(sol2.p_ref, sol1.p_ref, atol=1e-11)
    np.testing.assert_allclose(sol2.p_trn, sol1.p_trn, atol=1e-11)
    assert np.linalg.norm(E2 - E1) < 1e-10 * np.linalg.norm(E1)


def test_reduced_route_equals_unreduced_system():
    st = cwt.setup(_random_problem(6, False, nz=4))
    a = cwt.solve(st, "unreduced")
    b = cwt.solve(st, "reduced")
    np.testing.assert_allclose(b.p_ref, a.p_ref, atol=1e-12)
    np.testing.assert_allclose(b.p_trn, a.p_trn, atol=1e-12)
    for x, y in zip(a.alpha, b.alpha):
        assert np.linalg.norm(x - y) < 1e-11 * np.linalg.norm(x)


def test_interfaces_are_continuous():
    # tangential E and H match across every interface (Eqs. 17-18)
    st = cwt.setup(_random_problem(7, False, nz=3))
    sol = cwt.solve(st)
    M = st.M
    for layer in range(st.L - 1):
        z = (layer + 1) * st.d
        above = cwt.interior_R(st, sol, layer, z)
        below = cwt.interior_R(st, sol, layer + 1, z)
        assert np.linalg.norm(above - below) < 1e-12 * np.linalg.norm(above)
    # top surface: exterior incident + reflected = layer 1 at z0
    C_i = cwt.half_space_map(st.sx, st.sy, st.sz_top)
    C_r = cwt.half_space_map(st.sx, st.sy, -st.sz_top)
    ext = C_i @ st.p_inc + C_r @ sol.p_ref
    np.testing.assert_allclose(cwt.interior_R(st, sol, 0, 0.0), ext, atol=1e-12)
    C_t = cwt.half_space_map(st.sx, st.sy, st.sz_bot)
    zl = st.L * st.d
    np.testing.assert_allclose(cwt.interior_R(st, sol, st.L - 1, zl), C_t @ sol.p_trn,
                               atol=1e-12)
    assert M > 1


def test_sphere_mirror_symmetry():
    prob, grid = W.sphere_config(out=16)
    st, sol, E = cwt.simulate(prob, grid)
    fl = lambda a, ax: np.roll(np.flip(a, axis=ax), 1, axis=ax)   # f -> -f mod F
    Ex, Ey, Ez = E
    scale = np.abs(E).max()
    assert np.abs(Ex - fl(Ex, 2)).max() < 1e-12 * scale
    assert np.abs(Ex - fl(Ex, 1)).max() < 1e-12 * scale
    assert np.abs(Ey + fl(Ey, 2)).max() < 1e-12 * scale
    assert np.abs(Ey + fl(Ey, 1)).max() < 1e-12 * scale
    assert np.abs(Ez + fl(Ez, 2)).max() < 1e-12 * scale
    assert np.abs(Ez - fl(Ez, 1)).max() < 1e-12 * scale
    assert np.abs(Ey).max() > 1e-4 * scale and np.abs(Ez).max() > 1e-3 * scale


# ---------------------------------------------------------------- synthesis
def test_grid_synthesis_equals_pointwise_sum_and_fft():
    st = cwt.setup(_random_problem(9, False, nz=2, U=3))
    sol = cwt.solve(st)
    grid = W.Grid(fx=10, fy=12, fz=5, z_begin=-0.3, z_end=st.L * st.d + 0.3)
    E = cwt.synthesize(st, sol, grid)
    zs = grid.z_planes()
    rng = np.random.default_rng(0)
    j = rng.integers(0, grid.fz, 15)
    g = rng.integers(0, grid.fy, 15)
    f = rng.integers(0, grid.fx, 15)
    x = f * st.X / grid.fx
    y = g * st.Y / grid.fy
    pts = cwt.field_at_points(st, sol, x, y, zs[j])
    for q in range(15):
        ph = np.exp(1j * st.k * (st.sx * x[q] + st.sy * y[q]))
        want = cwt.plane_coefficients(st, sol, zs[j[q]]) @ ph
        np.testing.assert_allclose(pts[:, q], want, atol=1e-12)
        np.testing.assert_allclose(E[:, j[q], g[q], f[q]], want, atol=1e-12)
    # zero-padded inverse FFT gives the same plane
    p = cwt.plane_coefficients(st, sol, zs[2])
    for c in range(3):
        spec = np.zeros((grid.fy, grid.fx), complex)
        spec[st.v % grid.fy, st.u % grid.fx] = p[c]
        np.testing.assert_allclose(np.fft.ifft2(spec) * grid.fx * grid.fy, E[c, 2],
                                   atol=1e-12)


def test_grazing_frequency_is_rejected():
    # X = 2 lam puts (u, v) = (2, 0) exactly at |s| = 1 = n_top
    prob = _uniform_problem(1, 1.5, 1.0, 1.0, 5, 1, 2.0, 0.3, W.PlaneWave(0, 0, 1, 0))
    with pytest.raises(cwt.OracleError):
        cwt.setup(prob)


def test_even_truncation_rejected():
    prob = _uniform_problem(1, 1.5, 1.0, 1.0, 4, 3, 2.3, 0.3, W.PlaneWave(0, 0, 1, 0))
    with pytest.raises(cwt.OracleError):
        cwt.setup(prob)


# ---------------------------------------------------------------- interfaces (R14)
def _film_stack():
    """Three homogeneous layers of different index between two half-spaces,
    lit by an oblique p-polarised lattice plane wave (E_z != 0). Pitch 0.25 so
    that every interface z_l = l * 0.25 is exact in binary."""
    ns = [1.3, 1.7 + 0.02j, 1.5]
    n = np.stack([np.full((4, 4), complex(x)) for x in ns])
    prob = W.Problem(n=n, px=0.6, py=0.6, pz=0.25, lam=1.0, U=3, V=3, n_top=1.0,
                     n_bot=1.2 + 0.01j, plane_wave=W.PlaneWave(1, 0, 1.0, 0.0))
    return prob, [prob.n_top] + ns + [prob.n_bot]


def test_plane_on_an_interface_takes_the_layer_below():
    """Across an interface tangential E is continuous and the normal D = eps E_z
    is continuous (Gauss's law, no surface charge), so E_z jumps by
    eps_above / eps_below. A plane exactly on z_l must give the tangential
    field of both sides and the E_z of the region below it (including z0,
    which belongs to layer 1, and z_L, which belongs to the lower
    half-space)."""
    prob, n_regions = _film_stack()
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    m = int(np.nonzero((st.u == 1) & (st.v == 0))[0][0])
    delta = 1e-9
    for ell in range(st.L + 1):
        z = ell * st.d
        at = cwt.plane_coefficients(st, sol, z)[:, m]
        up = cwt.plane_coefficients(st, sol, z - delta)[:, m]
        dn = cwt.plane_coefficients(st, sol, z + delta)[:, m]
        scale = np.abs(at).max()
        eps_up, eps_dn = complex(n_regions[ell]) ** 2, complex(n_regions[ell + 1]) ** 2
        assert np.abs(at[:2] - up[:2]).max() < 1e-7 * scale, ell
        assert np.abs(at[:2] - dn[:2]).max() < 1e-7 * scale, ell
        assert abs(eps_up * up[2] - eps_dn * dn[2]) < 1e-7 * scale, ell
        assert abs(up[2] - dn[2]) > 1e-2 * scale, ell      # E_z does jump here
        assert abs(at[2] - dn[2]) < 1e-7 * scale, ell      # ... and z_l takes the side below
    # a cell-centred grid from -d/2 with one plane per layer lands on every
    # interface exactly; its synthesized planes are those coefficients
    grid = W.Grid(fx=3, fy=3, fz=st.L + 1, z_begin=-st.d / 2, z_end=(st.L + 0.5) * st.d)
    zs = grid.z_planes()
    assert np.array_equal(zs, np.arange(st.L + 1) * st.d)
    E = cwt.synthesize(st, sol, grid)
    for ell in range(st.L + 1):
        p = cwt.plane_coefficients(st, sol, ell * st.d)
        np.testing.assert_allclose(E[:, ell, 0, 0], p.sum(axis=1), atol=1e-13)


# ---------------------------------------------------------------- rejections
def test_layer_modes_rejects_unpaired_and_near_defective_spectra():
    # diagonal D: the eigenvalues are its entries, so the split is known
    ok = cwt.layer_modes(np.diag([1.0, 0.5 + 0.1j, -1.0, -0.5 - 0.1j]).astype(complex))
    assert ok.forward.tolist() == [True, True, False, False]
    with pytest.raises(cwt.OracleError, match="forward mode count"):
        cwt.layer_modes(np.diag([1.0, 2.0, 3.0, -1.0]).astype(complex))
    with pytest.raises(cwt.OracleError, match="near-defective"):
        cwt.layer_modes(np.diag([1.0, 1e-10, -1.0, -1e-10]).astype(complex))


def test_grazing_mode_inside_a_layer_is_rejected():
    """A homogeneous layer with eps = s_x^2 for a lattice mode (n = 0.5,
    X = 2 lambda, u = 1) has gamma = sqrt(eps - s^2) = 0 exactly: D is
    defective there and the layer cannot be expanded in its modes."""
    n = np.full((2, 1, 4), 0.5 + 0j)
    prob = W.Problem(n=n, px=0.5, py=0.5, pz=0.2, lam=1.0, U=3, V=1)
    with pytest.raises(cwt.OracleError):
        cwt.setup(prob)
    n[:] = 0.6  # away from grazing the same layout solves
    cwt.setup(prob)


def test_banded_full_system_equals_dense_solve():
    """The banded LU route of the full boundary system (rows reordered so
    that the matrix is banded) gives the dense solve's coefficients and layer
    amplitudes, on a lossy ragged stack with an oblique wave."""
    rng = np.random.default_rng(12)
    n = 1.3 + 0.3 * rng.random((4, 7, 9)) + 0.05j * rng.random((4, 7, 9))
    prob = W.Problem(n=n.astype(complex), px=0.29, py=0.31, pz=0.17, lam=1.0, U=5, V=5,
                     n_top=1.0, n_bot=1.35 + 0.02j, plane_wave=W.PlaneWave(1, 2, 0.6, -0.4j))
    st = cwt.setup(prob)
    dense = cwt.solve_unreduced(st)
    band = cwt.solve_unreduced_banded(st)
    assert np.abs(band.p_trn - dense.p_trn).max() <= 1e-12 * np.abs(dense.p_trn).max()
    assert np.abs(band.p_ref - dense.p_ref).max() <= 1e-12 * np.abs(dense.p_ref).max()
    for a, b in zip(band.alpha, dense.alpha):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
