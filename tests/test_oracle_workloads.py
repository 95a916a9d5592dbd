"""Oracle checks on the benchmark workload families (sub-stacks that finish
in seconds): the reduced connection route used to write the full-size
reference agrees with the full boundary system, and the absorbing random
field satisfies the energy inequality."""
import numpy as np

import workloads as W
from oracle import cwt


def _fluxes(st, sol):
    M = st.M
    pin, pre, ptr = (a.reshape(3, M) for a in (st.p_inc, sol.p_ref, sol.p_trn))
    fi = cwt.z_flux(pin, cwt.h_coefficients(pin, st.sx, st.sy, st.sz_top))
    fr = -cwt.z_flux(pre, cwt.h_coefficients(pre, st.sx, st.sy, -st.sz_top))
    ft = cwt.z_flux(ptr, cwt.h_coefficients(ptr, st.sx, st.sy, st.sz_bot))
    return fi, fr, ft


def test_working_family_reduced_equals_unreduced():
    prob, _ = W.random_field_config("working", nz=3, U=7)
    st = cwt.setup(prob)
    a = cwt.solve(st, "unreduced")
    b = cwt.solve(st, "reduced")
    assert np.linalg.norm(a.p_trn - b.p_trn) < 1e-11 * np.linalg.norm(a.p_trn)
    assert np.linalg.norm(a.p_ref - b.p_ref) < 1e-11 * np.linalg.norm(a.p_ref)
    fi, fr, ft = _fluxes(st, a)
    assert fi > 0 and fr >= 0 and ft > 0 and fi - fr - ft > 0


def test_working_family_lossless_energy_balance():
    prob, _ = W.random_field_config("working", nz=2, U=5)
    prob.n = prob.n.real.astype(complex)
    st = cwt.setup(prob)
    sol = cwt.solve(st)
    fi, fr, ft = _fluxes(st, sol)
    assert abs(fi - fr - ft) < 1e-11 * fi


def test_working_golden_file_is_consistent():
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "working_samples.npz"),
                allow_pickle=False)
    assert g["E"].shape == (3, 4096) and int(g["M"]) == 441
    assert int(g["fx"]) == 256 and int(g["fz"]) == 128
    assert np.all(np.isfinite(g["E"])) and np.abs(g["E"]).max() > 0
    # transversality of the stored exterior waves (Eq. 14)
    prob, _ = W.random_field_config("working", nz=1)
    u, v = cwt.mode_indices(prob.U, prob.V)
    sx, sy = cwt.spatial_frequencies(u, v, prob.X, prob.Y, prob.lam)
    szt = cwt.s_z(1.0, sx, sy)
    pre = g["p_ref"].reshape(3, -1)
    ptr = g["p_trn"].reshape(3, -1)
    scale = np.abs(g["p_inc"]).max()
    assert np.abs(sx * pre[0] + sy * pre[1] - szt * pre[2]).max() < 1e-12 * scale
    assert np.abs(sx * ptr[0] + sy * ptr[1] + szt * ptr[2]).max() < 1e-12 * scale


def test_large_family_reduced_equals_unreduced():
    prob, _ = W.random_field_config("large", nz=2, U=7)
    st = cwt.setup(prob)
    a = cwt.solve(st, "unreduced")
    b = cwt.solve(st, "reduced")
    assert np.linalg.norm(a.p_trn - b.p_trn) < 1e-11 * np.linalg.norm(a.p_trn)
    assert np.linalg.norm(a.p_ref - b.p_ref) < 1e-11 * np.linalg.norm(a.p_ref)


def test_large_golden_file_is_consistent():
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "large_samples.npz"),
                allow_pickle=False)
    assert g["E"].shape == (3, 4096) and int(g["M"]) == 961
    assert int(g["fx"]) == 512 and int(g["fz"]) == 256
    assert np.all(np.isfinite(g["E"])) and np.abs(g["E"]).max() > 0
    prob, _ = W.random_field_config("large", nz=1)
    u, v = cwt.mode_indices(prob.U, prob.V)
    sx, sy = cwt.spatial_frequencies(u, v, prob.X, prob.Y, prob.lam)
    szt = cwt.s_z(1.0, sx, sy)
    pin = g["p_inc"].reshape(3, -1)
    pre = g["p_ref"].reshape(3, -1)
    ptr = g["p_trn"].reshape(3, -1)
    scale = np.abs(pin).max()
    # transversality of the stored exterior waves (Eq. 14)
    assert np.abs(sx * pre[0] + sy * pre[1] - szt * pre[2]).max() < 1e-12 * scale
    assert np.abs(sx * ptr[0] + sy * ptr[1] + szt * ptr[2]).max() < 1e-12 * scale
    # the absorbing sample takes energy: incident flux > reflected + transmitted
    fi = cwt.z_flux(pin, cwt.h_coefficients(pin, sx, sy, szt))
    fr = -cwt.z_flux(pre, cwt.h_coefficients(pre, sx, sy, -szt))
    ft = cwt.z_flux(ptr, cwt.h_coefficients(ptr, sx, sy, szt))
    assert fi > 0 and fr >= 0 and ft > 0 and fi - fr - ft > 0


def test_hard_sweep_golden_file_is_consistent():
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "sweep_hard_job.npz"),
                allow_pickle=False)
    assert g["E"].shape == (3, 8, 64, 64) and int(g["U"]) == 21
    assert np.all(np.isfinite(g["E"])) and np.abs(g["E"]).max() > 0
    prob, _ = W.sweep_problem(float(g["nu"]), int(g["patch"]), int(g["U"]), nz=1)
    u, v = cwt.mode_indices(prob.U, prob.V)
    sx, sy = cwt.spatial_frequencies(u, v, prob.X, prob.Y, prob.lam)
    szb = cwt.s_z(1.0, sx, sy)
    ptr = g["p_trn"].reshape(3, -1)
    pre = g["p_ref"].reshape(3, -1)
    # transversality of the transmitted and reflected waves (Eq. 14)
    assert np.abs(sx * ptr[0] + sy * ptr[1] + szb * ptr[2]).max() < 1e-10
    assert np.abs(sx * pre[0] + sy * pre[1] - szb * pre[2]).max() < 1e-10
    # an absorbing sample under a unit plane wave: reflected + transmitted < 1
    fr = -cwt.z_flux(pre, cwt.h_coefficients(pre, sx, sy, -szb))
    ft = cwt.z_flux(ptr, cwt.h_coefficients(ptr, sx, sy, szb))
    pin = np.zeros_like(ptr)
    pin[0, (prob.V // 2) * prob.U + prob.U // 2] = 1.0
    fi = cwt.z_flux(pin, cwt.h_coefficients(pin, sx, sy, szb))
    assert fi > 0 and fr >= 0 and ft > 0 and fi - fr - ft > 0


def test_u25_sweep_golden_file_is_consistent():
    """The widest sweep job (U = 25, band wrapped on the 32-voxel patch):
    transversality of its stored waves and energy accounting of an absorbing
    sample, as for the U = 21 job; the paper's reduced route is far off here."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "sweep_u25_job.npz"),
                allow_pickle=False)
    assert g["E"].shape == (3, 8, 64, 64) and int(g["U"]) == 25
    assert np.all(np.isfinite(g["E"])) and np.abs(g["E"]).max() > 0
    assert float(g["reduced_route_rel_l2"]) > 1e-2
    prob, _ = W.sweep_problem(float(g["nu"]), int(g["patch"]), int(g["U"]), nz=1)
    u, v = cwt.mode_indices(prob.U, prob.V)
    sx, sy = cwt.spatial_frequencies(u, v, prob.X, prob.Y, prob.lam)
    szb = cwt.s_z(1.0, sx, sy)
    ptr = g["p_trn"].reshape(3, -1)
    pre = g["p_ref"].reshape(3, -1)
    assert np.abs(sx * ptr[0] + sy * ptr[1] + szb * ptr[2]).max() < 1e-10
    assert np.abs(sx * pre[0] + sy * pre[1] - szb * pre[2]).max() < 1e-10
    fr = -cwt.z_flux(pre, cwt.h_coefficients(pre, sx, sy, -szb))
    ft = cwt.z_flux(ptr, cwt.h_coefficients(ptr, sx, sy, szb))
    pin = np.zeros_like(ptr)
    pin[0, (prob.V // 2) * prob.U + prob.U // 2] = 1.0
    fi = cwt.z_flux(pin, cwt.h_coefficients(pin, sx, sy, szb))
    assert fi > 0 and fr >= 0 and ft > 0 and fi - fr - ft > 0


def test_sphere_golden_file_matches_the_oracle():
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "sphere_samples.npz"),
                allow_pickle=False)
    prob, grid = W.sphere_config()
    st = cwt.setup(prob)
    sol = cwt.solve(st, "reduced")
    zs = grid.z_planes()
    x = g["f"][:64] * prob.X / grid.fx
    y = g["g"][:64] * prob.Y / grid.fy
    E = cwt.field_at_points(st, sol, x, y, zs[g["j"][:64]])
    # another route and the literal per-point sum reproduce the stored values
    assert np.linalg.norm(E - g["E"][:, :64]) <= 1e-12 * np.linalg.norm(g["E"][:, :64])
