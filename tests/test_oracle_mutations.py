"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch each one. Several mistakes are the paper's own misprints, so these tests
also document why the oracle reads those passages the way it does."""
import numpy as np
import pytest

import workloads as W
from oracle import cwt


def _checks():
    """A compact set of pins; returns the list of names that fail."""
    failed = []
    # Airy slab, normal incidence
    n1, ns, n3, T = 1.0, 1.5 + 0.02j, 1.2, 0.37
    prob = W.Problem(n=np.full((3, 4, 4), ns), px=0.25, py=0.25, pz=T / 3, lam=1.0,
                     U=1, V=1, n_top=n1, n_bot=n3, plane_wave=W.PlaneWave(0, 0, 1, 0))
    try:
        st = cwt.setup(prob)
        sol = cwt.solve(st)
        b = 2 * np.pi * ns * T
        r12, r23 = (n1 - ns) / (n1 + ns), (ns - n3) / (ns + n3)
        den = 1 + r12 * r23 * np.exp(2j * b)
        r = (r12 + r23 * np.exp(2j * b)) / den
        if abs(sol.p_ref[0] - r) > 1e-10:
            failed.append("airy")
    except Exception:
        failed.append("airy")
    # homogeneous eigenvalues and a lossless energy balance with oblique modes
    rng = np.random.default_rng(1)
    n = (1.3 + 0.3 * rng.random((3, 6, 6))).astype(complex)
    prob = W.Problem(n=n, px=0.5, py=0.5, pz=0.2, lam=1.0, U=3, V=3, n_top=1.0,
                     n_bot=1.4, plane_wave=W.PlaneWave(1, 0, 0.6, 0.8))
    try:
        st = cwt.setup(prob)
        sol = cwt.solve(st)
        M = st.M
        pin, pre, ptr = (a.reshape(3, M) for a in (st.p_inc, sol.p_ref, sol.p_trn))
        fi = cwt.z_flux(pin, cwt.h_coefficients(pin, st.sx, st.sy, st.sz_top))
        fr = -cwt.z_flux(pre, cwt.h_coefficients(pre, st.sx, st.sy, -st.sz_top))
        ft = cwt.z_flux(ptr, cwt.h_coefficients(ptr, st.sx, st.sy, st.sz_bot))
        if abs(fi - fr - ft) > 1e-9 * fi or fr < 0 or ft < 0:
            failed.append("energy")
        a = cwt.solve(st, "reduced")
        if np.linalg.norm(a.p_trn - sol.p_trn) > 1e-9 * np.linalg.norm(sol.p_trn):
            failed.append("reduced")
    except Exception:
        failed.append("energy")
    # transversality of a homogeneous layer's eigenmodes
    U = V = 3
    u, v = cwt.mode_indices(U, V)
    sx, sy = cwt.spatial_frequencies(u, v, 2.1, 1.9, 1.0)
    eps = np.full((4, 4), 2.1 + 0.03j)
    try:
        Phi = cwt.toeplitz_from_band(cwt.band_coefficients(eps, U, V), u, v, U, V)
        Psi = cwt.toeplitz_from_band(cwt.band_coefficients(1 / eps, U, V), u, v, U, V)
        md = cwt.layer_modes(cwt.property_matrix(Phi, Psi, sx, sy))
        M = U * V
        for q in range(4 * M):
            col = md.Q[:, q]
            pz = Psi @ (sy * col[2 * M:3 * M] - sx * col[3 * M:])
            if np.abs(sx * col[:M] + sy * col[M:2 * M] + md.gamma[q] * pz).max() > 1e-9:
                failed.append("gauss")
                break
    except Exception:
        failed.append("gauss")
    return failed


def test_unmutated_oracle_passes_compact_checks():
    assert _checks() == []


def _printed_D(Phi, Psi, sx, sy):
    # Lower block rows exactly as printed (outer products, opposite sign).
    M = sx.size
    I = np.eye(M)
    A = np.block([[np.outer(sx, sy) * Psi, I - np.outer(sx, sx) * Psi],
                  [np.outer(sy, sy) * Psi - I, -np.outer(sy, sx) * Psi]])
    C = np.block([[np.outer(sx, sy), Phi - np.outer(sx, sx)],
                  [np.outer(sy, sy) - Phi, -np.outer(sy, sx)]])
    Z = np.zeros((2 * M, 2 * M))
    return np.block([[Z, A], [C, Z]])


def _printed_C(sx, sy, sigma):
    # Third block row with -diag(s_y), as printed.
    M = sx.size
    I, Z = np.eye(M), np.zeros((M, M))
    return np.block([[I, Z, Z], [Z, I, Z], [Z, -np.diag(sigma), -np.diag(sy)],
                     [np.diag(sigma), Z, -np.diag(sx)]])


def _swapped_boundaries(modes, k, d):
    T, B = _orig_boundaries(modes, k, d)
    return B, T


_orig_boundaries = cwt.boundary_matrices
_orig_band = cwt.band_coefficients


def _unnormalised_band(f, U, V):
    return _orig_band(f, U, V) * f.size


def _flipped_branch(n, sx, sy):
    return -_orig_sz(n, sx, sy)


_orig_sz = cwt.s_z


@pytest.mark.parametrize("name,attr,repl", [
    ("printed lower rows of D", "property_matrix", _printed_D),
    ("printed sign of C row 3", "half_space_map", _printed_C),
    ("swapped top/bottom matrices", "boundary_matrices", _swapped_boundaries),
    ("band sum without 1/N", "band_coefficients", _unnormalised_band),
    ("wrong s_z branch", "s_z", _flipped_branch),
])
def test_pins_catch_planted_mistake(monkeypatch, name, attr, repl):
    monkeypatch.setattr(cwt, attr, repl)
    assert _checks() != [], name


def _interface_to_layer_above(st, z):
    # a plane exactly on z_l assigned to the layer above it
    zL = st.L * st.d
    if z <= 0.0:
        return -1
    if z > zL:
        return st.L
    return min(int(np.ceil(z / st.d)) - 1, st.L - 1)


def test_interface_pin_catches_the_layer_above_reading(monkeypatch):
    import test_oracle_pins as pins
    pins.test_plane_on_an_interface_takes_the_layer_below()
    monkeypatch.setattr(cwt, "layer_of", _interface_to_layer_above)
    with pytest.raises(AssertionError):
        pins.test_plane_on_an_interface_takes_the_layer_below()
