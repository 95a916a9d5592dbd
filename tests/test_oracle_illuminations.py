"""Pins of the oracle used for several illuminations: the field is linear in
the incident coefficients of Sec. 2.3, so an incident image made of two
lattice plane waves (the image path: in-band DFT of the image) gives the sum
of the fields of the two plane waves taken one at a time (the plane-wave
path), on both boundary routes and on planes above, inside and below the
sample. Independent of the HIP library."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import cwt


def _problem():
    rng = np.random.default_rng(31)
    n = 1.3 + 0.3 * rng.random((3, 6, 8)) + 0.04j * rng.random((3, 6, 8))
    return W.Problem(n=n.astype(complex), px=0.31, py=0.27, pz=0.19, lam=1.0, U=5, V=5,
                     n_top=1.0, n_bot=1.45 + 0.01j)


@pytest.mark.parametrize("route", ["unreduced", "reduced"])
def test_image_of_two_plane_waves_is_the_sum_of_their_fields(route):
    prob = _problem()
    grid = W.Grid(fx=8, fy=6, fz=7, z_begin=-0.3, z_end=prob.thickness + 0.3)
    w1 = W.PlaneWave(1, -1, 0.8 + 0.1j, -0.3j)
    w2 = W.PlaneWave(-2, 2, -0.4, 0.5 + 0.5j)
    ny, nx = prob.ny, prob.nx
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")

    def wave(w):
        return np.exp(2j * np.pi * (w.u * ii / nx + w.v * jj / ny))

    img_x = w1.ex * wave(w1) + w2.ex * wave(w2)
    img_y = w1.ey * wave(w1) + w2.ey * wave(w2)

    def field(p):
        st = cwt.setup(p)
        return cwt.synthesize(st, cwt.solve(st, route=route), grid)

    both = field(dataclasses.replace(prob, inc_ex=img_x, inc_ey=img_y))
    one = field(dataclasses.replace(prob, plane_wave=w1))
    two = field(dataclasses.replace(prob, plane_wave=w2))
    np.testing.assert_allclose(both, one + two, rtol=0, atol=1e-11 * np.abs(both).max())
    # and the parts are not trivially related: each wave alone changes the field
    assert np.abs(one).max() > 0.1 * np.abs(both).max()
    assert np.abs(two).max() > 0.1 * np.abs(both).max()
