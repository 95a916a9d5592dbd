"""Lateral slices through the C ABI (Eq. 10 on an x-z or a y-z plane) against
the FP64 oracle: at on-grid positions against the oracle's volume, at
off-grid positions (also outside the first period) against its literal point
sum, on planes above, inside and below the sample."""
import numpy as np
import pytest

import workloads as W
from oracle import cwt

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-10, "fp32": 1e-4}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx():
    _torch()
    import paper_2404_07293_amd as P
    return P.Context(0)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def problem(seed=4):
    rng = np.random.default_rng(seed)
    nz, ny, nx = 3, 6, 8
    n = 1.3 + 0.3 * rng.random((nz, ny, nx)) + 0.04j * rng.random((nz, ny, nx))
    return W.Problem(n=n.astype(complex), px=0.31, py=0.27, pz=0.19, lam=1.0, U=5, V=3,
                     n_top=1.0, n_bot=1.45 + 0.01j,
                     plane_wave=W.PlaneWave(1, -1, 0.8, 0.3 - 0.2j))


def period(prob):
    return prob.n.shape[2] * prob.px, prob.n.shape[1] * prob.py


@pytest.fixture(scope="module")
def case(ctx):
    prob = problem()
    st = cwt.setup(prob)
    ref = cwt.solve(st)
    T = prob.thickness
    grid = W.Grid(fx=13, fy=7, fz=11, z_begin=-0.4, z_end=T + 0.4)
    return prob, st, ref, grid, cwt.synthesize(st, ref, grid), ctx.solve(prob)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_slice_on_grid_matches_oracle_volume(case, precision):
    torch = _torch()
    prob, st, ref, grid, vol, sol = case
    X, Y = period(prob)
    for g0 in (0, 3, 6):
        got = sol.synthesize_slice("xz", g0 * Y / grid.fy, grid.fx, grid.fz, grid.z_begin,
                                   grid.z_end, precision).cpu().numpy()
        torch.cuda.synchronize()
        err = rel_l2(got, vol[:, :, g0, :])
        print("%s x-z slice at row %d: rel-L2 %.3e" % (precision, g0, err))
        assert err <= TOL[precision]
    for f0 in (0, 5, 12):
        got = sol.synthesize_slice("yz", f0 * X / grid.fx, grid.fy, grid.fz, grid.z_begin,
                                   grid.z_end, precision).cpu().numpy()
        torch.cuda.synchronize()
        err = rel_l2(got, vol[:, :, :, f0])
        print("%s y-z slice at column %d: rel-L2 %.3e" % (precision, f0, err))
        assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_slice_off_grid_matches_point_sums(case, precision):
    torch = _torch()
    prob, st, ref, grid, vol, sol = case
    X, Y = period(prob)
    zs = grid.z_planes()
    for axis, pos, n in (("xz", 0.37 * Y - 2.0 * Y, 10), ("yz", 1.7 * X, 9), ("xz", 0.5, 1)):
        got = sol.synthesize_slice(axis, pos, n, grid.fz, grid.z_begin, grid.z_end,
                                   precision).cpu().numpy()
        torch.cuda.synchronize()
        lat = np.arange(n) * ((X if axis == "xz" else Y) / n)
        zz, ll = np.meshgrid(zs, lat, indexing="ij")
        xs = ll.ravel() if axis == "xz" else np.full(ll.size, pos)
        ys = np.full(ll.size, pos) if axis == "xz" else ll.ravel()
        want = cwt.field_at_points(st, ref, xs, ys, zz.ravel()).reshape(3, grid.fz, n)
        err = rel_l2(got, want)
        print("%s %s slice at %.3f, %d samples: rel-L2 %.3e" % (precision, axis, pos, n, err))
        assert err <= TOL[precision]


def test_slice_and_volume_plans_coexist(case):
    torch = _torch()
    prob, st, ref, grid, vol, sol = case
    X, Y = period(prob)
    first = sol.synthesize_slice("xz", 3 * Y / grid.fy, grid.fx, grid.fz, grid.z_begin,
                                 grid.z_end, "fp32").cpu().numpy()
    volume = sol.synthesize(grid, "fp32").cpu().numpy()
    again = sol.synthesize_slice("xz", 3 * Y / grid.fy, grid.fx, grid.fz, grid.z_begin,
                                 grid.z_end, "fp32").cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(first, again)
    assert rel_l2(volume, vol) <= TOL["fp32"]


def test_slice_rejects_bad_requests(case):
    import paper_2404_07293_amd as P
    prob, st, ref, grid, vol, sol = case
    with pytest.raises(P.ScwError):
        sol.synthesize_slice("xz", 0.1, 0, 4, 0.0, 1.0)
    with pytest.raises(P.ScwError):
        sol.synthesize_slice("xz", 0.1, 8, 4, 1.0, 1.0)
    with pytest.raises(P.ScwError):
        sol.synthesize_slice("yz", float("nan"), 8, 4, 0.0, 1.0)
    with pytest.raises(ValueError):
        sol.synthesize_slice("xz", 0.1, 8, 4, 0.0, 1.0, precision="bf16x3")
