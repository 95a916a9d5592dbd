"""Many plane-wave illuminations of one sample sharing one setup
(scw_solve_illuminations + scw_synthesize_illuminations) against the FP64
oracle run once per illumination: each illumination is the problem of Sec. 2.3
with that plane wave as its incident field, so the oracle needs no arithmetic
of its own here. Cases: both boundary routes, more illuminations than one
matrix-core launch group holds (a ragged last group), illumination 0 against
the single-illumination path, linearity in the incident amplitudes, a single
illumination, a plain solution's own incident image, grids with no interior
plane, and the 64x64x32 working sample at full size against separate single
solves."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import cwt

pytestmark = pytest.mark.gpu
TOL = 1e-4  # FP32 synthesis


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


def problem(seed=12, U=5, V=5):
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((3, 6, 8)) + 0.04j * rng.random((3, 6, 8))
    return W.Problem(n=n.astype(complex), px=0.31, py=0.27, pz=0.19, lam=1.0, U=U, V=V,
                     n_top=1.0, n_bot=1.45 + 0.01j)


def waves(count, U, V, seed=3):
    """Distinct-looking plane waves on the U x V band, random polarisation."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        u = int(rng.integers(-(U // 2), U // 2 + 1))
        v = int(rng.integers(-(V // 2), V // 2 + 1))
        ex, ey = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        out.append(W.PlaneWave(u, v, complex(ex), complex(ey)))
    return out


def oracle_fields(prob, ws, grid, route="unreduced"):
    out = []
    for w in ws:
        st = cwt.setup(dataclasses.replace(prob, plane_wave=w, inc_ex=None, inc_ey=None))
        out.append(cwt.synthesize(st, cwt.solve(st, route=route), grid))
    return np.stack(out)


@pytest.mark.parametrize("route,count", [("stable", 5), ("stable", 37), ("connection", 6)])
def test_illuminations_match_oracle(ctx, route, count):
    torch = _torch()
    prob = problem()
    ws = waves(count, prob.U, prob.V, seed=count)
    grid = W.Grid(fx=12, fy=10, fz=9, z_begin=-0.35, z_end=prob.thickness + 0.35)
    sol = ctx.solve(prob, route=route, waves=ws)
    got = sol.synthesize_illuminations(grid).cpu().numpy()
    torch.cuda.synchronize()
    want = oracle_fields(prob, ws, grid, "unreduced" if route == "stable" else "reduced")
    errs = [rel_l2(got[k], want[k]) for k in range(count)]
    print("%s route, %d illuminations: max rel-L2 %.3e" % (route, count, max(errs)))
    assert max(errs) <= TOL


def test_dense_planes_fill_the_launch_group(ctx):
    """8 planes per layer (4 illuminations per 32-column group): the groups
    hold full and partial plane sets, and exterior planes on both sides."""
    torch = _torch()
    prob = problem(seed=5, U=7, V=3)
    ws = waves(9, prob.U, prob.V, seed=9)
    T = prob.thickness
    grid = W.Grid(fx=16, fy=8, fz=30, z_begin=-0.1, z_end=T + 0.1)
    sol = ctx.solve(prob, waves=ws)
    got = sol.synthesize_illuminations(grid).cpu().numpy()
    torch.cuda.synchronize()
    want = oracle_fields(prob, ws, grid)
    errs = [rel_l2(got[k], want[k]) for k in range(len(ws))]
    print("30 planes, 9 illuminations: max rel-L2 %.3e" % max(errs))
    assert max(errs) <= TOL


def test_first_illumination_matches_single_path_and_linearity(ctx):
    torch = _torch()
    prob = problem(seed=2)
    w1 = W.PlaneWave(1, -1, 0.8, 0.3 - 0.2j)
    w2 = W.PlaneWave(1, -1, -0.1 + 0.5j, 0.7)
    w12 = W.PlaneWave(1, -1, w1.ex + w2.ex, w1.ey + w2.ey)
    grid = W.Grid(fx=16, fy=16, fz=12, z_begin=-0.3, z_end=prob.thickness + 0.3)
    sol = ctx.solve(prob, waves=[w1, w2, w12])
    E = sol.synthesize_illuminations(grid).cpu().numpy()
    E0 = sol.synthesize(grid, "fp32").cpu().numpy()
    torch.cuda.synchronize()
    single = rel_l2(E[0], E0)
    lin = rel_l2(E[0] + E[1], E[2])
    print("illumination 0 vs single path %.3e; linearity %.3e" % (single, lin))
    assert single <= 1e-5
    assert lin <= 1e-5
    # the exterior coefficients reported are illumination 0's
    st = cwt.setup(dataclasses.replace(prob, plane_wave=w1))
    ref = cwt.solve(st)
    p_inc, p_ref, p_trn = sol.exterior()
    assert rel_l2(p_ref.ravel(), ref.p_ref) <= 1e-10
    assert rel_l2(p_trn.ravel(), ref.p_trn) <= 1e-10


def test_illuminations_reject_bad_requests(ctx):
    import ctypes
    import paper_2404_07293_amd as P
    from paper_2404_07293_amd import _native as N
    prob = problem()
    with pytest.raises(P.ScwError):
        ctx.solve(prob, waves=[W.PlaneWave(5, 0, 1.0, 0.0)])  # outside the 5 x 5 band
    with pytest.raises(P.ScwError):
        ctx.solve(prob, waves=[])
    sol = ctx.solve(prob, waves=waves(2, 5, 5))
    grid = W.Grid(fx=8, fy=8, fz=4, z_begin=0.0, z_end=0.5)
    torch = _torch()
    buf = torch.empty((2, 3, 4, 8, 8), dtype=torch.complex128, device="cuda")
    rc = sol.lib.scw_synthesize_illuminations(ctx.handle, sol.handle, ctypes.byref(N.ScwGrid(
        8, 8, 4, 0.0, 0.5)), N.PRECISION["fp64"], ctypes.c_void_p(buf.data_ptr()), None)
    assert rc == -1
    with pytest.raises(ValueError):
        sol.synthesize_illuminations(grid, out=buf)


def test_working_sample_against_single_solves(ctx):
    """64x64x32 random-field sample, M = 441, 256 x 256 x 128 grid, 8
    illuminations: two of them against a separate scw_solve of the same
    plane wave through the single-illumination path (itself checked against
    the oracle at this size)."""
    torch = _torch()
    prob, grid = W.random_field_config("working")
    ws = [W.PlaneWave(0, 0, 1.0, 0.0)] + waves(7, prob.U, prob.V, seed=41)
    sol = ctx.solve(prob, waves=ws)
    E = sol.synthesize_illuminations(grid)
    for k in (0, 5):
        single = ctx.solve(dataclasses.replace(prob, plane_wave=ws[k], inc_ex=None, inc_ey=None))
        Es = single.synthesize(grid, "fp32")
        torch.cuda.synchronize()
        err = float(torch.linalg.vector_norm(E[k] - Es) / torch.linalg.vector_norm(Es))
        print("working sample, illumination %d vs its single solve: rel-L2 %.3e" % (k, err))
        assert err <= 1e-5
        single.free()


def test_single_illumination_and_plain_solution(ctx):
    """K = 1 (the single-illumination coefficient buffer) against the oracle,
    and the illumination synthesis of a plain scw_solve solution (its own
    incident image) against scw_synthesize."""
    torch = _torch()
    prob = problem(seed=4)
    w = W.PlaneWave(-1, 2, 0.3 + 0.4j, -0.9)
    grid = W.Grid(fx=10, fy=12, fz=8, z_begin=-0.2, z_end=prob.thickness + 0.2)
    sol = ctx.solve(prob, waves=[w])
    got = sol.synthesize_illuminations(grid).cpu().numpy()
    torch.cuda.synchronize()
    err = rel_l2(got[0], oracle_fields(prob, [w], grid)[0])
    print("one illumination: rel-L2 %.3e" % err)
    assert err <= TOL
    rng = np.random.default_rng(8)
    img = rng.standard_normal((6, 8)) + 1j * rng.standard_normal((6, 8))
    plain = ctx.solve(dataclasses.replace(prob, inc_ex=img, inc_ey=0.5 * img))
    E1 = plain.synthesize_illuminations(grid).cpu().numpy()
    E0 = plain.synthesize(grid, "fp32").cpu().numpy()
    torch.cuda.synchronize()
    assert E1.shape == (1,) + E0.shape
    assert rel_l2(E1[0], E0) <= 1e-5


def test_exterior_only_grid(ctx):
    """Planes only above and below the sample: no interior task."""
    torch = _torch()
    prob = problem(seed=6)
    ws = waves(3, prob.U, prob.V, seed=6)
    T = prob.thickness
    sol = ctx.solve(prob, waves=ws)
    for grid in (W.Grid(fx=8, fy=8, fz=5, z_begin=-0.6, z_end=-0.01),
                 W.Grid(fx=8, fy=8, fz=5, z_begin=T + 0.01, z_end=T + 0.7)):
        got = sol.synthesize_illuminations(grid).cpu().numpy()
        torch.cuda.synchronize()
        want = oracle_fields(prob, ws, grid)
        errs = [rel_l2(got[k], want[k]) for k in range(len(ws))]
        print("exterior-only grid [%.2f, %.2f]: max rel-L2 %.3e"
              % (grid.z_begin, grid.z_end, max(errs)))
        assert max(errs) <= TOL
