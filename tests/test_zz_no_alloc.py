"""The allocation-free synthesis (scw_synthesize_noalloc) against
scw_synthesize, through the C ABI.

Both run the same modal-sum, exterior and transform kernels; the no-alloc
form builds the plane tables and twiddles on the device into the static
scratch array. Bounds: FP64 1e-12 and FP32 1e-6 relative L2, and the same
per element relative to the largest value (the twiddles may differ from the
host's in the last bit of a double).

Each check runs two calls in a row, the second on a smaller grid, so the
second reuses scratch the first filled. Grids cover planes above, inside and
below the sample, planes exactly on interfaces, both transforms the no-alloc
form takes (factored and direct sum) and a grid where scw_synthesize would
take the matrix-core transform.
"""
import numpy as np
import pytest

import workloads as W
from paper_2404_07293_amd import _native as N
from paper_2404_07293_amd._native import ScwError

pytestmark = pytest.mark.gpu

BOUND = {"fp64": 1e-12, "fp32": 1e-6}


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


def _problem(seed=3, nx=12, ny=10, nz=4, U=7, V=5):
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((nz, ny, nx)) + 0.03j * rng.random((nz, ny, nx))
    return W.Problem(n=n.astype(complex), px=0.3, py=0.28, pz=0.2, lam=1.0, U=U, V=V,
                     n_top=1.0, n_bot=1.4 + 0.01j, plane_wave=W.PlaneWave(1, 0, 0.7, 0.2j))


def _compare(torch, sol, grid, precision):
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    shape = (3, grid.fz, grid.fy, grid.fx)
    want = sol.synthesize(grid, precision)
    got = torch.full(shape, float("nan"), dtype=dt, device="cuda")
    sol.synthesize_noalloc(grid, got, precision)
    torch.cuda.synchronize()
    w, g = want.cpu().numpy(), got.cpu().numpy()
    assert np.isfinite(g).all()
    rel = float(np.linalg.norm(g - w) / np.linalg.norm(w))
    elem = float(np.abs(g - w).max() / np.abs(w).max())
    print("noalloc %s grid %s rel-L2 %.3e max-element %.3e" % (
        precision, (grid.fx, grid.fy, grid.fz), rel, elem), flush=True)
    assert rel <= BOUND[precision] and elem <= BOUND[precision], (rel, elem)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_synthesize_two_calls(ctx, precision):
    torch = _torch()
    prob = _problem()
    sol = ctx.solve(prob)
    T = prob.thickness
    big = W.Grid(fx=64, fy=32, fz=24, z_begin=-0.5 * T, z_end=1.5 * T)   # factored transform
    small = W.Grid(fx=20, fy=12, fz=7, z_begin=0.1 * T, z_end=1.2 * T)  # direct / matrix cores
    _compare(torch, sol, big, precision)
    _compare(torch, sol, small, precision)
    sol.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_planes_on_interfaces(ctx, precision):
    torch = _torch()
    prob = _problem(seed=4, nz=5)
    sol = ctx.solve(prob)
    d = prob.pz
    # cell-centred planes at z = l d for l = 0..L: every plane on an interface
    on = W.Grid(fx=16, fy=16, fz=prob.nz + 1, z_begin=-0.5 * d, z_end=(prob.nz + 0.5) * d)
    many = W.Grid(fx=16, fy=8, fz=40, z_begin=0.0, z_end=prob.thickness)  # 8 planes per layer
    _compare(torch, sol, many, precision)
    _compare(torch, sol, on, precision)
    sol.free()


def test_noalloc_working_shape_fp32(ctx):
    """Working-size lateral grid and plane count on a cheaper sample (M = 121)."""
    torch = _torch()
    prob = _problem(seed=5, nx=24, ny=24, nz=8, U=11, V=11)
    sol = ctx.solve(prob)
    g1 = W.Grid(fx=256, fy=256, fz=32, z_begin=0.0, z_end=prob.thickness)
    g2 = W.Grid(fx=128, fy=64, fz=9, z_begin=-0.2, z_end=prob.thickness + 0.3)
    _compare(torch, sol, g1, "fp32")
    _compare(torch, sol, g2, "fp32")
    sol.free()


def test_noalloc_rejects_beyond_limit(ctx):
    torch = _torch()
    prob = _problem(seed=6, nx=16, ny=16, nz=2, U=15, V=15)
    sol = ctx.solve(prob)
    # FP64 spectra alone: fz * 3M * 16 bytes = 20000 * 675 * 16 > 32 MiB
    grid = W.Grid(fx=4, fy=4, fz=20000, z_begin=0.0, z_end=prob.thickness)
    out = torch.empty((3, grid.fz, grid.fy, grid.fx), dtype=torch.complex128, device="cuda")
    with pytest.raises(ScwError) as e:
        sol.synthesize_noalloc(grid, out, "fp64")
    assert e.value.code == -1 and "scratch" in str(e.value)
    with pytest.raises(ScwError) as e:
        sol.synthesize_noalloc(W.Grid(fx=4, fy=4, fz=2, z_begin=0.0, z_end=1.0),
                               torch.empty((3, 2, 4, 4), dtype=torch.complex64, device="cuda"),
                               "bf16x3")
    assert e.value.code == -1
    sol.free()


def test_noalloc_graph_replay(ctx):
    """Captured once, replayed three times with eager work between: every
    replay equals the eager field."""
    torch = _torch()
    prob = _problem(seed=7)
    sol = ctx.solve(prob)
    grid = W.Grid(fx=32, fy=32, fz=12, z_begin=-0.3, z_end=prob.thickness + 0.2)
    want = sol.synthesize(grid, "fp32")
    torch.cuda.synchronize()
    out = torch.zeros((3, grid.fz, grid.fy, grid.fx), dtype=torch.complex64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sol.synthesize_noalloc(grid, out, "fp32")  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sol.synthesize_noalloc(grid, out, "fp32")
    other = W.Grid(fx=16, fy=8, fz=5, z_begin=0.0, z_end=prob.thickness)
    scratch_user = torch.empty((3, 5, 8, 16), dtype=torch.complex64, device="cuda")
    for rep in range(3):
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        rel = float(torch.linalg.norm(out - want) / torch.linalg.norm(want))
        print("replay %d rel %.3e" % (rep, rel), flush=True)
        assert rel <= BOUND["fp32"], (rep, rel)
        sol.synthesize_noalloc(other, scratch_user, "fp32")  # eager call between replays
        torch.cuda.synchronize()
    del g
    sol.free()
