"""Large samples through the C ABI: the periodic display of one solution
(scw_synthesize_tiled, Sec. 4.6) and a sample composed of patches
(scw_synthesize_composed, Sec. 1), against the oracle's tiled and composed
fields (oracle/cwt.py, pinned in tests/test_oracle_tiling.py). Bounds: FP64
1e-10 and FP32 1e-5 relative L2 (the plain synthesis bounds); identical
patches compose to exactly the tiled field."""
import numpy as np
import pytest

import workloads as W
from oracle import cwt

pytestmark = pytest.mark.gpu

BOUND = {"fp64": 1e-10, "fp32": 1e-5}


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


def _patch(seed, U=5, V=3, nx=7, ny=6, px=0.3, n_in=1.45 + 0.02j):
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((2, ny, nx)) + 0.03j * rng.random((2, ny, nx))
    n[:, 2:4, 2:5] = n_in
    return W.Problem(n=n.astype(complex), px=px, py=0.32, pz=0.21, lam=1.0, U=U, V=V,
                     n_top=1.0, n_bot=1.3 + 0.0j, plane_wave=W.PlaneWave(0, 0, 0.9, 0.2j))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tiled_field_matches_oracle(ctx, precision):
    torch = _torch()
    prob = _patch(1)
    st = cwt.setup(prob)
    want = cwt.tiled(st, cwt.solve(st), W.Grid(fx=16, fy=8, fz=6, z_begin=-0.2,
                                                z_end=prob.thickness + 0.3), 3, 2)
    sol = ctx.solve(prob)
    grid = W.Grid(fx=16, fy=8, fz=6, z_begin=-0.2, z_end=prob.thickness + 0.3)
    got = sol.synthesize_tiled(grid, 3, 2, precision).cpu().numpy()
    torch.cuda.synchronize()
    err = rel_l2(got, want)
    print("tiled 3x2 %s: rel-L2 %.3e" % (precision, err))
    assert err <= BOUND[precision]
    sol.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_composed_patches_match_oracle(ctx, precision):
    """A 2 x 2 mosaic of four different patches: different samples, two
    truncations and two lateral periods."""
    torch = _torch()
    probs = [_patch(2), _patch(3, U=3, V=5), _patch(4, px=0.28), _patch(5, U=5, V=5)]
    grid = W.Grid(fx=12, fy=10, fz=5, z_begin=-0.1, z_end=0.6)
    parts = []
    for pr in probs:
        st = cwt.setup(pr)
        parts.append((st, cwt.solve(st)))
    want = cwt.compose(parts, 2, 2, grid)
    sols = [ctx.solve(pr) for pr in probs]
    got = ctx.synthesize_composed(sols, 2, 2, grid, precision).cpu().numpy()
    torch.cuda.synchronize()
    err = rel_l2(got, want)
    print("composed 2x2 %s: rel-L2 %.3e" % (precision, err))
    assert err <= BOUND[precision]
    for s in sols:
        s.free()


def test_identical_patches_compose_to_the_tiled_field(ctx):
    torch = _torch()
    prob = _patch(6)
    sol = ctx.solve(prob)
    grid = W.Grid(fx=16, fy=16, fz=4, z_begin=0.0, z_end=prob.thickness)  # factored transform
    tiled = sol.synthesize_tiled(grid, 3, 2, "fp32")
    comp = ctx.synthesize_composed([sol] * 6, 3, 2, grid, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(tiled, comp)
    plain = sol.synthesize(grid, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(tiled[:, :, 16:32, 32:48], plain)
    sol.free()


def test_tiling_rejects_bad_counts(ctx):
    import paper_2404_07293_amd as P
    sol = ctx.solve(_patch(7))
    grid = W.Grid(fx=8, fy=8, fz=2, z_begin=0.0, z_end=0.4)
    with pytest.raises(P.ScwError):
        sol.synthesize_tiled(grid, 0, 1)
    sol.free()
