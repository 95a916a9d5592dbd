"""Full-size parity of the FP32 synthesis on the 64x64x32 random-field
workload (M = 441, 256x256x128 grid) in the launch configuration bench.py
times, against FP64 oracle values at 4096 seeded voxels
(tests/golden/working_samples.npz, written by make_working_samples.py)."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "working_samples.npz")


@pytest.fixture(scope="module")
def solved():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_07293_amd as P
    prob, grid = W.random_field_config("working")
    ctx = P.Context(0)
    sol = ctx.solve(prob)
    yield ctx, sol, prob, grid
    sol.free()
    ctx.close()


def test_exterior_coefficients_match_oracle(solved):
    ctx, sol, prob, grid = solved
    g = np.load(GOLDEN, allow_pickle=False)
    p_inc, p_ref, p_trn = sol.exterior()
    for got, want in ((p_inc, g["p_inc"]), (p_ref, g["p_ref"]), (p_trn, g["p_trn"])):
        err = np.linalg.norm(got.ravel() - want) / np.linalg.norm(want)
        print("exterior rel-L2 %.3e" % err)
        assert err < 1e-9


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_field_matches_oracle_samples(solved, precision):
    import torch
    from parity_bounds import check
    ctx, sol, prob, grid = solved
    g = np.load(GOLDEN, allow_pickle=False)
    E = sol.synthesize(grid, precision)
    torch.cuda.synchronize()
    idx = torch.as_tensor(np.stack([g["j"], g["g"], g["f"]]), device=E.device)
    got = E[:, idx[0], idx[1], idx[2]].cpu().numpy()
    check(precision, got, g["E"], "working-size, %d samples:" % g["E"].shape[1])
    # every voxel finite, and the field is not trivially zero anywhere in z
    assert bool(torch.isfinite(torch.view_as_real(E)).all())
    per_plane = E.abs().amax(dim=(0, 2, 3))
    assert bool((per_plane > 0).all())
