"""Full-size parity on the 128x128x64 random-field workload (M = 961, 64
layers, 512x512x256 grid): plain FP32 synthesis and the BF16 / FP16 split
forms, in the launch configuration bench.py times, against FP64 oracle values
at 4096 seeded voxels (tests/golden/large_samples.npz, written by
make_large_samples.py), overall and per component."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "large_samples.npz")


@pytest.fixture(scope="module")
def solved():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_07293_amd as P
    prob, grid = W.random_field_config("large")
    print("large: solving 64 layers at M = 961", flush=True)
    ctx = P.Context(0)
    sol = ctx.solve(prob)
    yield ctx, sol, prob, grid
    sol.free()
    ctx.close()


def test_large_exterior_coefficients_match_oracle(solved):
    ctx, sol, prob, grid = solved
    g = np.load(GOLDEN, allow_pickle=False)
    p_inc, p_ref, p_trn = sol.exterior()
    for got, want in ((p_inc, g["p_inc"]), (p_ref, g["p_ref"]), (p_trn, g["p_trn"])):
        err = np.linalg.norm(got.ravel() - want) / np.linalg.norm(want)
        print("exterior rel-L2 %.3e" % err)
        assert err < 1e-9


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_large_field_matches_oracle_samples(solved, precision):
    import torch
    from parity_bounds import check
    ctx, sol, prob, grid = solved
    g = np.load(GOLDEN, allow_pickle=False)
    E = sol.synthesize(grid, precision)
    torch.cuda.synchronize()
    idx = torch.as_tensor(np.stack([g["j"], g["g"], g["f"]]), device=E.device)
    got = E[:, idx[0], idx[1], idx[2]].cpu().numpy()
    check(precision, got, g["E"], "large, %d samples:" % g["E"].shape[1])
    assert bool(torch.isfinite(torch.view_as_real(E)).all())
    del E
