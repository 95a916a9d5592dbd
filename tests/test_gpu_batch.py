"""Batched synthesis (one persistent, graph-captured launch over many solved
problems of uneven truncation) against the FP64 oracle and against the
single-problem synthesis, through the C ABI."""
import numpy as np
import pytest

import workloads as W
from oracle import cwt

pytestmark = pytest.mark.gpu
FP32_TOL = 1e-4


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


def small_job(seed, U, V, lam, nz=3, nx=10, ny=9):
    # U <= nx and V <= ny: every spatial frequency of the band is resolved by
    # the voxel grid (otherwise modes alias and the layer problem degenerates)
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((nz, ny, nx)) + 0.03j * rng.random((nz, ny, nx))
    return W.Problem(n=n.astype(complex), px=0.28, py=0.3, pz=0.2, lam=lam, U=U, V=V,
                     n_top=1.0, n_bot=1.2 + 0.0j, plane_wave=W.PlaneWave(0, 0, 1.0, 0.5j))


def well_conditioned(prob):
    st = cwt.setup(prob)
    return min(np.min(np.abs(md.gamma)) / np.max(np.abs(md.gamma)) for md in st.modes) > 1e-3


def test_batch_matches_oracle_and_single_synthesis(ctx):
    torch = _torch()
    specs = [(1, 3, 3, 1.0), (2, 7, 5, 0.9), (3, 5, 7, 1.1), (4, 9, 9, 1.3), (5, 1, 1, 1.0)]
    probs = [small_job(*s) for s in specs]
    assert all(well_conditioned(p) for p in probs)
    T = probs[0].thickness
    below = W.Grid(fx=70, fy=16, fz=3, z_begin=T, z_end=T + 0.9)
    sols = [ctx.solve(p) for p in probs]
    b = ctx.batch(sols, below)
    out = b.launch()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for j, (prob, sol) in enumerate(zip(probs, sols)):
        _, _, want = cwt.simulate(prob, below)
        err = rel_l2(got[j], want)
        print("job %d U=%d V=%d rel-L2 %.3e" % (j, prob.U, prob.V, err))
        assert err <= FP32_TOL
        single = sol.synthesize(below, "fp32").cpu().numpy()
        assert rel_l2(got[j], single) <= 1e-5
    # replaying the graph gives the same field bit for bit
    again = b.launch().cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(again, got)
    # a new output buffer re-captures the graph
    other = torch.zeros_like(out)
    b.launch(out=other)
    torch.cuda.synchronize()
    assert np.array_equal(other.cpu().numpy(), got)


def test_batch_tuner_keeps_a_correct_shape(ctx):
    torch = _torch()
    specs = [(21, 5, 5, 1.0), (22, 9, 7, 0.9), (23, 3, 3, 1.2)]
    probs = [small_job(*s) for s in specs]
    assert all(well_conditioned(p) for p in probs)
    T = max(p.thickness for p in probs)
    grid = W.Grid(fx=40, fy=64, fz=2, z_begin=T + 0.05, z_end=T + 0.6)
    sols = [ctx.solve(p) for p in probs]
    b = ctx.batch(sols, grid)
    base = b.launch().cpu().numpy()
    out = torch.empty_like(b.launch())
    rep = b.tune(out=out, reps=2)
    print(rep)
    assert rep["n_candidates"] >= 8
    assert 0 < rep["best_ms"] <= rep["default_ms"]
    assert rep["radix"] in (2, 4, 8, 16, 32) and rep["blocks_per_cu"] >= 1
    tuned = b.launch(out=out).cpu().numpy()
    torch.cuda.synchronize()
    for j, prob in enumerate(probs):
        _, _, want = cwt.simulate(prob, grid)
        assert rel_l2(tuned[j], want) <= FP32_TOL
        assert rel_l2(tuned[j], base[j]) <= 1e-5
    # a new batch on the same grid starts from the tuned shape
    again = ctx.batch(sols, grid).launch().cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(again, tuned)


@pytest.mark.parametrize("fx,fy", [(64, 64), (40, 32)])
def test_batch_every_radix_matches_oracle(ctx, fx, fy):
    """Every radix of the factored y pass, with the factored x pass (fx = 64,
    one 8-point FFT per row and column group) and with Horner's rule (fx =
    40), on jobs of uneven truncation; each shape against the FP64 oracle."""
    import paper_2404_07293_amd as P
    torch = _torch()
    specs = [(31, 9, 9, 1.0), (32, 3, 5, 0.9), (33, 7, 3, 1.2), (34, 1, 1, 1.1)]
    probs = [small_job(*s) for s in specs]
    assert all(well_conditioned(p) for p in probs)
    T = max(p.thickness for p in probs)
    grid = W.Grid(fx=fx, fy=fy, fz=2, z_begin=T + 0.05, z_end=T + 0.7)
    want = [cwt.simulate(p, grid)[2] for p in probs]
    sols = [ctx.solve(p) for p in probs]
    b = ctx.batch(sols, grid)
    out = torch.empty_like(b.launch())
    radix = 2
    while radix <= min(32, fy):
        for per_cu, chunk in ((1, 1), (4, 16)):
            b.configure(radix, per_cu, chunk)
            got = b.launch(out=out).cpu().numpy()
            torch.cuda.synchronize()
            errs = [rel_l2(got[j], want[j]) for j in range(len(probs))]
            print("fx %d fy %d radix %d blocks/CU %d chunk %d: max rel-L2 %.3e" % (
                fx, fy, radix, per_cu, chunk, max(errs)))
            assert max(errs) <= FP32_TOL
        radix *= 2
    with pytest.raises(P.ScwError):
        b.configure(3, 1, 1)
    with pytest.raises(P.ScwError):
        b.configure(2 * fy, 1, 1)
    with pytest.raises(P.ScwError):
        b.configure(2, 0, 1)
    with pytest.raises(P.ScwError):
        b.configure(2, 1, 0)


def test_batch_above_the_sample(ctx):
    torch = _torch()
    probs = [small_job(7, 5, 3, 1.0), small_job(8, 3, 5, 0.8, nz=2)]
    assert all(well_conditioned(p) for p in probs)
    grid = W.Grid(fx=16, fy=32, fz=2, z_begin=-0.6, z_end=-0.1)
    # jobs of different thickness share an exterior grid above the samples
    sols = [ctx.solve(p) for p in probs]
    got = ctx.batch(sols, grid).launch().cpu().numpy()
    torch.cuda.synchronize()
    for j, prob in enumerate(probs):
        _, _, want = cwt.simulate(prob, grid)
        assert rel_l2(got[j], want) <= FP32_TOL


def test_sweep_job_matches_oracle(ctx):
    # one job of the spectral sweep at its real size (32x32x16 voxels, U = 9)
    torch = _torch()
    jobs = [j for j in W.spectral_sweep_jobs() if j[2] == 9]
    nu, patch, U = jobs[0]
    prob, grid = W.sweep_problem(1650.0, patch, U)
    st = cwt.setup(prob)
    sol_o = cwt.solve(st, "unreduced")
    want = cwt.synthesize(st, sol_o, grid)
    sol = ctx.solve(prob)
    got = ctx.batch([sol, sol], grid).launch().cpu().numpy()
    torch.cuda.synchronize()
    err = rel_l2(got[0], want)
    print("sweep job nu=1650 patch=%d U=%d rel-L2 %.3e" % (patch, U, err))
    assert err <= FP32_TOL
    assert np.array_equal(got[0], got[1])


def test_high_growth_sweep_job_matches_full_system(ctx):
    """Patch 2 (U = 21, 16 layers) at 1000 cm^-1: the connection product's
    growth exponent is about 42, where the paper's reduced route (K of Eq. 27)
    degrades to a 2e-4 error against the full system in FP64 (stored with the
    oracle values; well-conditioned stacks agree to 1e-13). The library's
    default route eliminates from the bottom up with decaying exponentials
    only; its coefficients must match the oracle's full boundary system
    (tests/golden/sweep_hard_job.npz) to 1e-8 and its field to the precision
    of the synthesis."""
    import os
    import paper_2404_07293_amd as P
    torch = _torch()
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "sweep_hard_job.npz"),
                allow_pickle=False)
    patch, U = int(g["patch"]), int(g["U"])
    prob, grid = W.sweep_problem(float(g["nu"]), patch, U)
    sol = ctx.solve(prob)
    info = sol.info()
    print("growth exponent %.1f; reduced route error in the oracle %.2e" % (
        info["growth_exponent"], float(g["reduced_route_rel_l2"])))
    assert info["growth_exponent"] > 30
    assert float(g["reduced_route_rel_l2"]) > 1e-6  # the paper's route degrades here
    p_trn = sol.exterior()[2].ravel()
    assert rel_l2(p_trn, g["p_trn"]) <= 1e-8
    want = g["E"]
    e64 = sol.synthesize(grid, "fp64").cpu().numpy()
    e32 = ctx.batch([sol], grid).launch().cpu().numpy()[0]
    torch.cuda.synchronize()
    print("rel-L2 fp64 %.3e, batched fp32 %.3e" % (rel_l2(e64, want), rel_l2(e32, want)))
    assert rel_l2(e64, want) <= 1e-8
    assert rel_l2(e32, want) <= FP32_TOL
    # the paper's route, forced, reports the lost conditioning (growth
    # exponent above 25) instead of returning degraded coefficients
    for route in ("connection", "connection_device"):
        with pytest.raises(P.ScwError) as e:
            ctx.solve(prob, route=route)
        assert e.value.code == -7  # SCW_EILLCOND


def test_widest_sweep_job_matches_full_system(ctx):
    """Patch 0 (U = 25, M = 625, 16 layers; the 49-wide band wraps on the
    32-voxel patch) at 1000 cm^-1, growth exponent about 51: the oracle's full
    boundary system (43,750 unknowns, banded LU; tests/golden/sweep_u25_job.npz)
    against the library's default route, and the batched launch's field on it,
    alone and next to a job of the smallest truncation."""
    import os
    torch = _torch()
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "sweep_u25_job.npz"),
                allow_pickle=False)
    patch, U = int(g["patch"]), int(g["U"])
    prob, grid = W.sweep_problem(float(g["nu"]), patch, U)
    sol = ctx.solve(prob)
    info = sol.info()
    print("U=25 job: growth exponent %.1f, reduced route error in the oracle %.2e" % (
        info["growth_exponent"], float(g["reduced_route_rel_l2"])))
    assert info["growth_exponent"] > 40
    p_trn = sol.exterior()[2].ravel()
    assert rel_l2(p_trn, g["p_trn"]) <= 1e-8
    want = g["E"]
    e64 = sol.synthesize(grid, "fp64").cpu().numpy()
    small = ctx.solve(small_job(9, 3, 3, 1.0))
    eb = ctx.batch([small, sol, sol], grid).launch().cpu().numpy()
    torch.cuda.synchronize()
    print("rel-L2 fp64 %.3e, batched fp32 %.3e / %.3e" % (
        rel_l2(e64, want), rel_l2(eb[1], want), rel_l2(eb[2], want)))
    assert rel_l2(e64, want) <= 1e-8
    assert rel_l2(eb[1], want) <= FP32_TOL
    assert np.array_equal(eb[1], eb[2])
    small.free()
    sol.free()


def test_batch_rejects_interior_grid(ctx):
    import paper_2404_07293_amd as P
    sol = ctx.solve(small_job(9, 3, 3, 1.0))
    with pytest.raises(P.ScwError):
        ctx.batch([sol], W.Grid(fx=8, fy=8, fz=2, z_begin=0.0, z_end=0.6))
    with pytest.raises(P.ScwError):
        ctx.batch([sol], W.Grid(fx=8, fy=12, fz=2, z_begin=0.7, z_end=0.9))
