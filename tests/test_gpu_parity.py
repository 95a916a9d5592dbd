"""GPU parity of the HIP library against the FP64 oracle, through the C ABI.

Tolerances, checked by `field_check` on every synthesised field:
  FP64 synthesis  rel-L2 <= 1e-10 (both sides are FP64; the setups differ in
                  formulation: 2M product eigenproblem and stable elimination
                  vs. 4M geev and the full system)
  FP32 and the split forms: the bounds of SMALL_BOUNDS below, a few times the
                  errors these problems measure, far under the 1e-4 target:
                  total rel-L2, each component's error against the field's
                  norm (a component can vanish, e.g. E_y under TM incidence),
                  and the largest element error against the largest element.
"""
import numpy as np
import pytest

import workloads as W
from oracle import cwt
from paper_2404_07293_amd._native import ScwError

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-6

# (total rel-L2, per component against the field's norm, largest element) for
# the small problems of this file. FP32: complex64 storage of the coefficients
# and of P (unit roundoff 6e-8) and sums of up to 2M + U + V terms give about
# 1e-7 to 1e-6; the split forms add the lo * lo term and the rounding of lo
# (2^-16 of the operands for bf16, 2^-22 for fp16) over the K <= 2V terms of
# the transform.
# Measured on these problems: FP32 at most 2.2e-7 total and 4.6e-7 largest
# element; BF16x3 4.0e-6 and 1.1e-5; FP16x3 1.8e-7 and 4.4e-7; FP64 2e-14.
SMALL_BOUNDS = {
    "fp64": (1e-10, 1e-10, 1e-10),
    "fp32": (1e-6, 1e-6, 2e-6),
    "bf16x3": (2e-5, 2e-5, 6e-5),
    "fp16x3": (1e-6, 1e-6, 2e-6),
}


def field_check(precision, got, want, label=""):
    """Assert the bounds of SMALL_BOUNDS; returns (total, per component,
    element) and prints them."""
    norm = np.linalg.norm(want)
    total = float(np.linalg.norm(got - want) / norm)
    per = [float(np.linalg.norm(got[c] - want[c]) / norm) for c in range(got.shape[0])]
    elem = float(np.abs(got - want).max() / np.abs(want).max())
    print("%s %s rel-L2 %.3e per component %s max-element %.3e" % (
        label, precision, total, ["%.2e" % x for x in per], elem), flush=True)
    bt, bc, be = SMALL_BOUNDS[precision]
    assert total <= bt, (label, precision, total)
    assert max(per) <= bc, (label, precision, per)
    assert elem <= be, (label, precision, elem)
    return total, per, elem


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


def run(ctx, prob, grid, precision="fp64", route="stable"):
    torch = _torch()
    sol = ctx.solve(prob, route)
    E = sol.synthesize(grid, precision)
    torch.cuda.synchronize()
    return sol, E.cpu().numpy()


def ragged_problem(seed=1, nx=8, ny=6, nz=3, U=5, V=3, lossy=True, pw=(1, -1)):
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((nz, ny, nx))
    if lossy:
        n = n + 0.04j * rng.random((nz, ny, nx))
    return W.Problem(n=n.astype(complex), px=0.31, py=0.27, pz=0.19, lam=1.0, U=U, V=V,
                     n_top=1.0, n_bot=1.45 + 0.01j,
                     plane_wave=W.PlaneWave(pw[0], pw[1], 0.8, 0.3 - 0.2j))


def test_sphere_fp64_matches_oracle(ctx):
    prob, grid = W.sphere_config()
    _, _, want = cwt.simulate(prob, grid)
    _, got = run(ctx, prob, grid, "fp64")
    assert got.shape == want.shape
    field_check("fp64", got, want, "sphere")
    for c in range(3):
        assert rel_l2(got[c], want[c]) <= 10 * FP64_TOL


def test_sphere_fp32_matches_oracle(ctx):
    prob, grid = W.sphere_config()
    _, _, want = cwt.simulate(prob, grid)
    _, got = run(ctx, prob, grid, "fp32")
    field_check("fp32", got, want, "sphere")


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_planes_above_inside_below_ragged_grid(ctx, precision, tol):
    prob = ragged_problem()
    T = prob.thickness
    grid = W.Grid(fx=13, fy=7, fz=11, z_begin=-0.4, z_end=T + 0.4)
    _, _, want = cwt.simulate(prob, grid)
    _, got = run(ctx, prob, grid, precision)
    field_check(precision, got, want, "ragged")


def test_connection_route_matches_oracle(ctx):
    prob = ragged_problem(seed=2)
    grid = W.Grid(fx=9, fy=10, fz=6, z_begin=-0.2, z_end=prob.thickness + 0.2)
    _, _, want = cwt.simulate(prob, grid)
    sol, got = run(ctx, prob, grid, "fp64", route="connection")
    assert rel_l2(got, want) <= FP64_TOL
    assert sol.info()["connection_rcond"] > 0


def test_exterior_coefficients_match_oracle(ctx):
    prob = ragged_problem(seed=3, U=3, V=5)
    st = cwt.setup(prob)
    ref = cwt.solve(st)
    sol = ctx.solve(prob)
    p_inc, p_ref, p_trn = sol.exterior()
    M = st.M
    np.testing.assert_allclose(p_inc.ravel(), st.p_inc, atol=1e-13)
    assert rel_l2(p_ref.ravel(), ref.p_ref) < 1e-11
    assert rel_l2(p_trn.ravel(), ref.p_trn) < 1e-11
    assert p_ref.shape == (3, M)


def test_image_incidence_matches_oracle(ctx):
    prob = ragged_problem(seed=4)
    rng = np.random.default_rng(9)
    prob.inc_ex = rng.standard_normal((5, 9)) + 1j * rng.standard_normal((5, 9))
    prob.inc_ey = rng.standard_normal((5, 9)) + 1j * rng.standard_normal((5, 9))
    grid = W.Grid(fx=16, fy=12, fz=5, z_begin=0.0, z_end=prob.thickness)
    _, _, want = cwt.simulate(prob, grid)
    _, got = run(ctx, prob, grid, "fp64")
    assert rel_l2(got, want) <= FP64_TOL


def test_many_planes_per_layer(ctx):
    # 23 planes over 2 layers: tasks of 8 planes plus ragged remainders
    prob = ragged_problem(seed=5, nz=2)
    grid = W.Grid(fx=8, fy=8, fz=23, z_begin=0.0, z_end=prob.thickness)
    _, _, want = cwt.simulate(prob, grid)
    for precision in ("fp64", "fp32"):
        _, got = run(ctx, prob, grid, precision)
        field_check(precision, got, want, "23 planes")


def test_single_frequency(ctx):
    prob = ragged_problem(seed=6, U=1, V=1, pw=(0, 0))
    grid = W.Grid(fx=4, fy=4, fz=6, z_begin=-0.1, z_end=prob.thickness + 0.1)
    _, _, want = cwt.simulate(prob, grid)
    _, got = run(ctx, prob, grid, "fp64")
    assert rel_l2(got, want) <= FP64_TOL


def test_lossless_energy_balance_from_library(ctx):
    prob = ragged_problem(seed=7, lossy=False)
    prob.n_bot = 1.5 + 0j
    sol = ctx.solve(prob)
    st = cwt.setup(prob)   # only for s_x, s_y, s_z of the modes
    p_inc, p_ref, p_trn = sol.exterior()
    fi = cwt.z_flux(p_inc, cwt.h_coefficients(p_inc, st.sx, st.sy, st.sz_top))
    fr = -cwt.z_flux(p_ref, cwt.h_coefficients(p_ref, st.sx, st.sy, -st.sz_top))
    ft = cwt.z_flux(p_trn, cwt.h_coefficients(p_trn, st.sx, st.sy, st.sz_bot))
    assert abs(fi - fr - ft) < 1e-11 * fi


def test_fp32_is_deterministic(ctx):
    torch = _torch()
    prob, grid = W.sphere_config()
    sol = ctx.solve(prob)
    a = sol.synthesize(grid, "fp32").clone()
    b = sol.synthesize(grid, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_error_codes(ctx):
    import paper_2404_07293_amd as P
    prob = ragged_problem()
    prob.U = 4
    with pytest.raises(P.ScwError) as e:
        ctx.solve(prob)
    assert e.value.code == -1
    # X = 2 wavelengths puts (u, v) = (2, 0) at |s| = 1 = n_top: grazing
    n = np.full((1, 4, 4), 1.5 + 0j)
    prob = W.Problem(n=n, px=0.5, py=0.5, pz=0.2, lam=1.0, U=5, V=1)
    with pytest.raises(P.ScwError) as e:
        ctx.solve(prob)
    assert e.value.code == -5
    sol = ctx.solve(ragged_problem())
    with pytest.raises(P.ScwError):
        sol.synthesize(W.Grid(fx=0, fy=4, fz=4, z_begin=0, z_end=1), "fp32")
    with pytest.raises(P.ScwError):
        sol.synthesize(W.Grid(fx=4, fy=4, fz=4, z_begin=1, z_end=0), "fp32")


# Split-precision inverse transform on the matrix cores. Each operand is split
# x = hi + lo and three products are accumulated in FP32; the dropped lo*lo
# term and the rounding of lo leave a relative error per product of about
# 2^-16 (bf16) or 2^-22 (fp16) of the operand magnitudes. Over the K <= 2V
# terms of one output and the spread of magnitudes in a field, the bounds are:
BF16X3_TOL = SMALL_BOUNDS["bf16x3"][0]
FP16X3_TOL = SMALL_BOUNDS["fp16x3"][0]


@pytest.mark.parametrize("precision,tol", [("bf16x3", BF16X3_TOL), ("fp16x3", FP16X3_TOL),
                                           ("fp32", FP32_TOL)])
def test_split_precision_matches_oracle(ctx, precision, tol):
    for prob, grid in (W.sphere_config(),
                       (ragged_problem(seed=11),
                        W.Grid(fx=13, fy=7, fz=9, z_begin=-0.3, z_end=0.9))):
        _, _, want = cwt.simulate(prob, grid)
        _, got = run(ctx, prob, grid, precision)
        field_check(precision, got, want, "split form")


# every kernel configuration the FP32 and FP64 paths can take: the three
# inverse transforms (factored FFT y pass at each radix, matrix-core y pass at
# several plane tilings, direct Horner sums at several row tilings) and the
# modal-sum row blockings
CONFIGS = ([("fp32", dict(transform="fft", fft_radix=p)) for p in (2, 4, 8, 16, 32)]
           + [("fp32", dict(transform="fft", fft_radix=p, tiles=32)) for p in (4, 16)]
           + [("fp64", dict(transform="fft", fft_radix=8, tiles=32))]
           + [("fp32", dict(transform="mfma", tiles=t)) for t in (0, 1, 3)]
           + [("fp32", dict(transform="direct", tiles=t)) for t in (0, 1, 5)]
           + [("fp32", dict(modal_rows=r)) for r in (2, 4, 8, 16)]
           + [("fp64", dict(transform="fft", fft_radix=p)) for p in (4, 32)]
           + [("fp64", dict(transform="direct", tiles=t)) for t in (0, 2)])


@pytest.mark.parametrize("precision,cfg", CONFIGS)
def test_kernel_configurations_match_oracle(ctx, precision, cfg):
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    for prob, grid in (W.sphere_config(),
                       (ragged_problem(seed=12),
                        W.Grid(fx=24, fy=64, fz=7, z_begin=-0.2, z_end=0.8)),
                       (ragged_problem(seed=13, U=7, V=5),
                        W.Grid(fx=70, fy=512, fz=3, z_begin=0.1, z_end=0.5))):
        if cfg.get("fft_radix", 0) > grid.fy:
            continue
        sol = ctx.solve(prob)
        sol.configure(**cfg)
        P = cfg.get("fft_radix", 0)
        eb = 16 if precision == "fp64" else 8
        if P and (prob.U * prob.V + 32 * 64 + 32 * (grid.fy // P)) * eb > 64 * 1024:
            # the factored transform's tables must fit in 64 KB of LDS
            with pytest.raises(ScwError) as e:
                sol.synthesize(grid, precision)
            assert e.value.code == -1
            continue
        _, _, want = cwt.simulate(prob, grid)
        got = sol.synthesize(grid, precision).cpu().numpy()
        field_check(precision, got, want, "%s fy=%d" % (cfg, grid.fy))


def test_unsupported_configurations_are_rejected(ctx):
    prob, grid = W.sphere_config(out=16)
    sol = ctx.solve(prob)
    bad = [("fp64", dict(transform="mfma")),
           ("bf16x3", dict(transform="fft")),
           ("fp16x3", dict(transform="direct")),
           ("fp32", dict(modal_rows=3)),
           ("fp32", dict(transform="fft", fft_radix=64)),
           ("fp32", dict(transform="fft", fft_radix=12)),
           ("fp32", dict(transform="fft", fft_radix=8, tiles=48))]
    for precision, cfg in bad:
        sol.configure(**cfg)
        with pytest.raises(ScwError) as e:
            sol.synthesize(grid, precision)
        assert e.value.code == -1, (precision, cfg)
    sol.configure()
    sol.synthesize(grid, "fp32")
    # a factored transform needs fy a power of two
    sol.configure(transform="fft")
    with pytest.raises(ScwError):
        sol.synthesize(W.Grid(fx=16, fy=12, fz=4, z_begin=0.0, z_end=1.0), "fp32")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
def test_autotuner_keeps_a_correct_and_no_slower_configuration(ctx, precision):
    torch = _torch()
    tol = {"fp64": FP64_TOL, "fp32": FP32_TOL, "bf16x3": BF16X3_TOL}[precision]
    prob = ragged_problem(seed=14, nx=8, ny=10, U=7, V=9)
    grid = W.Grid(fx=96, fy=128, fz=12, z_begin=-0.2, z_end=1.1)
    _, _, want = cwt.simulate(prob, grid)
    sol = ctx.solve(prob)
    out = sol.synthesize(grid, precision)
    rep = sol.tune(grid, precision, out=out, reps=3)
    print(precision, rep)
    assert rep["n_candidates"] >= 2
    assert 0 < rep["best_ms"] <= rep["default_ms"]
    field_check(precision, out.cpu().numpy(), want, "tuned")
    if precision == "bf16x3":
        assert rep["transform"] == "mfma"
    # a second solution of the same shape takes the tuned configuration and
    # computes the same field
    sol2 = ctx.solve(prob)
    got = sol2.synthesize(grid, precision)
    torch.cuda.synchronize()
    assert torch.equal(got, sol.synthesize(grid, precision))


def test_synthesis_replays_in_a_captured_graph(ctx):
    """scw_synthesize enqueues plain kernels on the caller's stream, so once
    its plan exists (first call) it can be captured in a HIP graph: every
    replay, with eager work on the GPU in between, gives the eager field."""
    torch = _torch()
    prob = ragged_problem(seed=21, nx=8, ny=10, U=7, V=9)
    grid = W.Grid(fx=48, fy=64, fz=10, z_begin=-0.3, z_end=1.0)
    sol = ctx.solve(prob)
    eager = sol.synthesize(grid, "fp32")
    torch.cuda.synchronize()
    want = eager.clone()
    out = torch.zeros_like(eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sol.synthesize(grid, "fp32", out=out)  # plan already built: no host sync
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    out.zero_()
    with torch.cuda.graph(g):
        sol.synthesize(grid, "fp32", out=out)
    for k in range(3):
        out.zero_()
        junk = torch.randn(1 << 20, device="cuda") * k  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), k
        del junk


def _film_stack():
    ns = [1.3, 1.7 + 0.02j, 1.5]
    n = np.stack([np.full((4, 4), complex(x)) for x in ns])
    return W.Problem(n=n, px=0.6, py=0.6, pz=0.25, lam=1.0, U=3, V=3, n_top=1.0,
                     n_bot=1.2 + 0.01j, plane_wave=W.PlaneWave(1, 0, 1.0, 0.0))


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_planes_exactly_on_interfaces_match_oracle(ctx, precision, tol):
    """One plane per interface, z_j = j d exactly (pitch 0.25, binary-exact):
    z0 belongs to layer 1, z_l to layer l+1 and z_L to the lower half-space,
    where E_z differs from the layer above by eps_above / eps_below."""
    for prob in (W.sphere_config()[0], _film_stack()):
        L, d = prob.nz, prob.pz
        grid = W.Grid(fx=16, fy=8, fz=L + 1, z_begin=-d / 2, z_end=(L + 0.5) * d)
        assert np.array_equal(grid.z_planes(), np.arange(L + 1) * d)
        st = cwt.setup(prob)
        sol_o = cwt.solve(st)
        want = cwt.synthesize(st, sol_o, grid)
        _, got = run(ctx, prob, grid, precision)
        # each component's error against the whole field's norm: under TM
        # incidence on the film stack E_y vanishes identically, so its own
        # norm is rounding noise on both sides
        norm = np.linalg.norm(want)
        per = [float(np.linalg.norm(got[c] - want[c]) / norm) for c in range(3)]
        print("interfaces %s per component %s" % (precision, ["%.2e" % x for x in per]))
        assert rel_l2(got, want) <= tol
        assert max(per) <= tol
        # the E_z of the layer above would be off by the index ratio
        above = np.stack([cwt.plane_coefficients(st, sol_o, z - 1e-9)[2]
                          for z in grid.z_planes()])
        assert np.abs(above - np.stack([cwt.plane_coefficients(st, sol_o, z)[2]
                                        for z in grid.z_planes()])).max() > 1e-3


def test_defective_layer_is_rejected(ctx):
    """A homogeneous layer with eps = s_x^2 on a lattice mode (n = 0.5, X = 2
    lambda, u = 1): gamma = 0 exactly, D defective -> SCW_EDEFECTIVE."""
    import paper_2404_07293_amd as P
    n = np.full((2, 1, 4), 0.5 + 0j)
    prob = W.Problem(n=n, px=0.5, py=0.5, pz=0.2, lam=1.0, U=3, V=1)
    for route in ("stable", "connection", "stable_device"):
        with pytest.raises(P.ScwError) as e:
            ctx.solve(prob, route)
        assert e.value.code == -6, route
    prob.n = np.full((2, 1, 4), 0.6 + 0j)
    ctx.solve(prob)


def test_captured_synthesis_survives_other_grids_and_configurations(ctx):
    """A graph captured with one grid keeps its plan: synthesizing other grids,
    precisions and kernel configurations of the same solution, and tuning it,
    builds new plans and leaves the captured one intact."""
    torch = _torch()
    prob = ragged_problem(seed=22, nx=8, ny=10, U=7, V=9)
    grid_a = W.Grid(fx=48, fy=64, fz=10, z_begin=-0.3, z_end=1.0)
    grid_b = W.Grid(fx=96, fy=128, fz=31, z_begin=-0.5, z_end=1.3)
    sol = ctx.solve(prob)
    want = sol.synthesize(grid_a, "fp32").clone()
    torch.cuda.synchronize()
    out = torch.zeros_like(want)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sol.synthesize(grid_a, "fp32", out=out)
    other = [lambda: sol.synthesize(grid_b, "fp32"),
             lambda: sol.synthesize(grid_b, "bf16x3"),
             lambda: sol.synthesize(grid_a, "fp64"),
             lambda: (sol.configure(transform="direct"), sol.synthesize(grid_a, "fp32")),
             lambda: (sol.configure(), sol.tune(grid_b, "fp32", reps=1))]
    for k, fn in enumerate(other):
        fn()
        torch.cuda.synchronize()
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_synthesis_stages_compose_to_the_full_synthesis(ctx, precision):
    """scw_synthesize_stages: the modal sum, the exterior spectra and the
    transform run as separate calls (in any grouping) give the field of one
    scw_synthesize call bit for bit, and a transform-only call repeats it."""
    torch = _torch()
    prob = ragged_problem(seed=23)
    grid = W.Grid(fx=13, fy=16, fz=9, z_begin=-0.3, z_end=prob.thickness + 0.3)
    sol = ctx.solve(prob)
    full = sol.synthesize(grid, precision).clone()
    a = sol.synthesize_stages(grid, ["modal", "exterior"], precision=precision)
    a = sol.synthesize_stages(grid, "transform", out=a, precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(a, full)
    sol.synthesize_stages(grid, "modal", precision=precision)
    sol.synthesize_stages(grid, "exterior", precision=precision)
    b = sol.synthesize_stages(grid, "transform", precision=precision)
    c = sol.synthesize_stages(grid, "transform", precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(b, full) and torch.equal(c, full)
    with pytest.raises(ScwError) as e:
        sol.synthesize_stages(grid, [], precision=precision)
    assert e.value.code == -1
