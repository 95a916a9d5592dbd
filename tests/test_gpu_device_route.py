"""The boundary solve on the device in FP64 (rocSOLVER LU, rocBLAS GEMM): the
stable elimination (SCW_ROUTE_STABLE_DEVICE) and the connection route's layer
matrices, K product and alpha recursion (SCW_ROUTE_CONNECTION_DEVICE), against
the FP64 oracle on small lossy samples, with one and with several
illuminations, and against the host elimination on the 64x64x32 working
sample (same solution to rounding)."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import cwt

pytestmark = pytest.mark.gpu


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


def problem(seed, U=5, V=3, nz=4):
    rng = np.random.default_rng(seed)
    n = 1.3 + 0.3 * rng.random((nz, 6, 8)) + 0.05j * rng.random((nz, 6, 8))
    return W.Problem(n=n.astype(complex), px=0.31, py=0.27, pz=0.23, lam=1.0, U=U, V=V,
                     n_top=1.0, n_bot=1.45 + 0.01j,
                     plane_wave=W.PlaneWave(1, -1, 0.8, 0.3 - 0.2j))


ROUTES = ["stable_device", "connection_device"]


@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("seed,U,V", [(1, 5, 3), (2, 7, 5)])
def test_device_route_matches_oracle(ctx, route, seed, U, V):
    torch = _torch()
    prob = problem(seed, U, V)
    st = cwt.setup(prob)
    ref = cwt.solve(st)
    grid = W.Grid(fx=10, fy=8, fz=11, z_begin=-0.3, z_end=prob.thickness + 0.3)
    sol = ctx.solve(prob, route=route)
    E = sol.synthesize(grid, "fp64").cpu().numpy()
    torch.cuda.synchronize()
    err = rel_l2(E, cwt.synthesize(st, ref, grid))
    p_inc, p_ref, p_trn = sol.exterior()
    e_ref = rel_l2(p_ref.ravel(), ref.p_ref)
    e_trn = rel_l2(p_trn.ravel(), ref.p_trn)
    print("%s U=%d V=%d: field rel-L2 %.3e, p_ref %.3e, p_trn %.3e"
          % (route, U, V, err, e_ref, e_trn))
    assert err <= 1e-10 and e_ref <= 1e-10 and e_trn <= 1e-10


@pytest.mark.parametrize("route", ROUTES)
def test_device_route_with_illuminations(ctx, route):
    torch = _torch()
    prob = problem(3)
    rng = np.random.default_rng(4)
    ws = [W.PlaneWave(int(rng.integers(-2, 3)), int(rng.integers(-1, 2)),
                      complex(rng.standard_normal() + 1j * rng.standard_normal()),
                      complex(rng.standard_normal())) for _ in range(5)]
    grid = W.Grid(fx=8, fy=8, fz=9, z_begin=-0.2, z_end=prob.thickness + 0.2)
    sol = ctx.solve(prob, route=route, waves=ws)
    got = sol.synthesize_illuminations(grid).cpu().numpy()
    torch.cuda.synchronize()
    errs = []
    for k, w in enumerate(ws):
        st = cwt.setup(dataclasses.replace(prob, plane_wave=w))
        errs.append(rel_l2(got[k], cwt.synthesize(st, cwt.solve(st), grid)))
    print("%s, 5 illuminations: max rel-L2 %.3e" % (route, max(errs)))
    assert max(errs) <= 1e-4


@pytest.fixture(scope="module")
def working_host(ctx):
    prob, grid = W.random_field_config("working")
    return prob, grid, ctx.solve(prob, route="stable")


@pytest.mark.parametrize("route", ROUTES)
def test_device_route_agrees_with_host_route_at_working_size(ctx, working_host, route):
    torch = _torch()
    prob, grid, host = working_host
    dev = ctx.solve(prob, route=route)
    hi, di = host.info(), dev.info()
    hx, dx = host.exterior(), dev.exterior()
    e = [rel_l2(d.ravel(), h.ravel()) for d, h in zip(dx[1:], hx[1:])]
    Eh = host.synthesize(grid, "fp32")
    Ed = dev.synthesize(grid, "fp32")
    torch.cuda.synchronize()
    ef = float(torch.linalg.vector_norm(Ed - Eh) / torch.linalg.vector_norm(Eh))
    print("working sample: boundary solve %.2f s on the host (stable), %.2f s on the device "
          "(%s; setup %.2f s vs %.2f s); p_ref %.2e, p_trn %.2e, field %.2e"
          % (hi["boundary_seconds"], di["boundary_seconds"], route, hi["setup_seconds"],
             di["setup_seconds"], e[0], e[1], ef))
    dev.free()
    assert e[0] <= 1e-9 and e[1] <= 1e-9
    assert ef <= 1e-6


def test_device_connection_route_reports_its_condition(ctx):
    """The device connection route computes the 1-norm condition of its 6M x 6M
    system exactly (norm of the explicit inverse); the host route estimates it
    with zgecon, whose estimate of the inverse's norm is a lower bound that is
    usually within a small factor. Both must describe the same system."""
    prob = problem(3, U=7, V=5)
    host = ctx.solve(prob, route="connection")
    dev = ctx.solve(prob, route="connection_device")
    rh, rd = host.info()["connection_rcond"], dev.info()["connection_rcond"]
    hx, dx = host.exterior(), dev.exterior()
    err = rel_l2(dx[2].ravel(), hx[2].ravel())
    print("connection rcond: host estimate %.3e, device exact %.3e; p_trn rel diff %.2e"
          % (rh, rd, err))
    assert 0 < rd <= rh * (1 + 1e-6) and rd >= rh / 10
    assert err <= 1e-12
    host.free()
    dev.free()
