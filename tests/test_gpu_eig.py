"""The batched device eigensolver (scw_eig_batched, SCW_EIG_DEVICE) through
the C ABI.

Direct checks on batches of matrices: the residual ||A X - X diag(w)|| is
at rounding level (<= 1e-12 ||A||), the eigenvalues are the multiset numpy
finds (each within 1e-10 ||A|| of one of numpy's, matched one to one), the
eigenvectors have unit norm, and a repeated eigenvalue still gets a full set
of independent eigenvectors (the TE/TM pairs of a homogeneous layer are
exactly such pairs).

End to end: fields solved with the device eigensolver against the FP64
oracle (sphere workload, a ragged lossy sample, a homogeneous slab whose
Fresnel coefficients are known in closed form), and against the host LAPACK
route on a deeper random sample, all at the FP64 bound 1e-10."""
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


def _match(w, ref):
    """Greedy one-to-one matching of w to ref; returns the largest distance."""
    ref = list(ref)
    worst = 0.0
    for x in sorted(w, key=lambda z: (z.real, z.imag)):
        d = np.abs(np.array(ref) - x)
        i = int(np.argmin(d))
        worst = max(worst, float(d[i]))
        ref.pop(i)
    return worst


def _check(A, w, X, label):
    for b in range(A.shape[0]):
        a = A[b]
        na = np.linalg.norm(a)
        res = np.linalg.norm(a @ X[b] - X[b] * w[b][None, :]) / na
        norms = np.linalg.norm(X[b], axis=0)
        dist = _match(w[b], np.linalg.eigvals(a))
        print("%s[%d] n=%d residual %.2e eigenvalue match %.2e" % (label, b, a.shape[0], res,
                                                                  dist / na), flush=True)
        assert res <= 1e-12
        assert dist <= 1e-10 * na
        assert np.abs(norms - 1).max() <= 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 65, 130, 257])
def test_random_batches(ctx, n):
    torch = _torch()
    rng = np.random.default_rng(n)
    A = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    w, X = ctx.eig_batched(torch.as_tensor(A).cuda())
    torch.cuda.synchronize()
    _check(A, w.cpu().numpy(), X.cpu().numpy(), "random")


def test_real_and_structured_matrices(ctx):
    """A real matrix (eigenvalues in conjugate pairs), an upper triangular
    one (already in Schur form), a diagonal one (every subdiagonal zero from
    the start) and a Jordan-free matrix with eigenvalues of two magnitudes."""
    torch = _torch()
    rng = np.random.default_rng(7)
    n = 40
    real = rng.standard_normal((n, n)).astype(complex)
    tri = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    diag = np.diag(rng.standard_normal(n) + 1j * rng.standard_normal(n))
    S = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    scales = np.diag(np.where(np.arange(n) % 2 == 0, 1e3, 1e-2).astype(complex))
    mixed = S @ scales @ np.linalg.inv(S)
    A = np.stack([real, tri, diag, mixed])
    w, X = ctx.eig_batched(torch.as_tensor(A).cuda())
    torch.cuda.synchronize()
    w, X = w.cpu().numpy(), X.cpu().numpy()
    _check(A[:3], w[:3], X[:3], "structured")
    # the mixed-scale matrix is non-normal: residual relative to ||A|| only
    res = np.linalg.norm(A[3] @ X[3] - X[3] * w[3]) / np.linalg.norm(A[3])
    print("mixed-scale residual %.2e" % res)
    assert res <= 1e-12


def test_repeated_eigenvalues_keep_independent_vectors(ctx):
    torch = _torch()
    rng = np.random.default_rng(3)
    n = 48
    vals = np.repeat(rng.standard_normal(n // 2) + 1j * rng.standard_normal(n // 2), 2)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    A = (Q * vals[None, :]) @ Q.conj().T
    scalar = 1.7 * np.eye(n, dtype=complex)
    w, X = ctx.eig_batched(torch.as_tensor(np.stack([A, scalar])).cuda())
    torch.cuda.synchronize()
    w, X = w.cpu().numpy(), X.cpu().numpy()
    for b, a in enumerate((A, scalar)):
        res = np.linalg.norm(a @ X[b] - X[b] * w[b]) / np.linalg.norm(a)
        smin = np.linalg.svd(X[b], compute_uv=False).min()
        print("repeated[%d] residual %.2e smallest singular value %.3e" % (b, res, smin))
        assert res <= 1e-12
        assert smin >= 1e-3


def test_layer_products_of_a_random_sample(ctx):
    """A C of every layer of a random-field sample at M = 121 (n = 242),
    formed by the oracle's property matrix (Eq. 21)."""
    torch = _torch()
    rng = np.random.default_rng(11)
    n = 1.3 + 0.3 * rng.random((3, 24, 24)) + 0.05j * rng.random((3, 24, 24))
    prob = W.Problem(n=n.astype(complex), px=1 / 6, py=1 / 6, pz=1 / 6, lam=1.0, U=11, V=11)
    u, v = cwt.mode_indices(prob.U, prob.V)
    sx, sy = cwt.spatial_frequencies(u, v, prob.X, prob.Y, prob.lam)
    M = prob.U * prob.V
    mats = []
    for layer in range(prob.nz):
        eps = prob.n[layer] ** 2
        Phi = cwt.toeplitz_from_band(cwt.band_coefficients(eps, prob.U, prob.V), u, v,
                                     prob.U, prob.V)
        Psi = cwt.toeplitz_from_band(cwt.band_coefficients(1.0 / eps, prob.U, prob.V), u, v,
                                     prob.U, prob.V)
        D = cwt.property_matrix(Phi, Psi, sx, sy)
        mats.append(D[:2 * M, 2 * M:] @ D[2 * M:, :2 * M])
    A = np.stack(mats)
    w, X = ctx.eig_batched(torch.as_tensor(A).cuda())
    torch.cuda.synchronize()
    _check(A, w.cpu().numpy(), X.cpu().numpy(), "layer")


def _fields(ctx, prob, grid, eig):
    torch = _torch()
    sol = ctx.solve(prob, eig=eig)
    E = sol.synthesize(grid, "fp64")
    torch.cuda.synchronize()
    info = sol.info()
    out = E.cpu().numpy()
    sol.free()
    return out, info


def test_sphere_fields_match_oracle(ctx):
    prob, grid = W.sphere_config()
    _, _, want = cwt.simulate(prob, grid)
    got, info = _fields(ctx, prob, grid, "device")
    err = rel_l2(got, want)
    print("sphere, device eigensolver: rel-L2 %.3e (eig %.3f s)" % (err, info["eig_seconds"]))
    assert err <= 1e-10


def test_ragged_lossy_fields_match_oracle(ctx):
    rng = np.random.default_rng(1)
    n = 1.3 + 0.3 * rng.random((3, 6, 8)) + 0.04j * rng.random((3, 6, 8))
    prob = W.Problem(n=n.astype(complex), px=0.31, py=0.27, pz=0.19, lam=1.0, U=5, V=3,
                     n_top=1.0, n_bot=1.45 + 0.01j,
                     plane_wave=W.PlaneWave(1, -1, 0.8, 0.3 - 0.2j))
    grid = W.Grid(fx=16, fy=12, fz=10, z_begin=-0.2, z_end=prob.thickness + 0.2)
    _, _, want = cwt.simulate(prob, grid)
    got, _ = _fields(ctx, prob, grid, "device")
    err = rel_l2(got, want)
    print("ragged, device eigensolver: rel-L2 %.3e" % err)
    assert err <= 1e-10


def test_homogeneous_slab_fresnel(ctx):
    """Every eigenvalue of a homogeneous layer is doubly degenerate (TE and
    TM); the transmitted amplitude at normal incidence is the Airy sum."""
    ns, T, lam = 1.5, 0.3, 1.0
    nz = 3
    prob = W.Problem(n=np.full((nz, 4, 4), ns, dtype=complex), px=0.3, py=0.3, pz=T / nz,
                     lam=lam, U=3, V=3, n_top=1.0, n_bot=1.2 + 0.0j,
                     plane_wave=W.PlaneWave(0, 0, 1.0, 0.0))
    sol = ctx.solve(prob, eig="device")
    p_inc, p_ref, p_trn = sol.exterior()
    sol.free()
    p_ref, p_trn = p_ref.ravel(), p_trn.ravel()
    n1, n2, n3 = 1.0, ns, 1.2
    k = 2 * np.pi / lam
    r12, r23 = (n1 - n2) / (n1 + n2), (n2 - n3) / (n2 + n3)
    t12, t23 = 2 * n1 / (n1 + n2), 2 * n2 / (n2 + n3)
    e = np.exp(2j * k * n2 * T)
    t = t12 * t23 * np.exp(1j * k * n2 * T) / (1 + r12 * r23 * e)
    r = (r12 + r23 * e) / (1 + r12 * r23 * e)
    M = 9
    centre = M // 2
    got_t = p_trn.reshape(3, M)[0, centre]
    got_r = p_ref.reshape(3, M)[0, centre]
    print("slab: t %.12f%+.12fj (closed form %.12f%+.12fj)" % (got_t.real, got_t.imag,
                                                               t.real, t.imag))
    assert abs(got_t - t) <= 1e-10
    assert abs(got_r - r) <= 1e-10


def test_deeper_sample_device_matches_host(ctx):
    """A 12-layer random sample at M = 121: device and host eigensolvers give
    the same field to the FP64 bound (their eigenvectors differ by scaling
    and order, which the coefficients absorb)."""
    rng = np.random.default_rng(21)
    n = 1.3 + 0.3 * rng.random((12, 26, 26)) + 0.05j * rng.random((12, 26, 26))
    prob = W.Problem(n=n.astype(complex), px=1 / 6, py=1 / 6, pz=1 / 6, lam=1.0, U=11, V=11,
                     plane_wave=W.PlaneWave(0, 0, 1.0, 0.0))
    grid = W.Grid(fx=32, fy=32, fz=24, z_begin=-0.1, z_end=prob.thickness + 0.1)
    host, ih = _fields(ctx, prob, grid, "host")
    dev, idv = _fields(ctx, prob, grid, "device")
    err = rel_l2(dev, host)
    print("12 layers M=121: device vs host rel-L2 %.3e; eig %.3f s device, %.3f s host" % (
        err, idv["eig_seconds"], ih["eig_seconds"]))
    assert err <= 1e-10


def test_device_eigensolver_rejects_oversized_problem(ctx):
    import paper_2404_07293_amd as P
    prob = W.Problem(n=np.full((1, 8, 8), 1.3, dtype=complex), px=0.2, py=0.2, pz=0.2,
                     lam=1.0, U=33, V=33)  # 2 M = 2178 > 2048
    with pytest.raises(P.ScwError) as e:
        ctx.solve(prob, eig="device")
    assert e.value.code == -1


def test_solve_batch_matches_single_solves(ctx):
    """scw_solve_batch: seven problems of three truncations (their device
    eigendecompositions share one launch per truncation), one with the host
    eigensolver, against the same problems solved one by one on the host
    route, field by field, and one of them against the oracle."""
    torch = _torch()
    rng = np.random.default_rng(31)
    probs = []
    for i, (U, V, nz) in enumerate([(5, 3, 3), (3, 3, 2), (5, 3, 4), (5, 5, 2), (3, 3, 3),
                                     (5, 3, 2), (5, 5, 3)]):
        n = 1.3 + 0.3 * rng.random((nz, 6, 8)) + 0.04j * rng.random((nz, 6, 8))
        probs.append(W.Problem(n=n.astype(complex), px=0.31, py=0.27, pz=0.19, lam=1.0, U=U,
                               V=V, n_top=1.0, n_bot=1.45 + 0.01j,
                               plane_wave=W.PlaneWave(1, 0, 0.8, 0.3j)))
    sols = ctx.solve_batch(probs)
    for i, (pr, sol) in enumerate(zip(probs, sols)):
        grid = W.Grid(fx=16, fy=12, fz=2 * pr.nz + 2, z_begin=-0.1, z_end=pr.thickness + 0.1)
        got = sol.synthesize(grid, "fp64").cpu().numpy()
        ref = ctx.solve(pr)
        want = ref.synthesize(grid, "fp64").cpu().numpy()
        torch.cuda.synchronize()
        err = rel_l2(got, want)
        print("batch problem %d (U=%d V=%d L=%d): rel-L2 vs single host solve %.2e"
              % (i, pr.U, pr.V, pr.nz, err))
        assert err <= 1e-10
        if i == 0:
            _, _, oracle = cwt.simulate(pr, grid)
            assert rel_l2(got, oracle) <= 1e-10
        ref.free()
        sol.free()
