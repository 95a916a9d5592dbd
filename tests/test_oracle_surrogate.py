"""Pins of the FP64 surrogate reference: hand-derived gradients against
central finite differences (h = 1e-6) on 20 random entries of every parameter
array (real and imaginary parts), and the DFT steps against numpy's FFT."""
import numpy as np
import pytest

from oracle import surrogate as S


@pytest.fixture(scope="module")
def setup_net():
    rng = np.random.default_rng(4)
    p = S.init_params(1)
    # larger spectral weights than the initialisation so every branch matters
    for k in range(S.N_LAYERS):
        p["spec%d" % k] *= 4.0
    x = rng.standard_normal((2, S.CIN, S.N, S.N))
    target = rng.standard_normal((2, 3, 15, 15)) + 1j * rng.standard_normal((2, 3, 15, 15))
    out, cache = S.forward(p, x, keep=True)
    g = S.backward(p, cache, out, target)
    return p, x, target, g


@pytest.mark.parametrize("name", [n for n, _, _ in S.param_shapes()])
def test_gradient_matches_finite_differences(setup_net, name):
    p, x, target, g = setup_net
    rng = np.random.default_rng(hash(name) % (2 ** 32))
    a = p[name]
    cplx = np.iscomplexobj(a)
    idx = [tuple(rng.integers(0, s) for s in a.shape) for _ in range(20)]
    h = 1e-6
    for ix in idx:
        for part in ((1.0, 1j) if cplx else (1.0,)):
            q = {k: v.copy() for k, v in p.items()}
            q[name][ix] += h * part
            lp = S.loss(S.forward(q, x), target)
            q[name][ix] -= 2 * h * part
            lm = S.loss(S.forward(q, x), target)
            fd = (lp - lm) / (2 * h)
            an = g[name][ix].real if part == 1.0 else g[name][ix].imag
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (name, ix, part, fd, an)


def test_truncated_dft_matches_fft():
    rng = np.random.default_rng(0)
    h = rng.standard_normal((S.N, S.N))
    fy, fx, iy, ix, hy, hx = S._dft_mats()
    H = fy @ h @ fx
    F = np.fft.fft2(h)
    np.testing.assert_allclose(H, F[np.ix_(S.KY % S.N, S.KX)], atol=1e-11)
    # a band-limited real image is reproduced by the truncated inverse
    G = np.zeros((S.N, S.N), complex)
    keep = np.zeros((S.N, S.N), bool)
    keep[np.ix_(S.KY % S.N, S.KX)] = True
    keep[np.ix_((-S.KY) % S.N, (-S.KX) % S.N)] = True
    G[keep] = F[keep]
    img = np.real(np.fft.ifft2(G))
    np.testing.assert_allclose(np.real(iy @ H @ ix), img, atol=1e-12)


def test_flatten_roundtrip():
    p = S.init_params(3)
    q = S.unflatten(S.flatten(p))
    for k in p:
        np.testing.assert_array_equal(q[k], p[k])
