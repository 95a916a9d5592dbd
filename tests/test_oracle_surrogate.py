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


def test_bf16_rounding_follows_the_format():
    # bfloat16 keeps 8 significand bits: spacing 2^-7 on [1, 2)
    one = 1.0
    cases = [(one, one),
             (one + 2.0 ** -9, one),                      # below half a step: down
             (one + 2.0 ** -8, one),                      # tie: to even (1.0)
             (one + 3 * 2.0 ** -8, one + 2.0 ** -6),      # tie: to even (1 + 2^-6)
             (one + 2.0 ** -8 + 2.0 ** -20, one + 2.0 ** -7),  # above the tie: up
             (-3.140625, -3.140625),                      # representable
             (2.0 ** -130, 2.0 ** -130)]                  # subnormal, representable
    for x, want in cases:
        assert S.to_bf16(np.array([x]))[0] == want, (x, want)
    z = S.to_bf16(np.array([1.0 + 2.0 ** -9 + 1j * (one + 2.0 ** -6)]))[0]
    assert z == 1.0 + 1j * (one + 2.0 ** -6)
    # relative rounding error never exceeds the unit roundoff u = 2^-8
    rng = np.random.default_rng(1)
    a = rng.standard_normal(10000) * 10.0 ** rng.uniform(-20, 20, 10000)
    assert np.max(np.abs(S.to_bf16(a) - a) / np.abs(a)) <= 2.0 ** -8


def test_bf16_forward_stays_near_the_exact_network():
    # the rounded-operand network differs from the exact one by a few bf16
    # unit roundoffs (u = 2^-8) along its chain of products
    rng = np.random.default_rng(6)
    p = S.init_params(2)
    x = rng.standard_normal((1, S.CIN, S.N, S.N))
    a = S.forward(p, x)
    b = S.forward(p, x, bf16=True)
    err = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert 2.0 ** -13 < err < 10 * 2.0 ** -8
