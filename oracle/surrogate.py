"""FP64 CPU reference of the spectral-convolution surrogate (test infrastructure).

TEST INFRASTRUCTURE: used by the tests to check the HIP surrogate's forward
pass and gradients; shares no code with the library.

The surrogate maps a complex-index patch (8 layers x 32 x 32 voxels) to the
transmitted plane-wave coefficients of the CWT solution on a 15 x 15 band
(3 components), the quantity of Eq. 9 below the sample. Architecture (a
ruling; only "4 Fourier layers, width 32" is given):

  x      [16][32][32]  channels 2l, 2l+1 = (Re n_l - 1.45) / 0.15, Im n_l / 0.05
  lift   h0 = W_l^T x + b_l                                   (16 -> 32, pointwise)
  layer  for k = 0..3:
           H   = DFT2(h)  on ky in [-8, 8], kx in [0, 8]      (unnormalised)
           G   = per-mode complex mix  G[o, m] = sum_i H[i, m] W_k[i, o, m]
           s   = (1/1024) sum_m w(kx) Re(G[., m] e^{+2 pi i (ky y + kx x)/32}),
                 w(0) = 1, w(kx > 0) = 2
           t   = P_k^T h + c_k                                 (pointwise)
           h   = GELU(s + t)  (no GELU after the last layer)
  head   F = (1/1024) DFT2(h) on ky, kx in [-7, 7];  out[c, m] = sum_i F[i, m] W_h[i, c, m]
  loss   L = sum |out - target|^2 / sum |target|^2  over the batch

GELU(x) = x Phi(x) with Phi the standard normal CDF.
"""
import numpy as np
from scipy.special import erf

N = 32
WIDTH = 32
CIN = 16
KY = np.arange(-8, 9)          # 17
KX = np.arange(0, 9)           # 9
HK = np.arange(-7, 8)          # 15
N_LAYERS = 4


def param_shapes():
    """Ordered parameter list: (name, shape, complex?)."""
    shapes = [("lift_w", (CIN, WIDTH), False), ("lift_b", (WIDTH,), False)]
    for k in range(N_LAYERS):
        shapes += [("spec%d" % k, (WIDTH, WIDTH, KY.size, KX.size), True),
                   ("pw%d" % k, (WIDTH, WIDTH), False),
                   ("pb%d" % k, (WIDTH,), False)]
    shapes.append(("head", (WIDTH, 3, HK.size, HK.size), True))
    return shapes


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape, cplx in param_shapes():
        if name.endswith("_b") or name.startswith("pb"):
            p[name] = np.zeros(shape)
            continue
        fan_in = shape[0]
        scale = 1.0 / np.sqrt(fan_in)
        if cplx:
            scale = scale / np.sqrt(2.0)
            if name.startswith("spec"):
                scale = scale / 4.0
            p[name] = scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
        else:
            p[name] = scale * rng.standard_normal(shape)
    return p


def encode(n):
    """Complex index [8][32][32] -> input channels [16][32][32]."""
    x = np.empty((2 * n.shape[0],) + n.shape[1:])
    x[0::2] = (n.real - 1.45) / 0.15
    x[1::2] = n.imag / 0.05
    return x


def _dft_mats():
    y = np.arange(N)
    fy = np.exp(-2j * np.pi * np.outer(KY, y) / N)            # [17][32]
    fx = np.exp(-2j * np.pi * np.outer(y, KX) / N)            # [32][9]
    w = np.where(KX > 0, 2.0, 1.0)
    iy = np.exp(2j * np.pi * np.outer(y, KY) / N)             # [32][17]
    ix = (w[:, None] * np.exp(2j * np.pi * np.outer(KX, y) / N)) / (N * N)  # [9][32]
    hy = np.exp(-2j * np.pi * np.outer(HK, y) / N) / N        # [15][32]
    hx = np.exp(-2j * np.pi * np.outer(y, HK) / N) / N        # [32][15]
    return fy, fx, iy, ix, hy, hx


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)


def to_bf16(a):
    """Round to bfloat16 (8-bit significand, round to nearest even) through
    float32, as the library stages matrix-product operands; complex values
    are rounded part by part. Returned in float64 / complex128."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return to_bf16(a.real) + 1j * to_bf16(a.imag)
    bits = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, x, keep=False, bf16=False):
    """x [B][16][32][32] -> out [B][3][15][15] complex; with keep, also the
    intermediate values the backward pass needs. With bf16, both operands of
    every matrix product are rounded to bfloat16 first (the library's
    matrix-core mode); sums, biases and GELU stay in float64."""
    r = to_bf16 if bf16 else (lambda a: a)
    fy, fx, iy, ix, hy, hx = _dft_mats()
    h = np.einsum("co,bcyx->boyx", r(p["lift_w"]), r(x)) + p["lift_b"][None, :, None, None]
    cache = {"x": x, "h": [h], "z": [], "H": []}
    for k in range(N_LAYERS):
        Hx = r(h) @ r(fx)[None, None]
        H = r(fy)[None, None] @ r(Hx)                               # [B][32][17][9]
        G = np.einsum("bikm,iokm->bokm", r(H), r(p["spec%d" % k]))
        Gy = r(iy)[None, None] @ r(G)
        s = np.real(r(Gy) @ r(ix)[None, None])                      # [B][32][32][32]
        t = (np.einsum("io,biyx->boyx", r(p["pw%d" % k]), r(h))
             + p["pb%d" % k][None, :, None, None])
        z = s + t
        cache["H"].append(H)
        cache["z"].append(z)
        h = gelu(z) if k < N_LAYERS - 1 else z
        cache["h"].append(h)
    Fx = r(h) @ r(hx)[None, None]
    F = r(hy)[None, None] @ r(Fx)                                   # [B][32][15][15]
    out = np.einsum("bikm,ickm->bckm", r(F), r(p["head"]))
    cache["F"] = F
    return (out, cache) if keep else out


def loss(out, target):
    return float(np.sum(np.abs(out - target) ** 2) / np.sum(np.abs(target) ** 2))


def backward(p, cache, out, target):
    """Gradients of loss() with respect to every parameter. A complex
    parameter's gradient is dL/dRe + i dL/dIm."""
    fy, fx, iy, ix, hy, hx = _dft_mats()
    g = {}
    gout = 2.0 * (out - target) / np.sum(np.abs(target) ** 2)       # dL/dRe + i dL/dIm
    F = cache["F"]
    g["head"] = np.einsum("bikm,bckm->ickm", np.conj(F), gout)
    gF = np.einsum("bckm,ickm->bikm", gout, np.conj(p["head"]))
    # F = hy h hx with h real: dL/dh = Re(hy^H gF hx^H)
    gh = np.real(np.conj(hy.T)[None, None] @ gF @ np.conj(hx.T)[None, None])
    for k in reversed(range(N_LAYERS)):
        z = cache["z"][k]
        gz = gh * gelu_grad(z) if k < N_LAYERS - 1 else gh
        hin = cache["h"][k]
        # pointwise branch
        g["pw%d" % k] = np.einsum("biyx,boyx->io", hin, gz)
        g["pb%d" % k] = np.sum(gz, axis=(0, 2, 3))
        gh_new = np.einsum("io,boyx->biyx", p["pw%d" % k], gz)
        # spectral branch: s = Re(iy G ix), G = mix(H), H = fy h fx
        gG = np.conj(iy.T)[None, None] @ gz @ np.conj(ix.T)[None, None]   # [B][32][17][9]
        H = cache["H"][k]
        g["spec%d" % k] = np.einsum("bikm,bokm->iokm", np.conj(H), gG)
        gH = np.einsum("bokm,iokm->bikm", gG, np.conj(p["spec%d" % k]))
        gh_new = gh_new + np.real(np.conj(fy.T)[None, None] @ gH @ np.conj(fx.T)[None, None])
        gh = gh_new
    x = cache["x"]
    g["lift_w"] = np.einsum("bcyx,boyx->co", x, gh)
    g["lift_b"] = np.sum(gh, axis=(0, 2, 3))
    return g


def flatten(p):
    """Parameters (or gradients) in the library's flat FP32 order: each array
    C-contiguous, complex arrays as interleaved (re, im)."""
    parts = []
    for name, shape, cplx in param_shapes():
        a = np.asarray(p[name])
        if cplx:
            parts.append(np.stack([a.real, a.imag], axis=-1).ravel())
        else:
            parts.append(a.ravel())
    return np.concatenate(parts)


def unflatten(v):
    p, off = {}, 0
    for name, shape, cplx in param_shapes():
        n = int(np.prod(shape))
        if cplx:
            a = v[off:off + 2 * n].reshape(shape + (2,))
            p[name] = a[..., 0] + 1j * a[..., 1]
            off += 2 * n
        else:
            p[name] = v[off:off + n].reshape(shape).astype(np.float64)
            off += n
    return p
