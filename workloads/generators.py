"""Seeded generators of sample volumes and incident fields.

Every generator takes an explicit seed and uses numpy's PCG64 generator, so a
given call returns the same array on any machine.
"""
import numpy as np


def sphere_sample(nx, ny, nz, pitch, center, radius, n_in, n_bg=1.0):
    """Index volume [nz][ny][nx] of a sphere in a uniform background.

    Voxel (i, j, l) is represented by the point (i*pitch, j*pitch, (l+1/2)*pitch)
    and takes ``n_in`` when that point lies within ``radius`` of ``center``.
    """
    i = np.arange(nx) * pitch
    j = np.arange(ny) * pitch
    zl = (np.arange(nz) + 0.5) * pitch
    Z, J, I = np.meshgrid(zl, j, i, indexing="ij")
    cx, cy, cz = center
    inside = (I - cx) ** 2 + (J - cy) ** 2 + (Z - cz) ** 2 <= radius ** 2
    out = np.full((nz, ny, nx), complex(n_bg), dtype=np.complex128)
    out[inside] = complex(n_in)
    return out


def smoothed_field(shape, sigma, seed):
    """White N(0,1) noise smoothed periodically by a Gaussian kernel of standard
    deviation ``sigma`` voxels (applied in the Fourier domain), then min-max
    scaled to [0, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(shape)
    freqs = [np.fft.fftfreq(s) for s in shape]
    grids = np.meshgrid(*freqs, indexing="ij")
    f2 = sum(g ** 2 for g in grids)
    kernel = np.exp(-2.0 * (np.pi ** 2) * (sigma ** 2) * f2)
    sm = np.real(np.fft.ifftn(np.fft.fftn(w) * kernel))
    lo, hi = sm.min(), sm.max()
    return (sm - lo) / (hi - lo)


def random_index_sample(shape, seed, n_lo=1.3, n_hi=1.6, kappa_max=0.05, sigma=4.0):
    """Complex index n + i*kappa with n in [n_lo, n_hi] and kappa in
    [0, kappa_max], each from an independent smoothed field (the kappa stream
    uses ``seed + 1000``)."""
    f1 = smoothed_field(shape, sigma, seed)
    f2 = smoothed_field(shape, sigma, seed + 1000)
    return (n_lo + (n_hi - n_lo) * f1) + 1j * (kappa_max * f2)


def focused_pupil_image(n_px, period, lam, na, focus_depth, n_medium=1.0):
    """E_x image [n_px][n_px] of a field focused by a hard circular pupil.

    The image is the periodic inverse DFT of a pupil spectrum that is nonzero
    for spatial frequencies with |s| <= na, where s = lam * (u, v) / period.
    Each pupil frequency carries the phase -2*pi/lam * sqrt(n_medium**2-|s|**2)
    * focus_depth, so that the waves meet in phase ``focus_depth`` below the
    image plane in a medium of index ``n_medium``.
    """
    idx = np.fft.fftfreq(n_px) * n_px
    v, u = np.meshgrid(idx, idx, indexing="ij")
    sx = lam * u / period
    sy = lam * v / period
    r2 = sx ** 2 + sy ** 2
    pupil = r2 <= na ** 2
    spec = np.zeros((n_px, n_px), dtype=np.complex128)
    kz = (2.0 * np.pi / lam) * np.sqrt(np.maximum(n_medium ** 2 - r2, 0.0))
    spec[pupil] = np.exp(-1j * kz[pupil] * focus_depth)
    return np.fft.ifft2(spec) * (n_px * n_px)


def lorentzian_kappa(nu, nu0=1650.0, fwhm=20.0, peak=0.1):
    """Absorption index of a Lorentzian band: peak at ``nu0`` and full width at
    half maximum ``fwhm`` (same unit as ``nu``)."""
    hw = 0.5 * fwhm
    return peak * hw ** 2 / ((nu - nu0) ** 2 + hw ** 2)
