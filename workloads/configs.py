"""The workloads used for parity tests and measurement, built from seeds.

sphere_config          16x16x4 voxels, one sphere n=1.4+0.01i of radius 5 voxels
                       in n=1 at pitch lam/4, 5x5 frequencies (M=25), normal
                       x-polarised plane wave, 32^3 interior output grid.
random_field_config    smoothed Gaussian random index n in [1.3,1.6], kappa in
                       [0,0.05] (correlation sigma 4 voxels); the 64x64x32 /
                       21x21 / 256^2x128 working size by default, and the
                       128x128x64 / 31x31 / 512^2x256 large size.
spectral_sweep_jobs    256 wavenumbers over 1000-3500 cm^-1 x 16 patches of
                       32x32x16 voxels at 1.1 um pitch, per-patch truncation
                       drawn from the odd orders 9..25, Lorentzian absorbing
                       inclusions at 1650 cm^-1; 8 transmitted planes of 64x64.
"""
import numpy as np

from .problem import Problem, Grid, PlaneWave
from .generators import (
    sphere_sample, random_index_sample, focused_pupil_image, smoothed_field,
    lorentzian_kappa,
)

CONFIG_NAMES = {
    "sphere": "16x16x4 sphere, M=25, 32^3 grid, complex128",
    "working": "64x64x32 random field, M=441, 256x256x128 grid, complex64",
    "large": "128x128x64 random field, M=961, 512x512x256 grid",
    "sweep": "256 wavenumbers x 16 patches 32x32x16, U in 9..25, 8x64x64 transmitted",
}


def sphere_config(out=32, nz=4):
    """The 16x16x4 sphere problem and its out^3 interior grid."""
    lam = 1.0
    p = lam / 4.0
    n = sphere_sample(16, 16, nz, p, center=(8 * p, 8 * p, 2 * p), radius=5 * p,
                      n_in=1.4 + 0.01j, n_bg=1.0)
    prob = Problem(n=n, px=p, py=p, pz=p, lam=lam, U=5, V=5, n_top=1.0,
                   n_bot=1.0 + 0.0j, plane_wave=PlaneWave(0, 0, 1.0, 0.0))
    grid = Grid(fx=out, fy=out, fz=out, z_begin=0.0, z_end=prob.thickness)
    return prob, grid


_RANDOM_SIZES = {
    # name: (lateral voxels, layers, pitch in wavelengths, U, lateral out, planes)
    "working": (64, 32, 1.0 / 6.0, 21, 256, 128),
    "large": (128, 64, 1.0 / 8.0, 31, 512, 256),
}


def random_field_config(name="working", seed=None, nz=None, U=None, out_xy=None,
                        planes_per_layer=4):
    """Random-field problem at one of the named sizes.

    ``nz`` keeps only the first nz layers (a sub-stack with the same lateral
    statistics), ``U`` overrides the truncation and ``out_xy`` the lateral
    output size. The incident field is an x-polarised NA 0.9 focus at half the
    full stack depth, given as an image at the top surface.
    """
    nxy, nz_full, pitch, U0, fxy, _ = _RANDOM_SIZES[name]
    if seed is None:
        seed = 2 if name == "working" else 3
    lam = 1.0
    p = pitch * lam
    n = random_index_sample((nz_full, nxy, nxy), seed)
    if nz is not None:
        n = n[:nz].copy()
    U = U0 if U is None else U
    X = nxy * p
    img = focused_pupil_image(nxy, X, lam, 0.9, 0.5 * nz_full * p)
    prob = Problem(n=n, px=p, py=p, pz=p, lam=lam, U=U, V=U, n_top=1.0,
                   n_bot=1.0 + 0.0j, inc_ex=img,
                   inc_ey=np.zeros_like(img))
    fo = fxy if out_xy is None else out_xy
    grid = Grid(fx=fo, fy=fo, fz=planes_per_layer * n.shape[0], z_begin=0.0,
                z_end=prob.thickness)
    return prob, grid


SWEEP_PITCH_UM = 1.1


def spectral_sweep_jobs(n_nu=256, n_patch=16, seed_u=7):
    """Job list of the spectral sweep: tuples (nu_cm1, patch, U)."""
    rng = np.random.Generator(np.random.PCG64(seed_u))
    orders = np.arange(9, 26, 2)
    u_of_patch = rng.choice(orders, size=n_patch)
    nus = 1000.0 + np.arange(n_nu) * (2500.0 / (n_nu - 1))
    return [(float(nu), int(pt), int(u_of_patch[pt])) for nu in nus
            for pt in range(n_patch)]


def sweep_problem(nu_cm1, patch, U, nz=16, nxy=32, planes=8, out_xy=64):
    """Problem and transmitted-field grid of one sweep job (lengths in um)."""
    lam = 1.0e4 / nu_cm1
    p = SWEEP_PITCH_UM
    base = random_index_sample((nz, nxy, nxy), 100 + patch, kappa_max=0.0)
    incl = smoothed_field((nz, nxy, nxy), 4.0, 500 + patch)
    mask = incl > np.quantile(incl, 0.8)
    n = base.real + 1j * lorentzian_kappa(nu_cm1) * mask
    prob = Problem(n=n.astype(np.complex128), px=p, py=p, pz=p, lam=lam, U=U,
                   V=U, n_top=1.0, n_bot=1.0 + 0.0j,
                   plane_wave=PlaneWave(0, 0, 1.0, 0.0))
    T = nz * p
    grid = Grid(fx=out_xy, fy=out_xy, fz=planes, z_begin=T, z_end=T + planes * p)
    return prob, grid


SURROGATE_SEED0 = 10000


def surrogate_patch(seed):
    """One 8 x 32 x 32 complex-index patch of the random-field family (the
    surrogate's input distribution)."""
    return random_index_sample((8, 32, 32), seed)


def surrogate_problem(n):
    """The CWT problem of a surrogate patch: pitch lambda/4 (lambda = 1),
    index 1 above and below, 15 x 15 band, normal x-polarised plane wave."""
    return Problem(n=np.asarray(n, dtype=np.complex128), px=0.25, py=0.25, pz=0.25, lam=1.0,
                   U=15, V=15, n_top=1.0, n_bot=1.0 + 0.0j,
                   plane_wave=PlaneWave(0, 0, 1.0, 0.0))
