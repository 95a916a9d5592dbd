"""Plain-data description of one scattering problem and one output grid.

Mirrors the problem statement of the paper (Sec. 2.3 and Sec. 3): a sample of
complex refractive index on a voxel grid, bounded by a real-index half-space
above and a complex-index half-space below, illuminated by a field given either
as a 2D image at the top surface or as one plane wave; the spatial-frequency
truncation U x V; and the grid of points where the field is evaluated.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class PlaneWave:
    """One incident plane wave at integer spatial frequency (u, v).

    ``ex``/``ey`` are the complex transverse amplitudes; the z amplitude is
    implied by transversality.
    """
    u: int = 0
    v: int = 0
    ex: complex = 1.0 + 0.0j
    ey: complex = 0.0 + 0.0j


@dataclass
class Problem:
    """A CWT problem. Lengths share the unit of ``lam``.

    n       complex128 [nz][ny][nx]; voxel (i, j, l) sits at x = i*px, y = j*py,
            layer l spans z in [l*pz, (l+1)*pz] (top surface z0 = 0).
    n_top   real index of the upper half-space.
    n_bot   complex index of the lower half-space.
    U, V    odd spatial-frequency counts along x and y (M = U*V).
    inc_ex, inc_ey
            optional complex images [inc_ny][inc_nx] of the incident field at
            the top surface, spanning one lateral period; when both are None the
            incident field is ``plane_wave``.
    """
    n: np.ndarray
    px: float
    py: float
    pz: float
    lam: float
    U: int
    V: int
    n_top: float = 1.0
    n_bot: complex = 1.0 + 0.0j
    inc_ex: Optional[np.ndarray] = None
    inc_ey: Optional[np.ndarray] = None
    plane_wave: PlaneWave = field(default_factory=PlaneWave)

    @property
    def nz(self) -> int:
        return int(self.n.shape[0])

    @property
    def ny(self) -> int:
        return int(self.n.shape[1])

    @property
    def nx(self) -> int:
        return int(self.n.shape[2])

    @property
    def X(self) -> float:
        return self.nx * self.px

    @property
    def Y(self) -> float:
        return self.ny * self.py

    @property
    def thickness(self) -> float:
        return self.nz * self.pz


@dataclass
class Grid:
    """Output grid: fx*fy points per plane spanning one lateral period
    (x_f = f*X/fx, y_g = g*Y/fy) and fz cell-centred planes
    z_j = z_begin + (j + 1/2) * (z_end - z_begin) / fz."""
    fx: int
    fy: int
    fz: int
    z_begin: float
    z_end: float

    def z_planes(self) -> np.ndarray:
        dz = (self.z_end - self.z_begin) / self.fz
        return self.z_begin + (np.arange(self.fz) + 0.5) * dz
