"""FP64 CPU oracle of coupled-wave-theory (CWT) scattering and field synthesis.

TEST INFRASTRUCTURE. This module exists to check the HIP library; it is not
part of the library. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it. It shares no code with the HIP path: it reads
its inputs from the ``workloads`` package (plain seeded data) and nothing else
of this repository.

Everything is complex128 and written as the paper states it, with plain numpy /
scipy primitives (FFT, dense eigendecomposition, LU solves, matrix products)
and no blocking or fusion. Section and equation numbers refer to the paper
("sCWatter: Open source coupled wave scattering simulation for spectroscopy and
microscopy", Sun, Reddy, Mayerich).

Readings where the paper is silent, ambiguous or misprinted (each is pinned by
a closed-form test under tests/):

* Reflected waves travel towards -z: exp(-i k s_z (z - z0)) (Sec. 2.3, Eq. 9).
* s_z and layer eigenvalues take the branch Im >= 0 (Re >= 0 when Im == 0)
  (Eq. 2).
* Band coefficients are normalised by 1/(Nx*Ny), so phi(0,0) is the mean of
  n^2; voxel (i, j) sits at (i*px, j*py) (Eqs. 11-12).
* Phi and Psi are two-level block-Toeplitz (convolution in (u, v)), with the
  difference index taken modulo the voxel grid as the FFT gives it (Sec. 2.5.2).
* The lower two block rows of D follow from Faraday's and Ampere's laws
  (Eqs. 15-16); the upper two block rows are as printed in Eq. 21.
* A mode is forward when Im(gamma) > 1e-12 max|gamma|, or when |Im(gamma)| is
  below that and Re(gamma) > 0 (Sec. 2.5.3).
* The top-of-layer matrix T_l evaluates forward modes referenced at z_{l-1}
  and backward modes referenced at z_l, both at z_{l-1}; B_l evaluates them at
  z_l (Sec. 2.5.4, Eqs. 24-26).
* C maps (p_x, p_y, p_z) to (p_x, p_y, b_x, b_y) with b = s x p, using the s_z
  of each half-space wave: +s_z(n_top) incident, -s_z(n_top) reflected,
  +s_z(n_bot) transmitted (Eq. 28).
* The incident image is given at the top surface, z_bar = z0 (Sec. 2.3).
* p_z inside a layer is +Psi (S_y b_x - S_x b_y) (Sec. 2.6.2, Eqs. 32-33).
* Output planes that fall exactly on an interface belong to the layer below.

The full boundary system is solved densely (solve_unreduced) or, for deep
stacks at large M, by banded LU after a row reordering that makes it banded
(solve_unreduced_banded); the two agree to rounding (tests/test_oracle_pins.py).

Parity pinning of each function is listed in tests/test_oracle_*.py.
"""
from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sps
import scipy.sparse.linalg as spsla


class OracleError(RuntimeError):
    pass


# --------------------------------------------------------------------------
# Sec. 2.2: discrete spatial frequencies.
# --------------------------------------------------------------------------
def mode_indices(U, V):
    """Integer frequencies (u_m, v_m) in the flat order
    m = (v + floor(V/2)) * U + u + floor(U/2)  (Sec. 2.2)."""
    m = np.arange(U * V)
    v = m // U - V // 2
    u = m - (v + V // 2) * U - U // 2
    return u, v


def spatial_frequencies(u, v, X, Y, lam):
    """s_bar = (2 pi / k) [u / X, v / Y] = lam [u / X, v / Y]  (Eq. 6)."""
    return lam * u / X, lam * v / Y


def s_z(n, sx, sy):
    """s_z = sqrt(n^2 - s_x^2 - s_y^2)  (Eq. 2), branch Im >= 0."""
    w = np.sqrt(np.asarray(n, dtype=np.complex128) ** 2 - sx ** 2 - sy ** 2 + 0j)
    flip = (w.imag < 0) | ((w.imag == 0) & (w.real < 0))
    return np.where(flip, -w, w)


# --------------------------------------------------------------------------
# Sec. 2.4: layer Fourier coefficients.
# --------------------------------------------------------------------------
def band_coefficients(f, U, V):
    """Fourier coefficients of one layer's f(x, y) on the band
    |du| <= U-1, |dv| <= V-1 (Eqs. 11-12, normalised by 1/(Nx Ny)).

    Returns c[dv + V-1, du + U-1] = (1/(Nx Ny)) sum_{j,i} f[j, i]
    exp(-2 pi i (du i / Nx + dv j / Ny)).
    """
    ny, nx = f.shape
    F = np.fft.fft2(f) / (nx * ny)
    du = np.arange(-(U - 1), U)
    dv = np.arange(-(V - 1), V)
    return F[np.ix_(dv % ny, du % nx)]


def band_coefficients_direct(f, U, V):
    """The same coefficients as a literal double sum (small inputs only)."""
    ny, nx = f.shape
    out = np.zeros((2 * V - 1, 2 * U - 1), dtype=np.complex128)
    for a, dv in enumerate(range(-(V - 1), V)):
        for b, du in enumerate(range(-(U - 1), U)):
            acc = 0j
            for j in range(ny):
                for i in range(nx):
                    acc += f[j, i] * np.exp(-2j * np.pi * (du * i / nx + dv * j / ny))
            out[a, b] = acc / (nx * ny)
    return out


def toeplitz_from_band(c, u, v, U, V):
    """Block-Toeplitz convolution matrix T[m, m'] = c(u_m - u_m', v_m - v_m')
    (the Phi / Psi matrices of Sec. 2.5.2)."""
    du = u[:, None] - u[None, :]
    dv = v[:, None] - v[None, :]
    return c[dv + V - 1, du + U - 1]


# --------------------------------------------------------------------------
# Sec. 2.5.2: property matrix D.
# --------------------------------------------------------------------------
def property_matrix(Phi, Psi, sx, sy):
    """4M x 4M property matrix D with dR/dz = i k D R, R = [Px, Py, Bx, By]
    (Eqs. 19, 21). Upper-right blocks as printed; lower-left blocks from
    Faraday's and Ampere's laws (Eqs. 15-16)."""
    M = sx.size
    I = np.eye(M)
    Z = np.zeros((M, M))
    A = np.block([
        [np.outer(sx, sy) * Psi, I - np.outer(sx, sx) * Psi],
        [np.outer(sy, sy) * Psi - I, -np.outer(sy, sx) * Psi],
    ])
    Sx = np.diag(sx)
    Sy = np.diag(sy)
    C = np.block([
        [-Sx @ Sy, Sx @ Sx - Phi],
        [Phi - Sy @ Sy, Sy @ Sx],
    ])
    Z2 = np.zeros((2 * M, 2 * M))
    return np.block([[Z2, A], [C, Z2]])


# --------------------------------------------------------------------------
# Sec. 2.5.3: eigendecomposition and forward/backward split.
# --------------------------------------------------------------------------
@dataclass
class LayerModes:
    gamma: np.ndarray     # [4M] eigenvalues
    Q: np.ndarray         # [4M, 4M] eigenvectors (columns)
    forward: np.ndarray   # [4M] bool


def layer_modes(D, tol=1e-12):
    """D = Q Gamma Q^-1 (Sec. 2.5.3) via LAPACK geev, with the forward /
    backward split of the eigenvalues."""
    gamma, Q = np.linalg.eig(D)
    scale = np.max(np.abs(gamma))
    t = tol * scale
    fwd = (gamma.imag > t) | ((np.abs(gamma.imag) <= t) & (gamma.real > 0))
    n = D.shape[0]
    if int(fwd.sum()) != n // 2:
        raise OracleError("forward mode count %d != %d" % (int(fwd.sum()), n // 2))
    if np.min(np.abs(gamma)) < 1e-9 * scale:
        raise OracleError("near-defective property matrix (|gamma| ~ 0)")
    return LayerModes(gamma=gamma, Q=Q, forward=fwd)


def boundary_matrices(modes, k, d):
    """Top and bottom field matrices of a layer of thickness d (Eqs. 24-26).

    R(z) = Q diag(g(z)) alpha with g_q = exp(i k gamma_q (z - z_top)) for
    forward and exp(i k gamma_q (z - z_bottom)) for backward modes.
    T = field at the top surface, B = field at the bottom surface.
    """
    g = modes.gamma
    tau = np.where(modes.forward, 1.0 + 0j, np.exp(-1j * k * g * d))
    beta = np.where(modes.forward, np.exp(1j * k * g * d), 1.0 + 0j)
    return modes.Q * tau[None, :], modes.Q * beta[None, :]


# --------------------------------------------------------------------------
# Sec. 2.5.4: half-space P -> R map.
# --------------------------------------------------------------------------
def half_space_map(sx, sy, sigma):
    """C(sigma): [px, py, pz] -> [px, py, bx, by] with b = s x p and
    s = (s_x, s_y, sigma)  (Eq. 28)."""
    M = sx.size
    I = np.eye(M)
    Z = np.zeros((M, M))
    return np.block([
        [I, Z, Z],
        [Z, I, Z],
        [Z, -np.diag(sigma), np.diag(sy)],
        [np.diag(sigma), Z, -np.diag(sx)],
    ])


# --------------------------------------------------------------------------
# Problem setup.
# --------------------------------------------------------------------------
class BoundaryMatrices:
    """T_l (which=0) or B_l (which=1) of every layer, formed from the layer's
    modes when indexed, so that a deep stack holds one matrix per layer (Q)
    rather than three."""

    def __init__(self, modes, k, d, which):
        self._modes, self._k, self._d, self._which = modes, k, d, which

    def __len__(self):
        return len(self._modes)

    def __getitem__(self, layer):
        return boundary_matrices(self._modes[layer], self._k, self._d)[self._which]


@dataclass
class Setup:
    U: int
    V: int
    M: int
    L: int
    lam: float
    k: float
    X: float
    Y: float
    d: float
    u: np.ndarray
    v: np.ndarray
    sx: np.ndarray
    sy: np.ndarray
    sz_top: np.ndarray
    sz_bot: np.ndarray
    phi: List[np.ndarray]      # band coefficients of n^2 per layer
    psi: List[np.ndarray]      # band coefficients of 1/n^2 per layer
    Psi: List[np.ndarray]      # M x M per layer
    modes: List[LayerModes]
    T: "BoundaryMatrices"      # top-surface matrix of each layer
    B: "BoundaryMatrices"      # bottom-surface matrix of each layer
    p_inc: np.ndarray          # [3M] incident coefficients at z0


def incident_coefficients(prob, u, v, sx, sy, sz_top):
    """p_bar at the top surface (Sec. 2.3): in-band DFT coefficients of the
    incident images, or one plane wave; p_z from s . p = 0 (Eq. 14)."""
    M = u.size
    px = np.zeros(M, dtype=np.complex128)
    py = np.zeros(M, dtype=np.complex128)
    if prob.inc_ex is None and prob.inc_ey is None:
        pw = prob.plane_wave
        hit = np.nonzero((u == pw.u) & (v == pw.v))[0]
        if hit.size != 1:
            raise OracleError("plane wave frequency outside the band")
        px[hit[0]] = pw.ex
        py[hit[0]] = pw.ey
    else:
        for img, dst in ((prob.inc_ex, px), (prob.inc_ey, py)):
            if img is None:
                continue
            ny, nx = img.shape
            F = np.fft.fft2(img) / (nx * ny)
            dst[:] = F[v % ny, u % nx]
    pz = -(sx * px + sy * py) / sz_top
    return np.concatenate([px, py, pz])


def setup(prob, grazing_tol=1e-9):
    """Steps of Sec. 3.1-3.2: band coefficients, Phi/Psi, D and its
    eigendecomposition for every layer, and the boundary matrices."""
    U, V = prob.U, prob.V
    if U % 2 == 0 or V % 2 == 0 or U < 1 or V < 1:
        raise OracleError("U and V must be odd and positive")
    M = U * V
    lam = prob.lam
    k = 2.0 * np.pi / lam
    u, v = mode_indices(U, V)
    sx, sy = spatial_frequencies(u, v, prob.X, prob.Y, lam)
    sz_top = s_z(prob.n_top, sx, sy)
    sz_bot = s_z(prob.n_bot, sx, sy)
    if np.min(np.abs(sz_top)) < grazing_tol or np.min(np.abs(sz_bot)) < grazing_tol:
        raise OracleError("grazing spatial frequency in a half-space")
    phis, psis, Psis, modes = [], [], [], []
    for layer in range(prob.nz):
        eps = prob.n[layer] ** 2
        phi = band_coefficients(eps, U, V)
        psi = band_coefficients(1.0 / eps, U, V)
        Phi = toeplitz_from_band(phi, u, v, U, V)
        Psi = toeplitz_from_band(psi, u, v, U, V)
        D = property_matrix(Phi, Psi, sx, sy)
        del Phi
        md = layer_modes(D)
        del D
        phis.append(phi)
        psis.append(psi)
        Psis.append(Psi)
        modes.append(md)
    p_inc = incident_coefficients(prob, u, v, sx, sy, sz_top)
    return Setup(U=U, V=V, M=M, L=prob.nz, lam=lam, k=k, X=prob.X, Y=prob.Y,
                 d=prob.pz, u=u, v=v, sx=sx, sy=sy, sz_top=sz_top,
                 sz_bot=sz_bot, phi=phis, psi=psis, Psi=Psis, modes=modes,
                 T=BoundaryMatrices(modes, k, prob.pz, 0),
                 B=BoundaryMatrices(modes, k, prob.pz, 1), p_inc=p_inc)


# --------------------------------------------------------------------------
# Boundary-value solve.
# --------------------------------------------------------------------------
@dataclass
class Solution:
    p_ref: np.ndarray          # [3M] reflected coefficients at z0
    p_trn: np.ndarray          # [3M] transmitted coefficients at zL
    alpha: List[np.ndarray]    # [L] x [4M]


def _gauss_rows(st):
    M = st.M
    G = np.zeros((2 * M, 6 * M), dtype=np.complex128)
    idx = np.arange(M)
    # reflected wave, s = (sx, sy, -sz_top)
    G[idx, idx] = st.sx
    G[idx, M + idx] = st.sy
    G[idx, 2 * M + idx] = -st.sz_top
    # transmitted wave, s = (sx, sy, +sz_bot)
    G[M + idx, 3 * M + idx] = st.sx
    G[M + idx, 4 * M + idx] = st.sy
    G[M + idx, 5 * M + idx] = st.sz_bot
    return G


def solve_unreduced(st, dense_limit=6000):
    """The full boundary-value system with every layer's alpha as unknowns
    (Eqs. 24-26 and the two Gauss constraints of Eq. 14).

    Unknowns [p_ref (3M), alpha_1..alpha_L (4M each), p_trn (3M)].
    """
    M, L = st.M, st.L
    C_i = half_space_map(st.sx, st.sy, st.sz_top)
    C_r = half_space_map(st.sx, st.sy, -st.sz_top)
    C_t = half_space_map(st.sx, st.sy, st.sz_bot)
    N = 4 * M * L + 6 * M
    a0 = 3 * M                           # first alpha column
    pt0 = 3 * M + 4 * M * L              # first p_trn column
    rows = []
    rhs = np.zeros(N, dtype=np.complex128)
    A = sps.lil_matrix((N, N), dtype=np.complex128) if N > dense_limit else \
        np.zeros((N, N), dtype=np.complex128)

    def put(r0, c0, blk):
        A[r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] = blk

    r = 0
    # upper boundary: T_1 alpha_1 - C_r p_ref = C_i p_inc   (Eq. 24, z_bar = z0)
    put(r, a0, st.T[0])
    put(r, 0, -C_r)
    rhs[r:r + 4 * M] = C_i @ st.p_inc
    r += 4 * M
    # middle boundaries: B_{l-1} alpha_{l-1} - T_l alpha_l = 0   (Eq. 25)
    for layer in range(1, L):
        put(r, a0 + 4 * M * (layer - 1), st.B[layer - 1])
        put(r, a0 + 4 * M * layer, -st.T[layer])
        r += 4 * M
    # lower boundary: B_L alpha_L - C_t p_trn = 0   (Eq. 26)
    put(r, a0 + 4 * M * (L - 1), st.B[L - 1])
    put(r, pt0, -C_t)
    r += 4 * M
    # Gauss constraints on the reflected and transmitted waves (Eq. 14)
    G = _gauss_rows(st)
    put(r, 0, G[:, :3 * M])
    put(r, pt0, G[:, 3 * M:])
    r += 2 * M
    assert r == N
    if isinstance(A, np.ndarray):
        x = np.linalg.solve(A, rhs)
    else:
        x = spsla.spsolve(A.tocsc(), rhs)
    alpha = [x[a0 + 4 * M * layer: a0 + 4 * M * (layer + 1)] for layer in range(L)]
    return Solution(p_ref=x[:3 * M], p_trn=x[pt0:], alpha=alpha)


def solve_unreduced_banded(st):
    """The same full system as solve_unreduced (Eqs. 24-26 and the Gauss rows
    of Eq. 14), solved by banded LU with partial pivoting.

    Only the row order differs: the reflected wave's Gauss rows come first and
    the transmitted wave's last, so that every equation sits next to the
    unknowns it touches. The matrix is then banded (lower bandwidth about 5M,
    upper about 7M) and stored as bands only, which keeps a 16-layer stack at
    M = 625 (43,750 unknowns) within a few GB.
    """
    M, L = st.M, st.L
    C_i = half_space_map(st.sx, st.sy, st.sz_top)
    C_r = half_space_map(st.sx, st.sy, -st.sz_top)
    C_t = half_space_map(st.sx, st.sy, st.sz_bot)
    G = _gauss_rows(st)
    N = 4 * M * L + 6 * M
    a0 = 3 * M
    pt0 = 3 * M + 4 * M * L
    blocks = []
    rhs = np.zeros(N, dtype=np.complex128)
    r = 0
    blocks.append((r, 0, G[:M, :3 * M]))                 # reflected Gauss rows
    r += M
    blocks.append((r, a0, st.T[0]))                      # upper boundary (Eq. 24)
    blocks.append((r, 0, -C_r))
    rhs[r:r + 4 * M] = C_i @ st.p_inc
    r += 4 * M
    for layer in range(1, L):                            # middle boundaries (Eq. 25)
        blocks.append((r, a0 + 4 * M * (layer - 1), st.B[layer - 1]))
        blocks.append((r, a0 + 4 * M * layer, -st.T[layer]))
        r += 4 * M
    blocks.append((r, a0 + 4 * M * (L - 1), st.B[L - 1]))  # lower boundary (Eq. 26)
    blocks.append((r, pt0, -C_t))
    r += 4 * M
    blocks.append((r, pt0, G[M:, 3 * M:]))               # transmitted Gauss rows
    r += M
    assert r == N
    kl = max(r0 + b.shape[0] - 1 - c0 for r0, c0, b in blocks)
    ku = max(c0 + b.shape[1] - 1 - r0 for r0, c0, b in blocks)
    ab = np.zeros((kl + ku + 1, N), dtype=np.complex128)
    for r0, c0, b in blocks:
        h, w = b.shape
        for jj in range(w):
            j = c0 + jj
            # ab[ku + i - j, j] = A[i, j] for rows i = r0 .. r0 + h - 1
            ab[ku + r0 - j: ku + r0 + h - j, j] = b[:, jj]
    x = sla.solve_banded((kl, ku), ab, rhs, overwrite_ab=True, check_finite=False)
    alpha = [x[a0 + 4 * M * layer: a0 + 4 * M * (layer + 1)] for layer in range(L)]
    return Solution(p_ref=x[:3 * M], p_trn=x[pt0:], alpha=alpha)


def connection_matrix(st):
    """K = B_L T_L^-1 ... B_1 T_1^-1, the connection product of Eq. 27 in the
    top/bottom matrix reading."""
    K = np.eye(4 * st.M, dtype=np.complex128)
    for layer in range(st.L):
        K = st.B[layer] @ np.linalg.solve(st.T[layer], K)
    return K


def solve_reduced(st):
    """The paper's reduced system: C_t p_trn - K C_r p_ref = K C_i p_inc plus
    the Gauss rows (Eq. 29, Fig. 2), then the alpha recursion of Sec. 2.5.4."""
    M = st.M
    C_i = half_space_map(st.sx, st.sy, st.sz_top)
    C_r = half_space_map(st.sx, st.sy, -st.sz_top)
    C_t = half_space_map(st.sx, st.sy, st.sz_bot)
    K = connection_matrix(st)
    A = np.zeros((6 * M, 6 * M), dtype=np.complex128)
    A[:4 * M, :3 * M] = -K @ C_r
    A[:4 * M, 3 * M:] = C_t
    A[4 * M:, :] = _gauss_rows(st)
    rhs = np.zeros(6 * M, dtype=np.complex128)
    rhs[:4 * M] = K @ (C_i @ st.p_inc)
    x = np.linalg.solve(A, rhs)
    p_ref, p_trn = x[:3 * M], x[3 * M:]
    alpha = [np.linalg.solve(st.T[0], C_i @ st.p_inc + C_r @ p_ref)]
    for layer in range(1, st.L):
        alpha.append(np.linalg.solve(st.T[layer], st.B[layer - 1] @ alpha[-1]))
    return Solution(p_ref=p_ref, p_trn=p_trn, alpha=alpha)


def solve(st, route="unreduced"):
    if route == "unreduced":
        return solve_unreduced(st)
    if route == "banded":
        return solve_unreduced_banded(st)
    if route == "reduced":
        return solve_reduced(st)
    raise ValueError(route)


# --------------------------------------------------------------------------
# Sec. 2.6: field coefficients at a plane z.
# --------------------------------------------------------------------------
def layer_of(st, z):
    """Index of the layer containing z (an interface belongs to the layer
    below), -1 above the sample, L below it."""
    zL = st.L * st.d
    if z < 0.0:
        return -1
    if z >= zL:
        return st.L
    return min(int(np.floor(z / st.d)), st.L - 1)


def interior_R(st, sol, layer, z):
    """R(z) = [Q_fwd G_fwd(z) + Q_bwd G_bwd(z)] alpha  (Eqs. 30-31)."""
    md = st.modes[layer]
    z_top = layer * st.d
    z_bot = (layer + 1) * st.d
    ref = np.where(md.forward, z_top, z_bot)
    g = np.exp(1j * st.k * md.gamma * (z - ref))
    return md.Q @ (sol.alpha[layer] * g)


def plane_coefficients(st, sol, z):
    """Electric-field plane-wave coefficients p(m, z) as [3, M] (Eq. 9 outside
    the sample, Eqs. 30-33 inside)."""
    M = st.M
    layer = layer_of(st, z)
    if layer < 0:
        ginc = np.exp(1j * st.k * st.sz_top * (z - 0.0))
        gref = np.exp(-1j * st.k * st.sz_top * (z - 0.0))
        p = st.p_inc.reshape(3, M) * ginc + sol.p_ref.reshape(3, M) * gref
        return p
    if layer >= st.L:
        gt = np.exp(1j * st.k * st.sz_bot * (z - st.L * st.d))
        return sol.p_trn.reshape(3, M) * gt
    R = interior_R(st, sol, layer, z)
    px, py, bx, by = R[:M], R[M:2 * M], R[2 * M:3 * M], R[3 * M:]
    pz = st.Psi[layer] @ (st.sy * bx - st.sx * by)
    return np.stack([px, py, pz])


# --------------------------------------------------------------------------
# Eq. 10: field on the pixel grid.
# --------------------------------------------------------------------------
def dft_matrices(st, fx, fy):
    """W_x[f, m_u] = exp(2 pi i u f / fx), W_y[g, m_v] = exp(2 pi i v g / fy),
    since k s_bar . r_bar = 2 pi (u x / X + v y / Y) at x = f X/fx, y = g Y/fy."""
    us = np.arange(st.U) - st.U // 2
    vs = np.arange(st.V) - st.V // 2
    Wx = np.exp(2j * np.pi * np.outer(np.arange(fx), us) / fx)
    Wy = np.exp(2j * np.pi * np.outer(np.arange(fy), vs) / fy)
    return Wx, Wy


def synthesize(st, sol, grid):
    """E[3, fz, fy, fx] on the grid: E_c(x_f, y_g, z) = sum_m p_c(m, z)
    exp(i k s_bar_m . r_bar)  (Eq. 10), as W_y S W_x^T per plane."""
    Wx, Wy = dft_matrices(st, grid.fx, grid.fy)
    zs = grid.z_planes()
    E = np.zeros((3, grid.fz, grid.fy, grid.fx), dtype=np.complex128)
    for j, z in enumerate(zs):
        p = plane_coefficients(st, sol, z)
        for c in range(3):
            S = p[c].reshape(st.V, st.U)
            E[c, j] = Wy @ S @ Wx.T
    return E


def field_at_points(st, sol, x, y, z):
    """E at arbitrary points as the literal sum of Eq. 10 (one point at a
    time; for sampled parity checks at large sizes)."""
    out = np.zeros((3, len(x)), dtype=np.complex128)
    cache = {}
    for n_, (xx, yy, zz) in enumerate(zip(x, y, z)):
        key = float(zz)
        if key not in cache:
            cache[key] = plane_coefficients(st, sol, zz)
        p = cache[key]
        ph = np.exp(1j * st.k * (st.sx * xx + st.sy * yy))
        out[:, n_] = p @ ph
    return out


# --------------------------------------------------------------------------
# Large samples (Sec. 1: a large sample composed of small patches in two
# dimensions; Sec. 4.6: the field of one unit cell applied to the whole
# periodic pattern).
# --------------------------------------------------------------------------
def tiled(st, sol, grid, tx, ty):
    """The field over tx x ty lateral periods, [3, fz, ty*fy, tx*fx]: every
    plane wave of Eq. 10 has a lattice frequency (s_x = lam u / X), so the
    sum repeats with the period; the grid of each period is grid's."""
    return np.tile(synthesize(st, sol, grid), (1, 1, ty, tx))


def compose(parts, px, py, grid):
    """A large sample of px x py patches, each solved as its own periodic
    unit cell: parts[j * px + i] = (setup, solution) of the patch at lateral
    position (i, j); its field on grid (one period of that patch) fills
    columns i*fx .. (i+1)*fx - 1 and rows j*fy .. (j+1)*fy - 1 of the result
    [3, fz, py*fy, px*fx]. Coupling across patch borders is not modelled."""
    out = np.zeros((3, grid.fz, py * grid.fy, px * grid.fx), dtype=np.complex128)
    for j in range(py):
        for i in range(px):
            st, sol = parts[j * px + i]
            out[:, :, j * grid.fy:(j + 1) * grid.fy, i * grid.fx:(i + 1) * grid.fx] = \
                synthesize(st, sol, grid)
    return out


# --------------------------------------------------------------------------
# Optics: an ideal objective acting on the plane-wave spectrum (Sec. 1: the
# Fourier representation lets an optical system be applied directly to the
# field's spectrum).
# --------------------------------------------------------------------------
def objective_pass(st, na):
    """Coherent transfer function of an ideal objective of numerical aperture
    na, unit magnification: 1 for the modes whose direction sine
    |s_bar| = sqrt(s_x^2 + s_y^2) is at most na, else 0."""
    return (st.sx ** 2 + st.sy ** 2 <= na * na).astype(float)


def image(st, sol, grid, na):
    """The field through the objective on the grid (Eq. 10 with every mode's
    coefficients multiplied by the transfer function) and its intensity
    |E_x|^2 + |E_y|^2 + |E_z|^2; returns (E [3, fz, fy, fx], I [fz, fy, fx])."""
    H = objective_pass(st, na)
    Wx, Wy = dft_matrices(st, grid.fx, grid.fy)
    E = np.zeros((3, grid.fz, grid.fy, grid.fx), dtype=np.complex128)
    for j, z in enumerate(grid.z_planes()):
        p = plane_coefficients(st, sol, z) * H
        for c in range(3):
            E[c, j] = Wy @ p[c].reshape(st.V, st.U) @ Wx.T
    return E, np.sum(np.abs(E) ** 2, axis=0)


def filtered(st, sol, grid, H):
    """The field with a transfer function H[m] (complex, one value per mode in
    mode order) applied to every plane's plane-wave coefficients before Eq. 10
    (Sec. 1: optical elements act linearly on the spectrum), and its
    intensity; returns (E [3, fz, fy, fx], I [fz, fy, fx])."""
    H = np.asarray(H, dtype=np.complex128)
    Wx, Wy = dft_matrices(st, grid.fx, grid.fy)
    E = np.zeros((3, grid.fz, grid.fy, grid.fx), dtype=np.complex128)
    for j, z in enumerate(grid.z_planes()):
        p = plane_coefficients(st, sol, z) * H
        for c in range(3):
            E[c, j] = Wy @ p[c].reshape(st.V, st.U) @ Wx.T
    return E, np.sum(np.abs(E) ** 2, axis=0)


def simulate(prob, grid, route="unreduced"):
    st = setup(prob)
    sol = solve(st, route)
    return st, sol, synthesize(st, sol, grid)


# --------------------------------------------------------------------------
# Diagnostics used by the pins.
# --------------------------------------------------------------------------
def h_coefficients(p, sx, sy, sigma):
    """b = s x p for plane waves with s = (s_x, s_y, sigma); p is [3, M]."""
    px, py, pz = p
    return np.stack([sy * pz - sigma * py, sigma * px - sx * pz, sx * py - sy * px])


def z_flux(p, b):
    """Sum over modes of Re(p_x b_y* - p_y b_x*): the z component of the
    time-averaged Poynting vector integrated over one lateral period (up to a
    positive constant)."""
    return float(np.sum(np.real(p[0] * np.conj(b[1]) - p[1] * np.conj(b[0]))))
