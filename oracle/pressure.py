"""Pressure correction (pressure-correction appendix).

The predictor velocity u~ is made divergence-free by u = u~ - dt_eff grad p
where p solves the discrete Poisson equation  lap p = div(u~) / dt_eff
(pressure-poisson equation).  On a uniform rectilinear grid the discrete
second-order Laplacian is diagonalised by Fourier modes in periodic
directions and by cosine modes (DCT-II) in a wall-bounded direction with
no-normal-flow walls (eigenfunction expansion "evaluated via the FFT in
equispaced directions").  The wall condition n.u~ = n.u (w~ = 0 on the
walls) is already built into u~, whose wall faces are never updated.

Readings: the mean of p is set to zero (the (0,0,0) mode), and dt_eff is the
caller's (for an RK3 substage, (gamma_m - zeta_m) dt; the projected velocity
does not depend on it).

On a grid stretched in a wall-bounded z the solver is the mixed one of the
same paragraph: Fourier modes in the equispaced x and y, then for every
horizontal mode a tridiagonal solve along z of the second-order operator
(1/dzc_k) [(p_{k+1} - p_k)/dzf_{k+1} - (p_k - p_{k-1})/dzf_k] + lam_xy p_k
with no flux through the walls.  The horizontally uniform mode is singular
(constants); its gauge is the zero volume-weighted mean, sum_k dzc_k p_k = 0,
which on a uniform grid is the zero mean above.

Inputs and outputs are interior arrays (u, v: (nz, ny, nx); w: (nz+1, ny, nx)
with walls, (nz, ny, nx) periodic; p: (nz, ny, nx)).
"""
import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

from .fv import is_stretched, z_spacings


def divergence(u, v, w, ph):
    """Discrete divergence at cell centres: delta_x u/dx + delta_y v/dy +
    delta_z w/dzc (dzc the cell thickness; dz on a uniform grid)."""
    dx, dy, _ = ph.spacing
    dzc, _ = z_spacings(ph)
    dzc = dzc[:, None, None]
    d = (np.roll(u, -1, axis=2) - u) / dx + (np.roll(v, -1, axis=1) - v) / dy
    if ph.z_bounded:
        d = d + (w[1:] - w[:-1]) / dzc
    else:
        d = d + (np.roll(w, -1, axis=0) - w) / dzc
    return d


def horizontal_eigenvalues(ph):
    """Eigenvalues of delta_x^2/dx^2 + delta_y^2/dy^2 on Fourier modes, (ny, nx)."""
    dx, dy, _ = ph.spacing
    lx = -(4.0 / dx ** 2) * np.sin(np.pi * np.arange(ph.nx) / ph.nx) ** 2
    ly = -(4.0 / dy ** 2) * np.sin(np.pi * np.arange(ph.ny) / ph.ny) ** 2
    return ly[:, None] + lx[None, :]


def z_operator_bands(ph):
    """Sub- and super-diagonal of the vertical part of the Laplacian on cell
    centres, lo_k = 1/(dzc_k dzf_k) (k >= 1) and up_k = 1/(dzc_k dzf_{k+1})
    (k <= nz-2); the wall terms are absent (no flux through the walls)."""
    dzc, dzf = z_spacings(ph)
    nz = ph.nz
    lo = np.zeros(nz)
    up = np.zeros(nz)
    lo[1:] = 1.0 / (dzc[1:] * dzf[1:nz])
    up[:-1] = 1.0 / (dzc[:-1] * dzf[1:nz])
    return lo, up


def solve_poisson_stretched(rhs, ph):
    """FFT in x and y, a tridiagonal solve along z per mode, inverse FFT."""
    assert ph.z_bounded
    nz, ny, nx = rhs.shape
    dzc, _ = z_spacings(ph)
    r = np.fft.fft(np.fft.fft(rhs, axis=2), axis=1)
    lam = horizontal_eigenvalues(ph)
    lo, up = z_operator_bands(ph)
    phat = np.empty_like(r)
    for j in range(ny):
        for i in range(nx):
            if i == 0 and j == 0:
                # singular mode: least-squares (minimum-norm) solution of the
                # consistent system, then the volume-weighted mean removed
                A = np.diag(-(lo + up)) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
                x = np.linalg.lstsq(A, r[:, 0, 0], rcond=None)[0]
                phat[:, 0, 0] = x - np.sum(dzc * x) / np.sum(dzc)
                continue
            ab = np.zeros((3, nz))
            ab[0, 1:] = up[:-1]
            ab[1, :] = lam[j, i] - lo - up
            ab[2, :-1] = lo[1:]
            phat[:, j, i] = sla.solve_banded((1, 1), ab, r[:, j, i])
    p = np.fft.ifft(np.fft.ifft(phat, axis=1), axis=2)
    return p.real


def laplacian_eigenvalues(ph):
    """Eigenvalues of the 7-point Laplacian for the transform basis, as a
    (nz, ny, nx) array."""
    dx, dy, dz = ph.spacing
    kx = np.arange(ph.nx)
    ky = np.arange(ph.ny)
    kz = np.arange(ph.nz)
    lx = -(4.0 / dx ** 2) * np.sin(np.pi * kx / ph.nx) ** 2
    ly = -(4.0 / dy ** 2) * np.sin(np.pi * ky / ph.ny) ** 2
    if ph.z_bounded:
        lz = -(4.0 / dz ** 2) * np.sin(np.pi * kz / (2 * ph.nz)) ** 2
    else:
        lz = -(4.0 / dz ** 2) * np.sin(np.pi * kz / ph.nz) ** 2
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


def solve_poisson(rhs, ph):
    """Solve lap p = rhs with periodic x, y and periodic or Neumann z; mean(p) = 0
    (volume-weighted on a stretched grid)."""
    if is_stretched(ph):
        return solve_poisson_stretched(rhs, ph)
    if ph.z_bounded:
        r = sfft.dct(rhs, type=2, axis=0)
    else:
        r = np.fft.fft(rhs, axis=0)
    r = np.fft.fft(np.fft.fft(r, axis=2), axis=1)
    lam = laplacian_eigenvalues(ph)
    lam[0, 0, 0] = 1.0
    phat = r / lam
    phat[0, 0, 0] = 0.0
    p = np.fft.ifft(np.fft.ifft(phat, axis=1), axis=2)
    if ph.z_bounded:
        p = sfft.idct(p, type=2, axis=0)
    else:
        p = np.fft.ifft(p, axis=0)
    return p.real


def apply_gradient(u, v, w, p, scale, ph):
    """u -= scale * grad p at interior faces (pressure-correction equation);
    wall faces of w are left untouched."""
    dx, dy, _ = ph.spacing
    _, dzf = z_spacings(ph)
    dzf = dzf[:, None, None]
    u = u - scale * (p - np.roll(p, 1, axis=2)) / dx
    v = v - scale * (p - np.roll(p, 1, axis=1)) / dy
    w = w.copy()
    if ph.z_bounded:
        w[1:ph.nz] = w[1:ph.nz] - scale * (p[1:] - p[:-1]) / dzf[1:ph.nz]
    else:
        w = w - scale * (p - np.roll(p, 1, axis=0)) / dzf[:ph.nz]
    return u, v, w


def project(u, v, w, dt_eff, ph):
    """Pressure correction of a predictor velocity; returns (u, v, w, p)."""
    rhs = divergence(u, v, w, ph) / dt_eff
    p = solve_poisson(rhs, ph)
    u, v, w = apply_gradient(u, v, w, p, dt_eff, ph)
    return u, v, w, p
