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

Inputs and outputs are interior arrays (u, v: (nz, ny, nx); w: (nz+1, ny, nx)
with walls, (nz, ny, nx) periodic; p: (nz, ny, nx)).
"""
import numpy as np
import scipy.fft as sfft


def divergence(u, v, w, ph):
    """Discrete divergence at cell centres: delta_x u/dx + delta_y v/dy + delta_z w/dz."""
    dx, dy, dz = ph.spacing
    d = (np.roll(u, -1, axis=2) - u) / dx + (np.roll(v, -1, axis=1) - v) / dy
    if ph.z_bounded:
        d = d + (w[1:] - w[:-1]) / dz
    else:
        d = d + (np.roll(w, -1, axis=0) - w) / dz
    return d


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
    """Solve lap p = rhs with periodic x, y and periodic or Neumann z; mean(p) = 0."""
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
    dx, dy, dz = ph.spacing
    u = u - scale * (p - np.roll(p, 1, axis=2)) / dx
    v = v - scale * (p - np.roll(p, 1, axis=1)) / dy
    w = w.copy()
    if ph.z_bounded:
        w[1:ph.nz] = w[1:ph.nz] - scale * (p[1:] - p[:-1]) / dz
    else:
        w = w - scale * (p - np.roll(p, 1, axis=0)) / dz
    return u, v, w


def project(u, v, w, dt_eff, ph):
    """Pressure correction of a predictor velocity; returns (u, v, w, p)."""
    rhs = divergence(u, v, w, ph) / dt_eff
    p = solve_poisson(rhs, ph)
    u, v, w = apply_gradient(u, v, w, p, dt_eff, ph)
    return u, v, w, p
