"""Grid-fitted immersed boundaries on a rectilinear grid (the immersed-boundary
grid of the paper's examples, GridFittedBoundary / GridFittedBottom, and the
pressure solver for irregular domains of the pressure-correction appendix).

Geometry: every cell is either fluid or immersed (solid); `ph.solid` is a
boolean (nz, ny, nx) array, True in immersed cells (None: no immersed cells).
A face is closed when either of its two cells is immersed (the domain walls
of a bounded z are closed too).

Readings where the paper is silent (it defers the scheme near the boundary
and its preconditioner to other works):
* velocities on closed faces are zero (impenetrable boundary) and their
  tendencies are zero;
* no tracer flux crosses a closed face: the advective flux vanishes with the
  normal velocity, the diffusive flux is set to zero; the prescribed top flux
  enters fluid top cells only;
* everything else is the unmodified discretisation (the masking method):
  reconstructions next to the boundary read the stored values of immersed
  cells (zero velocities; tracers that never change there), and viscous
  fluxes see the zero velocities of closed faces;
* the pressure solves the discrete Poisson equation on the fluid cells with
  no flux through closed faces (the 7-point operator with closed-face terms
  removed), gauge: zero mean over the fluid cells, p = 0 in immersed cells;
  the predictor is corrected on open faces only.

The oracle solves that equation directly (a sparse LU factorisation of the
operator with one cell's value fixed, then the gauge); the GPU iterates to it with
conjugate gradients preconditioned by the FFT solver of the whole box
applied to the masked residual (the preconditioner the appendix describes).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .pressure import apply_gradient, divergence


def has_immersed(ph):
    return getattr(ph, "solid", None) is not None


def fluid(ph):
    """1.0 in fluid cells, 0.0 in immersed cells, shape (nz, ny, nx)."""
    if not has_immersed(ph):
        return np.ones((ph.nz, ph.ny, ph.nx))
    return 1.0 - np.asarray(ph.solid, dtype=float)


def open_faces(ph):
    """Open flags of the x, y and z faces: ox[k, j, i] for the face between
    cells i-1 and i (periodic), oy likewise in y, oz[k] for the face between
    levels k-1 and k (nz + 1 faces with walls, the walls closed; nz faces
    periodic)."""
    c = fluid(ph)
    ox = c * np.roll(c, 1, axis=2)
    oy = c * np.roll(c, 1, axis=1)
    if ph.z_bounded:
        oz = np.zeros((ph.nz + 1, ph.ny, ph.nx))
        oz[1:ph.nz] = c[1:] * c[:-1]
    else:
        oz = c * np.roll(c, 1, axis=0)
    return ox, oy, oz


def mask_velocities(u, v, w, ph):
    """Zero velocities on closed faces (wall faces of w keep their zero)."""
    ox, oy, oz = open_faces(ph)
    if ph.z_bounded:
        w = w.copy()
        w[1:ph.nz] = w[1:ph.nz] * oz[1:ph.nz]
        return u * ox, v * oy, w
    return u * ox, v * oy, w * oz


def laplacian(p, ph):
    """The masked 7-point operator applied to p (nz, ny, nx): the divergence
    of the gradient with the closed-face gradients set to zero, in fluid
    cells (zero in immersed cells)."""
    dx, dy, dz = ph.spacing
    ox, oy, oz = open_faces(ph)
    gx = (p - np.roll(p, 1, axis=2)) / dx * ox
    gy = (p - np.roll(p, 1, axis=1)) / dy * oy
    if ph.z_bounded:
        gz = np.zeros((ph.nz + 1, ph.ny, ph.nx))
        gz[1:ph.nz] = (p[1:] - p[:-1]) / dz * oz[1:ph.nz]
        dgz = (gz[1:] - gz[:-1]) / dz
    else:
        gz = (p - np.roll(p, 1, axis=0)) / dz * oz
        dgz = (np.roll(gz, -1, axis=0) - gz) / dz
    out = (np.roll(gx, -1, axis=2) - gx) / dx + (np.roll(gy, -1, axis=1) - gy) / dy + dgz
    return out * fluid(ph)


def operator_matrix(ph):
    """Sparse matrix of the masked operator on the fluid cells, and the flat
    indices of those cells (x fastest)."""
    dx, dy, dz = ph.spacing
    nz, ny, nx = ph.nz, ph.ny, ph.nx
    c = fluid(ph).ravel() > 0
    cells = np.nonzero(c)[0]
    index = -np.ones(nz * ny * nx, dtype=np.int64)
    index[cells] = np.arange(cells.size)
    ox, oy, oz = open_faces(ph)
    rows, cols, vals = [], [], []

    def couple(flat_a, flat_b, open_flag, h2):
        # face between cells a and b: -1/h2 on the diagonals, +1/h2 off them
        sel = (open_flag > 0) & c[flat_a] & c[flat_b]
        a, b = index[flat_a[sel]], index[flat_b[sel]]
        w = np.full(a.size, 1.0 / h2)
        rows.extend([a, b, a, b])
        cols.extend([b, a, a, b])
        vals.extend([w, w, -w, -w])

    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    flat = (K * ny + J) * nx + I
    # x face i between cells i-1 and i
    couple(((K * ny + J) * nx + (I - 1) % nx).ravel(), flat.ravel(), ox.ravel(), dx * dx)
    couple(((K * ny + (J - 1) % ny) * nx + I).ravel(), flat.ravel(), oy.ravel(), dy * dy)
    if ph.z_bounded:
        kk = K[1:]
        couple((((kk - 1) * ny + J[1:]) * nx + I[1:]).ravel(), flat[1:].ravel(),
               oz[1:nz].ravel(), dz * dz)
    else:
        couple(((((K - 1) % nz) * ny + J) * nx + I).ravel(), flat.ravel(), oz.ravel(), dz * dz)
    n = cells.size
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A, cells


def solve_poisson_immersed(rhs, ph):
    """Solve the masked Poisson equation on the fluid cells with zero mean
    there, p = 0 in immersed cells.  On a connected fluid region the
    operator's null space is the constants and the equations are consistent
    (the right-hand side, a divergence, sums to zero), so the solution is
    found with the first fluid cell's value fixed at zero (its equation then
    holds by consistency) and the fluid mean removed afterwards."""
    A, cells = operator_matrix(ph)
    A = A.tocsc()
    b = rhs.ravel()[cells]
    x = np.zeros(cells.size)
    # the reduced operator is symmetric definite: no pivoting, a symmetric
    # fill-reducing ordering
    lu = spla.splu(A[1:, 1:], permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options={"SymmetricMode": True})
    x[1:] = lu.solve(b[1:])
    x -= np.mean(x)
    p = np.zeros(ph.nz * ph.ny * ph.nx)
    p[cells] = x
    return p.reshape(ph.nz, ph.ny, ph.nx)


def project_immersed(u, v, w, dt_eff, ph):
    """Pressure correction in an immersed domain: the masked divergence of
    the predictor (closed faces carry nothing), the masked Poisson solve and
    the correction on open faces; returns (u, v, w, p)."""
    u, v, w = mask_velocities(u, v, w, ph)
    rhs = divergence(u, v, w, ph) * fluid(ph) / dt_eff
    p = solve_poisson_immersed(rhs, ph)
    u, v, w = apply_gradient(u, v, w, p, dt_eff, ph)
    u, v, w = mask_velocities(u, v, w, ph)
    return u, v, w, p
