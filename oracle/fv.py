"""Halo-padded staggered fields (finite-volume appendix, C-grid staggering).

Fields are float64 arrays of shape (nz + 2H, ny + 2H, nx + 2H), indexed
[k, j, i] with x fastest, H = 5 halo cells on every side (the reach of
the widest reconstruction, fifth-order-in-radius WENO9).  Interior cell i
(0-based) sits at padded index H + i.  Face i is the left face of cell i
("face indices are left of cell indices", composable-operator subsection), so
u[face i] is at padded index H + i too.  A bounded z axis has nz + 1 w faces;
face nz (the top wall) is stored in the first upper halo cell.

x and y are periodic.  z is periodic, or bounded by impenetrable, free-slip,
no-flux walls; halos at a wall mirror the interior evenly for cell-centred
data in z (u, v, tracers) and oddly about the wall face for w (w = 0 on the
wall).  The paper uses halos for distributed exchange (parallelisation
appendix); the wall mirroring is the reading adopted for walls.
"""
import numpy as np

H = 5


def padded_shape(ph):
    return (ph.nz + 2 * H, ph.ny + 2 * H, ph.nx + 2 * H)


def fill_halo(a, ph, kind):
    """Fill the halo of a padded field in place.

    kind: "c" for data centred in z (u, v, tracers, pressure), "w" for data on
    z faces.  Periodic wrap in x and y, then z; corner halos follow because
    each pass covers the full extent of the previously filled axes.
    """
    nx, ny, nz = ph.nx, ph.ny, ph.nz
    # x: periodic
    a[:, :, :H] = a[:, :, nx:nx + H]
    a[:, :, H + nx:] = a[:, :, H:2 * H]
    # y: periodic
    a[:, :H, :] = a[:, ny:ny + H, :]
    a[:, H + ny:, :] = a[:, H:2 * H, :]
    if not ph.z_bounded:
        a[:H] = a[nz:nz + H]
        a[H + nz:] = a[H:2 * H]
        return a
    if kind == "c":
        for s in range(H):
            a[H - 1 - s] = a[H + s]              # below the bottom wall
            a[H + nz + s] = a[H + nz - 1 - s]    # above the top wall
    elif kind == "w":
        a[H] = 0.0                               # bottom wall face
        a[H + nz] = 0.0                          # top wall face
        for s in range(1, H + 1):
            a[H - s] = -a[H + s]
        for s in range(1, H):
            a[H + nz + s] = -a[H + nz - s]
    else:
        raise ValueError(kind)
    return a


def z_spacings(ph):
    """Vertical spacings of a (possibly stretched) grid, from its faces
    (one-dimensional staggered-grid listing: cells between unevenly spaced
    faces, centres at the midpoints).

    Returns (dzc, dzf): dzc[k] = z_f[k+1] - z_f[k], the thickness of cell k
    (k = 0..nz-1), and dzf[k] = z_c[k] - z_c[k-1], the distance between the
    centres on either side of face k (k = 0..nz).  At a wall face the outside
    centre is the mirror image of the inside one, so dzf[0] = dzc[0] and
    dzf[nz] = dzc[nz-1]; periodic z wraps.  A uniform grid has dzc = dzf = dz.
    """
    nz = ph.nz
    if getattr(ph, "z_faces", None) is None:
        dz = ph.lz / nz
        return np.full(nz, dz), np.full(nz + 1, dz)
    zf = np.asarray(ph.z_faces, dtype=np.float64)
    assert zf.shape == (nz + 1,) and np.all(np.diff(zf) > 0)
    dzc = zf[1:] - zf[:-1]
    zc = 0.5 * (zf[1:] + zf[:-1])
    dzf = np.empty(nz + 1)
    dzf[1:nz] = zc[1:] - zc[:-1]
    if ph.z_bounded:
        dzf[0] = dzc[0]
        dzf[nz] = dzc[nz - 1]
    else:
        dzf[0] = dzf[nz] = 0.5 * (dzc[0] + dzc[nz - 1])
    return dzc, dzf


def is_stretched(ph):
    return getattr(ph, "z_faces", None) is not None


FIELD_KIND = {"u": "c", "v": "c", "w": "w"}


def kind_of(name):
    return FIELD_KIND.get(name, "c")


def w_faces(ph):
    """Number of stored z faces of w: nz + 1 with walls, nz if periodic."""
    return ph.nz + 1 if ph.z_bounded else ph.nz


def to_padded(interior, ph, name):
    """Place an interior array into a new padded array and fill its halo."""
    a = np.zeros(padded_shape(ph))
    nzf = interior.shape[0]
    a[H:H + nzf, H:H + ph.ny, H:H + ph.nx] = interior
    return fill_halo(a, ph, kind_of(name))


def interior(a, ph, name):
    """Copy of the interior (for w with walls: all nz + 1 faces)."""
    nzf = w_faces(ph) if name == "w" else ph.nz
    return a[H:H + nzf, H:H + ph.ny, H:H + ph.nx].copy()


def view(a, di=0, dj=0, dk=0, ni=None, nj=None, nk=None, ph=None, i0=0, j0=0, k0=0):
    """Block of a padded array starting at interior index (k0+dk, j0+dj, i0+di)
    with extent (nk, nj, ni); negative starts reach into the halo."""
    ni = ph.nx if ni is None else ni
    nj = ph.ny if nj is None else nj
    nk = ph.nz if nk is None else nk
    ks, js, is_ = H + k0 + dk, H + j0 + dj, H + i0 + di
    assert ks >= 0 and js >= 0 and is_ >= 0
    assert ks + nk <= a.shape[0] and js + nj <= a.shape[1] and is_ + ni <= a.shape[2]
    return a[ks:ks + nk, js:js + nj, is_:is_ + ni]
