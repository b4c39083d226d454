"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only *synthesises* data: random numbers, analytic profiles and
physical parameter sets.  It contains none of the model's arithmetic (no
reconstruction, flux, time-stepping or pressure-solve code), so a mistake in
the model cannot hide here behind a shared helper.

Array conventions (interior values only, C order, x fastest):

* tracer-like fields (T, S, c) at cell centres: shape (nz, ny, nx);
* u at x-faces (face i is the left face of cell i): (nz, ny, nx);
* v at y-faces: (nz, ny, nx);
* w at z-faces: (nz + 1, ny, nx) when z is bounded (faces 0 and nz are the
  walls and hold 0), (nz, ny, nx) when z is periodic.

The staggering is the Arakawa C-grid of the paper (finite-volume appendix,
staggered-grid listing: "face indices are left of cell indices").
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
import numpy as np

G_EARTH = 9.81


@dataclass
class Physics:
    """Physical parameters of a nonhydrostatic configuration (plain data)."""

    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    z_bounded: bool
    x0: float = 0.0
    y0: float = 0.0
    z0: float = 0.0
    advection: str = "weno5z"          # "weno{5,7,9}z" | "weno{5,7,9}_linear" | "none"
    weno_eps: float = 1e-15
    weno_q: int = 2
    f: float = 0.0                      # f-plane Coriolis parameter
    g: float = G_EARTH
    alpha: float = 0.0                  # thermal expansion (linear EOS)
    beta: float = 0.0                   # haline contraction (linear EOS)
    t_ref: float = 0.0                  # EOS reference temperature
    s_ref: float = 0.0                  # EOS reference salinity
    nu: float = 0.0
    kappa: float = 0.0
    tracers: tuple = ("c",)
    top_flux: dict = field(default_factory=dict)   # tracer -> upward flux at the top wall
    buoyancy: bool = False
    closure: bool = False               # reserve room for a learned closure
    z_faces: tuple = None               # nz + 1 ascending z faces (bounded z); None: uniform
    implicit_z: bool = False            # vertical diffusion treated implicitly per substage
    les: str = "none"                   # "none" | "smagorinsky" | "amd"
    les_cs: float = 0.16                # Smagorinsky constant C_s
    les_cb: float = 1.0                 # Lilly stratification coefficient C_b
    les_pr: float = 1.0                 # turbulent Prandtl number
    les_camd: float = 1.0 / 12.0        # AMD constant C
    solid: object = None                # (nz, ny, nx) bool: immersed cells (None: none)
    cg_tol: float = 1e-13               # relative residual of the immersed pressure solve
    cg_maxiter: int = 200

    def as_dict(self):
        return asdict(self)

    @property
    def spacing(self):
        return (self.lx / self.nx, self.ly / self.ny, self.lz / self.nz)


# ---------------------------------------------------------------------------
# Configuration presets
# ---------------------------------------------------------------------------

def periodic_box_physics(n: int = 32) -> Physics:
    """Triply periodic box, 2*pi on a side, WENO5 u,v,w,c, nu = kappa = 1e-3."""
    L = 2.0 * np.pi
    return Physics(nx=n, ny=n, nz=n, lx=L, ly=L, lz=L, z_bounded=False,
                   nu=1e-3, kappa=1e-3, tracers=("c",))


def convection_physics(n=(256, 256, 256), extent=(512.0, 512.0, 256.0),
                       surface_buoyancy_flux: float = 1e-8,
                       nu: float = 1e-5, kappa: float = 1e-5) -> Physics:
    """Free-convection LES: periodic x,y, walls in z, f-plane, linear EOS.

    The surface buoyancy flux Jb (upward positive: buoyancy leaves through the
    top, i.e. the surface cools) becomes a temperature flux Jb / (g alpha).
    """
    nx, ny, nz = n
    lx, ly, lz = extent
    alpha, beta = 2e-4, 8e-4
    return Physics(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, z_bounded=True,
                   z0=-lz, f=1e-4, g=G_EARTH, alpha=alpha, beta=beta,
                   t_ref=20.0, s_ref=35.0,
                   nu=nu, kappa=kappa, tracers=("T", "S"), buoyancy=True,
                   top_flux={"T": surface_buoyancy_flux / (G_EARTH * alpha)})


def stretched_faces(nz: int, lz: float, z0: float, sigma: float = 1.5) -> tuple:
    """z faces refined toward the top (the ocean surface): z_k = z0 + lz
    tanh(sigma k / nz) / tanh(sigma), k = 0..nz.  sigma = 1.5 makes the top
    cell about 5.5 times thinner than the bottom one."""
    xi = np.arange(nz + 1) / nz
    zf = z0 + lz * np.tanh(sigma * xi) / np.tanh(sigma)
    zf[0], zf[-1] = z0, z0 + lz
    return tuple(float(x) for x in zf)


def cell_thickness(ph: Physics) -> np.ndarray:
    """Thickness of each cell layer, shape (nz, 1, 1) (the face differences
    of ph.z_faces, or lz / nz)."""
    if ph.z_faces is None:
        return np.full((ph.nz, 1, 1), ph.lz / ph.nz)
    return np.diff(np.asarray(ph.z_faces, dtype=np.float64))[:, None, None]


def cell_centres_z(ph: Physics) -> np.ndarray:
    """z of the cell centres (midpoints of the faces), shape (nz,)."""
    if ph.z_faces is None:
        return ph.z0 + (np.arange(ph.nz) + 0.5) * (ph.lz / ph.nz)
    zf = np.asarray(ph.z_faces, dtype=np.float64)
    return 0.5 * (zf[1:] + zf[:-1])


def stretched_convection_physics(n=(256, 256, 256), extent=(512.0, 512.0, 256.0),
                                 sigma: float = 1.5, implicit_z: bool = True,
                                 **kw) -> Physics:
    """The free-convection LES on a vertically stretched grid (surface-refined
    tanh faces), optionally with vertically implicit diffusion."""
    ph = convection_physics(n, extent, **kw)
    ph.z_faces = stretched_faces(n[2], extent[2], -extent[2], sigma)
    ph.implicit_z = implicit_z
    return ph


# ---------------------------------------------------------------------------
# Random velocity fields that are discretely divergence-free by construction
# ---------------------------------------------------------------------------

def grid_fitted_bottom(ph: Physics, height) -> np.ndarray:
    """Immersed cells of a bottom at z0 + height(x, y) (grid-fitted: a cell is
    immersed when its centre lies below the bottom).  `height` takes the
    (ny, nx) arrays of cell-centre x and y."""
    dx, dy, _ = ph.spacing
    xc = ph.x0 + (np.arange(ph.nx) + 0.5) * dx
    yc = ph.y0 + (np.arange(ph.ny) + 0.5) * dy
    X, Y = np.meshgrid(xc, yc)
    zc = cell_centres_z(ph)
    return zc[:, None, None] < ph.z0 + np.asarray(height(X, Y))[None, :, :]


def seamount(ph: Physics, height_frac: float = 0.4, width_frac: float = 0.15,
             centre=(0.5, 0.5)) -> np.ndarray:
    """A Gaussian seamount of height height_frac * lz and e-folding width
    width_frac * lx, centred at `centre` (fractions of the extents)."""
    x0 = ph.x0 + centre[0] * ph.lx
    y0 = ph.y0 + centre[1] * ph.ly
    sig = width_frac * ph.lx
    return grid_fitted_bottom(
        ph, lambda X, Y: height_frac * ph.lz * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2)
                                                      / (2.0 * sig ** 2)))


def seamount_convection_physics(n=(256, 256, 256), extent=(512.0, 512.0, 256.0),
                                height_frac: float = 0.4, width_frac: float = 0.15,
                                **kw) -> Physics:
    """The free-convection workload over a Gaussian seamount (immersed
    grid-fitted bottom)."""
    ph = convection_physics(n, extent, **kw)
    ph.solid = seamount(ph, height_frac, width_frac)
    return ph


def _curl_of_potential(ax, ay, az, dx, dy, dz, bounded):
    """Staggered curl of an edge-centred vector potential.

    ax lives at (C, F, F), ay at (F, C, F), az at (F, F, C).  All arrays are
    periodic in x and y; in z they have nz faces (periodic) or nz + 1 faces
    (bounded, with the wall values already zero).  dz is a scalar or the
    per-layer thickness, shape (nz, 1, 1).  The discrete divergence of the
    result (z differences over the layer thickness) is zero identically, so
    the generator needs no pressure solve.
    """
    def dx_f(a):  # forward difference along x, periodic
        return (np.roll(a, -1, axis=2) - a) / dx

    def dy_f(a):
        return (np.roll(a, -1, axis=1) - a) / dy

    if bounded:
        def dz_f(a):  # a has nz + 1 faces -> nz centres
            return (a[1:] - a[:-1]) / dz
    else:
        def dz_f(a):
            return (np.roll(a, -1, axis=0) - a) / dz

    u = dy_f(az) - dz_f(ay)
    v = dz_f(ax) - dx_f(az)
    w = dx_f(ay) - dy_f(ax)
    return u, v, w


def _spectral_potential(rng, n, kmax, slope, shifts, L):
    """Random trigonometric field with modes 1 <= |k| <= kmax sampled at a
    staggered offset `shifts` (fractions of a cell per axis)."""
    nz, ny, nx = n
    kx = np.fft.fftfreq(nx, d=1.0 / nx)
    ky = np.fft.fftfreq(ny, d=1.0 / ny)
    kz = np.fft.fftfreq(nz, d=1.0 / nz)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    K = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shell = np.rint(K)
    mask = (shell >= 1) & (shell <= kmax)
    amp = np.zeros_like(K)
    # energy E(K) ~ K^slope spread over the modes of each integer shell; the
    # potential is one derivative smoother than the velocity.
    for s in range(1, kmax + 1):
        sel = mask & (shell == s)
        nmodes = max(int(sel.sum()), 1)
        amp[sel] = np.sqrt(s ** slope / nmodes) / s
    coef = amp * (rng.standard_normal(K.shape) + 1j * rng.standard_normal(K.shape))
    sx, sy, sz = shifts
    phase = np.exp(2j * np.pi * (KX * sx / nx + KY * sy / ny + KZ * sz / nz))
    field_ = np.fft.ifftn(coef * phase).real * (nx * ny * nz)
    return field_


def periodic_box_initial(ph: Physics, seed: int = 0, kmax: int = 8,
                         slope: float = -5.0 / 3.0, rms: float = 1.0,
                         nblobs: int = 8, sigma: float = 0.3):
    """Initial state of the triply periodic box.

    Velocity: curl of a random potential whose modes lie on integer shells
    1 <= |k| <= kmax with energy ~ K^slope, scaled so that
    sqrt(mean(u^2 + v^2 + w^2) / 3) = rms.  Tracer c: `nblobs` periodic
    Gaussian blobs of width sigma and amplitude 1 at seeded positions.
    """
    assert not ph.z_bounded
    rng = np.random.default_rng(seed)
    n = (ph.nz, ph.ny, ph.nx)
    dx, dy, dz = ph.spacing
    L = (ph.lx, ph.ly, ph.lz)
    ax = _spectral_potential(rng, n, kmax, slope, (0.5, 0.0, 0.0), L)
    ay = _spectral_potential(rng, n, kmax, slope, (0.0, 0.5, 0.0), L)
    az = _spectral_potential(rng, n, kmax, slope, (0.0, 0.0, 0.5), L)
    u, v, w = _curl_of_potential(ax, ay, az, dx, dy, dz, bounded=False)
    scale = rms / np.sqrt((np.mean(u * u) + np.mean(v * v) + np.mean(w * w)) / 3.0)
    u, v, w = u * scale, v * scale, w * scale

    xc = ph.x0 + (np.arange(ph.nx) + 0.5) * dx
    yc = ph.y0 + (np.arange(ph.ny) + 0.5) * dy
    zc = ph.z0 + (np.arange(ph.nz) + 0.5) * dz
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    centres = rng.uniform(0.0, 1.0, size=(nblobs, 3)) * np.array(L) + np.array([ph.x0, ph.y0, ph.z0])
    c = np.zeros(n)
    for (bx, by, bz) in centres:
        for mx in (-1, 0, 1):
            for my in (-1, 0, 1):
                for mz in (-1, 0, 1):
                    r2 = ((X - bx - mx * ph.lx) ** 2 + (Y - by - my * ph.ly) ** 2
                          + (Z - bz - mz * ph.lz) ** 2)
                    c += np.exp(-r2 / (2.0 * sigma ** 2))
    return {"u": u, "v": v, "w": w, "c": c}


def convection_initial(ph: Physics, seed: int = 0, noise: float = 1e-3,
                       t_surface: float = 20.0, n2: float = 1e-5, s0: float = 35.0,
                       tracer_noise: float = 0.0):
    """Initial state of the free-convection LES.

    T(z) = t_surface + n2 / (g alpha) * z at cell centres (z <= 0), S = s0.
    Velocity: curl of an i.i.d. Gaussian edge potential (zero on the walls),
    scaled to an RMS of `noise` m/s per component; it is discretely
    divergence-free and has w = 0 on the walls.  tracer_noise > 0 adds i.i.d.
    Gaussian perturbations of that standard deviation to T and S (drawn after
    the velocity, so the velocity does not depend on it).
    """
    assert ph.z_bounded
    rng = np.random.default_rng(seed)
    nz, ny, nx = ph.nz, ph.ny, ph.nx
    dx, dy, _ = ph.spacing
    dz = cell_thickness(ph)
    ax = rng.standard_normal((nz + 1, ny, nx))
    ay = rng.standard_normal((nz + 1, ny, nx))
    az = rng.standard_normal((nz, ny, nx))
    ax[0] = ax[-1] = 0.0
    ay[0] = ay[-1] = 0.0
    u, v, w = _curl_of_potential(ax, ay, az, dx, dy, dz, bounded=True)
    scale = noise / np.sqrt((np.mean(u * u) + np.mean(v * v) + np.mean(w[1:-1] * w[1:-1])) / 3.0)
    u, v, w = u * scale, v * scale, w * scale
    w[0] = 0.0
    w[-1] = 0.0
    zc = cell_centres_z(ph)
    T = np.broadcast_to((t_surface + n2 / (ph.g * ph.alpha) * zc)[:, None, None], (nz, ny, nx)).copy()
    S = np.full((nz, ny, nx), s0)
    if tracer_noise > 0:
        T += tracer_noise * rng.standard_normal((nz, ny, nx))
        S += tracer_noise * rng.standard_normal((nz, ny, nx))
    return {"u": u, "v": v, "w": w, "T": T, "S": S}


def ensemble_physics(sizes=(64, 96, 128), per_size: int = 16, seed: int = 0,
                     extent=(512.0, 512.0, 256.0), flux_range=(0.5e-8, 2.0e-8)):
    """Members of the uneven-size LES ensemble: `per_size` free-convection
    runs at each N^3 of `sizes`, all in the same domain, with surface
    buoyancy fluxes drawn uniformly from flux_range (seeded).  Returns a list
    of (Physics, member seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        for _ in range(per_size):
            jb = float(rng.uniform(*flux_range))
            out.append((convection_physics((n, n, n), extent, surface_buoyancy_flux=jb),
                        int(rng.integers(0, 2 ** 31 - 1))))
    return out


def random_state(ph: Physics, seed: int = 0, vel: float = 1.0, tracer_scale: float = 1.0,
                 divergence_free: bool = True, tracer_means=None):
    """Rough random state for parity tests (every cell independent).

    Velocities are the curl of an i.i.d. potential (divergence-free) unless
    `divergence_free` is False, in which case they are i.i.d. Gaussian (w = 0
    on walls).  Tracers are i.i.d. Gaussian around distinct means: 0, 10,
    20, ... or, if given, tracer_means (one per tracer, e.g. the equation of
    state's reference values).
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = ph.nz, ph.ny, ph.nx
    nwz = nz + 1 if ph.z_bounded else nz
    dx, dy, _ = ph.spacing
    dz = cell_thickness(ph)
    if divergence_free:
        ax = rng.standard_normal((nwz, ny, nx))
        ay = rng.standard_normal((nwz, ny, nx))
        az = rng.standard_normal((nz, ny, nx))
        if ph.z_bounded:
            ax[0] = ax[-1] = 0.0
            ay[0] = ay[-1] = 0.0
        u, v, w = _curl_of_potential(ax, ay, az, dx, dy, dz, bounded=ph.z_bounded)
        s = vel / np.sqrt(np.mean(u * u))
        u, v, w = u * s, v * s, w * s
    else:
        u = vel * rng.standard_normal((nz, ny, nx))
        v = vel * rng.standard_normal((nz, ny, nx))
        w = vel * rng.standard_normal((nwz, ny, nx))
    if ph.z_bounded:
        w[0] = 0.0
        w[-1] = 0.0
    out = {"u": u, "v": v, "w": w}
    for idx, name in enumerate(ph.tracers):
        mean = 10.0 * idx if tracer_means is None else float(tracer_means[idx])
        out[name] = (mean + tracer_scale * rng.standard_normal((nz, ny, nx)))
    return out


def smooth_random_state(ph: Physics, seed: int = 0, kmax: int = 3, vel: float = 1.0):
    """Smooth random state (low-wavenumber modes) for parity tests where the
    nonlinear WENO weights should be close to their ideal values."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = ph.nz, ph.ny, ph.nx
    dx, dy, dz = ph.spacing
    X = (np.arange(nx) + 0.5) / nx
    Y = (np.arange(ny) + 0.5) / ny
    Z = (np.arange(nz) + 0.5) / nz
    Zc, Yc, Xc = np.meshgrid(Z, Y, X, indexing="ij")

    def trig(shift=(0.0, 0.0, 0.0), zparity=None):
        f = np.zeros((nz, ny, nx))
        xs = Xc + shift[0] / nx
        ys = Yc + shift[1] / ny
        zs = Zc + shift[2] / nz
        for _ in range(6):
            kx, ky = rng.integers(-kmax, kmax + 1, size=2)
            kz = rng.integers(0 if zparity else -kmax, kmax + 1)
            a = rng.standard_normal()
            ph_ = rng.uniform(0, 2 * np.pi)
            arg = 2 * np.pi * (kx * xs + ky * ys) + ph_
            if zparity == "even":
                f += a * np.cos(np.pi * kz * zs) * np.cos(arg)
            elif zparity == "odd":
                f += a * np.sin(np.pi * max(kz, 1) * zs) * np.cos(arg)
            else:
                f += a * np.cos(arg + 2 * np.pi * kz * zs)
        return f

    even = "even" if ph.z_bounded else None
    u = vel * trig((-0.5, 0, 0), even)
    v = vel * trig((0, -0.5, 0), even)
    if ph.z_bounded:
        Zf = np.arange(nz + 1) / nz
        wz = np.zeros((nz + 1, ny, nx))
        Yw = (np.arange(ny) + 0.5) / ny
        Xw = (np.arange(nx) + 0.5) / nx
        Zg, Yg, Xg = np.meshgrid(Zf, Yw, Xw, indexing="ij")
        for _ in range(6):
            kx, ky = rng.integers(-kmax, kmax + 1, size=2)
            kz = rng.integers(1, kmax + 1)
            a = rng.standard_normal()
            p = rng.uniform(0, 2 * np.pi)
            wz += a * np.sin(np.pi * kz * Zg) * np.cos(2 * np.pi * (kx * Xg + ky * Yg) + p)
        w = vel * wz
        w[0] = 0.0
        w[-1] = 0.0
    else:
        w = vel * trig((0, 0, -0.5))
    out = {"u": u, "v": v, "w": w}
    for idx, name in enumerate(ph.tracers):
        out[name] = 10.0 * idx + trig((0, 0, 0), even)
    return out


# ---------------------------------------------------------------------------
# Hydrostatic model on a latitude-longitude sector
# ---------------------------------------------------------------------------

@dataclass
class HydrostaticPhysics:
    """Parameters of the hydrostatic model on a lat-lon grid (plain data).
    Longitude is periodic; walls at the southern/northern edges and in z."""

    nx: int
    ny: int
    nz: int
    lon0: float = 0.0
    lon_extent: float = 360.0
    lat0: float = -70.0
    lat_extent: float = 140.0
    depth: float = 3000.0
    radius: float = 6.371e6
    omega: float = 7.292115e-5
    g: float = G_EARTH
    advection: str = "weno5z"
    weno_eps: float = 1e-15
    weno_q: int = 2
    alpha: float = 2e-4
    beta: float = 8e-4
    t_ref: float = 0.0
    s_ref: float = 35.0
    nu: float = 1e-4                   # vertical viscosity
    kappa: float = 1e-4                # vertical diffusivity
    tracers: tuple = ("T", "S")
    buoyancy: bool = True
    kind: str = "hydrostatic"

    @property
    def dz(self):
        return self.depth / self.nz


def sector_physics(n=(1440, 560, 50)) -> HydrostaticPhysics:
    """Idealised 1/4-degree sector between 70S and 70N, 3000 m deep."""
    nx, ny, nz = n
    return HydrostaticPhysics(nx=nx, ny=ny, nz=nz)


def averaging_weights(N: int, M: int = None):
    """Cosine-bell averaging weights a_1..a_M for the barotropic substeps,
    symmetric about substep N (M = 2N - 1 by default) and summing to one, so
    the average is centred on the end of the baroclinic step."""
    M = 2 * N - 1 if M is None else M
    n = np.arange(1, M + 1)
    w = np.cos(0.5 * np.pi * (n - N) / N) ** 2
    return w / w.sum()


def barotropic_random_state(ph: HydrostaticPhysics, seed: int = 0, eta_scale: float = 0.5,
                            transport_scale: float = 50.0, forcing_scale: float = 1e-4):
    """Random free surface, transports and slow forcing (V = 0 on walls)."""
    rng = np.random.default_rng(seed)
    ny, nx = ph.ny, ph.nx
    out = {"eta": eta_scale * rng.standard_normal((1, ny, nx)),
           "U": transport_scale * rng.standard_normal((1, ny, nx)),
           "V": transport_scale * rng.standard_normal((1, ny + 1, nx)),
           "GU": forcing_scale * rng.standard_normal((1, ny, nx)),
           "GV": forcing_scale * rng.standard_normal((1, ny + 1, nx))}
    for k in ("V", "GV"):
        out[k][:, 0] = 0.0
        out[k][:, -1] = 0.0
    return out


RHO0 = 1026.0


def hydrostatic_initial(ph: HydrostaticPhysics, seed: int = 0, flow: float = 0.0,
                        t_noise: float = 0.1, stress_scale: float = 0.05,
                        s_noise: float = 0.0):
    """Seeded state of the lat-lon sector (arrays in the model's field shapes).

    T = T_b + (T_s - T_b)(1 + z / depth) with T_s ~ U(18, 22) and T_b = 2,
    plus N(0, t_noise^2) K; S = 35 (plus N(0, s_noise^2)); eta = 0.  Zonal wind stress bands
    tau_x(phi) = sum_{m=1..6} a_m sin(m pi (phi - lat0) / lat_extent) with
    a_m ~ N(0, stress_scale^2) N m^-2, handed over as the kinematic stress
    tau_x / rho_0; tau_y = 0.  flow > 0 adds a smooth random velocity of that
    scale (m/s): a few seeded modes in longitude, latitude (v vanishing on the
    walls) and depth; U, V are the depth integrals of u, v.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = ph.nx, ph.ny, ph.nz
    dz = ph.depth / nz
    dlam = np.deg2rad(ph.lon_extent / nx)
    dphi = np.deg2rad(ph.lat_extent / ny)
    phi0 = np.deg2rad(ph.lat0)
    lam_f = np.deg2rad(ph.lon0) + np.arange(nx) * dlam
    lam_c = lam_f + 0.5 * dlam
    phi_f = phi0 + np.arange(ny + 1) * dphi
    phi_c = phi_f[:-1] + 0.5 * dphi
    z = -ph.depth + (np.arange(nz) + 0.5) * dz
    Ts = rng.uniform(18.0, 22.0)
    Tb = 2.0
    T = (Tb + (Ts - Tb) * (1.0 + z / ph.depth))[:, None, None] * np.ones((1, ny, nx))
    T = T + t_noise * rng.standard_normal((nz, ny, nx))
    S = np.full((nz, ny, nx), 35.0)
    if s_noise > 0:
        S = S + s_noise * rng.standard_normal((nz, ny, nx))
    a = stress_scale * rng.standard_normal(6)
    s = (phi_c - phi0) / (ny * dphi)
    taux = sum(a[m - 1] * np.sin(m * np.pi * s) for m in range(1, 7)) / RHO0
    u = np.zeros((nz, ny, nx))
    v = np.zeros((nz, ny + 1, nx))
    if flow > 0:
        for _ in range(6):
            m = rng.integers(1, 4)
            n = rng.integers(1, 4)
            l = rng.integers(0, 3)
            th = rng.uniform(0, 2 * np.pi, 3)
            au, av = rng.standard_normal(2)
            zf = np.cos(l * np.pi * (z + ph.depth) / ph.depth + th[2])[:, None, None]
            u += au * zf * (np.cos(m * lam_f + th[0])[None, None, :]
                            * np.cos(n * np.pi * (phi_c - phi0) / (ny * dphi) + th[1])[None, :, None])
            v += av * zf * (np.cos(m * lam_c + th[0])[None, None, :]
                            * np.sin(n * np.pi * (phi_f - phi0) / (ny * dphi))[None, :, None])
        scale = flow / max(np.abs(u).max(), np.abs(v).max())
        u *= scale
        v *= scale
        v[:, 0] = 0.0
        v[:, ny] = 0.0
    return {"u": u, "v": v, "T": T, "S": S,
            "eta": np.zeros((1, ny, nx)),
            "U": (dz * u.sum(axis=0))[None], "V": (dz * v.sum(axis=0))[None],
            "tau_x": (taux[:, None] * np.ones((1, nx)))[None],
            "tau_y": np.zeros((1, ny + 1, nx))}
