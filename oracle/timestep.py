"""Low-storage third-order Runge-Kutta time stepping with pressure correction
(time-discretisation appendix, rk3 equation and pressure-correction method).

Substage m = 1, 2, 3:  X~ = X^m + dt (gamma_m G^m - zeta_m G^{m-1}) for every
prognostic field, gamma = (8/15, 5/12, 3/4), zeta = (0, 17/60, 5/12); with
vertically implicit diffusion every field then solves
(1 - dt_eff d/dz K d/dz) X = X~ (predictor-velocity and tracer
time-discretisation equations); then the velocity is projected with
dt_eff = (gamma_m - zeta_m) dt, the fraction of the step the substage spans
(8/15, 2/15, 1/3).
"""
from .fv import to_padded, interior, w_faces
from .tendencies import tendencies
from .pressure import project
from .implicit import implicit_diffusion
from . import immersed

GAMMA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
ZETA = (0.0, 17.0 / 60.0, 5.0 / 12.0)


def fields_of(ph):
    return ("u", "v", "w") + tuple(ph.tracers)


def make_state(interiors, ph):
    """Padded state dict (halos filled) from interior arrays; with immersed
    cells the velocities on closed faces are set to zero first."""
    it = dict(interiors)
    if immersed.has_immersed(ph):
        it["u"], it["v"], it["w"] = immersed.mask_velocities(it["u"], it["v"], it["w"], ph)
    return {n: to_padded(it[n], ph, n) for n in fields_of(ph)}


def state_interior(state, ph):
    return {n: interior(state[n], ph, n) for n in fields_of(ph)}


def rk3_substage(state, G_prev, m, dt, ph, project_velocity=True, workers=1):
    """One substage (m = 0, 1, 2).  Returns (new padded state, G^m, p).
    workers: threads for the tendencies (see tendencies.tendencies)."""
    G = tendencies(state, ph, workers)
    X = state_interior(state, ph)
    new = {}
    for n in fields_of(ph):
        incr = GAMMA[m] * G[n]
        if m > 0:
            incr = incr - ZETA[m] * G_prev[n]
        new[n] = X[n] + dt * incr
    dt_eff = (GAMMA[m] - ZETA[m]) * dt
    if getattr(ph, "implicit_z", False):
        for n in fields_of(ph):
            new[n] = implicit_diffusion(n, new[n], ph, dt_eff)
    p = None
    if project_velocity:
        proj = immersed.project_immersed if immersed.has_immersed(ph) else project
        new["u"], new["v"], new["w"], p = proj(new["u"], new["v"], new["w"], dt_eff, ph)
    return make_state(new, ph), G, p


def rk3_step(state, dt, ph, project_velocity=True, workers=1):
    """One full RK3 time step; returns (new state, last pressure)."""
    G = None
    p = None
    for m in range(3):
        state, G, p = rk3_substage(state, G, m, dt, ph, project_velocity, workers)
    return state, p


def run(state, dt, nsteps, ph):
    for _ in range(nsteps):
        state, _ = rk3_step(state, dt, ph)
    return state
