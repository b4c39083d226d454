"""Learned subgrid closure: coarse-graining, the MLP and its training step,
and the closure's flux-divergence tendency.

The paper motivates trainable parameterizations (introduction, conclusions)
and defines coarse-graining as volume-weighted averaging that preserves
integrals ("regrid!" in the finite-volume appendix).  The closure itself is
this build's: an MLP maps the 5x5x5 staggered neighbourhood of (u, v, w, b)
around a coarse cell (500 standardised values) through 256 -> 256 GELU
layers to 4 standardised vertical subgrid fluxes (tau_uw, tau_vw, tau_ww,
J_bw) at the cell centre; the model takes their vertical flux divergence.

Precision: the GPU multiplies BF16 operands with FP32 accumulation.  The
oracle computes in FP64 and, when `bf16=True`, rounds the operands of every
product (inputs, weights, activations, back-propagated errors) to BF16 with
round-to-nearest-even, as the GPU does.  Master weights and Adam state are
FP32-valued; Adam follows Kingma & Ba (2015).
"""
import numpy as np
from scipy.special import erf

from .fv import H, view

NIN, NH, NOUT = 500, 256, 4


# ---------------------------------------------------------------------------
# BF16 rounding
# ---------------------------------------------------------------------------

def bf16(x):
    """Round to the nearest BF16 value (ties to even) via FP32, as values
    computed in FP32 on the GPU are."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# MLP
# ---------------------------------------------------------------------------

def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def init_params(seed=0):
    """Weights ~ N(0, 1/fan_in), biases 0 (FP32-valued)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((NH, NIN)) / np.sqrt(NIN), "b1": np.zeros(NH),
         "W2": rng.standard_normal((NH, NH)) / np.sqrt(NH), "b2": np.zeros(NH),
         "W3": rng.standard_normal((NOUT, NH)) / np.sqrt(NH), "b3": np.zeros(NOUT)}
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def forward(p, X, use_bf16=True):
    """X: (B, 500).  Returns (Y, cache) with Y: (B, 4)."""
    r = bf16 if use_bf16 else (lambda a: a)
    x = r(X)
    z1 = x @ r(p["W1"]).T + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ r(p["W2"]).T + p["b2"]
    h2 = r(gelu(z2))
    y = h2 @ r(p["W3"]).T + p["b3"]
    return y, {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(p, cache, Y, T, use_bf16=True):
    """Gradients of mse(Y, T) with respect to every parameter."""
    r = bf16 if use_bf16 else (lambda a: a)
    B = Y.shape[0]
    dy = 2.0 * (Y - T) / (B * NOUT)
    g = {}
    g["W3"] = r(dy).T @ cache["h2"]
    g["b3"] = dy.sum(axis=0)
    dh2 = r(dy) @ r(p["W3"])
    dz2 = dh2 * gelu_prime(cache["z2"])
    g["W2"] = r(dz2).T @ cache["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = r(dz2) @ r(p["W2"])
    dz1 = dh1 * gelu_prime(cache["z1"])
    g["W1"] = r(dz1).T @ cache["x"]
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the FP32 master weights (state holds m, v, t)."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    out = {}
    for k in p:
        m = beta1 * state.get("m_" + k, 0.0) + (1 - beta1) * g[k]
        v = beta2 * state.get("v_" + k, 0.0) + (1 - beta2) * g[k] ** 2
        state["m_" + k], state["v_" + k] = m, v
        mhat = m / (1 - beta1 ** t)
        vhat = v / (1 - beta2 ** t)
        out[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return out


# ---------------------------------------------------------------------------
# Coarse-graining (integral-preserving averages)
# ---------------------------------------------------------------------------

def coarse_grain(u, v, w, c, r):
    """Average fine interior fields to a grid r times coarser.

    c (centres, (nz, ny, nx)): mean over r^3 fine cells.  u (x faces): mean
    over the r x r fine faces lying on each coarse x face; v, w likewise.
    w has nz + 1 faces (walls) or nz (periodic); the result matches.
    Sums of volume-weighted values (and of face fluxes) are preserved.
    """
    nz, ny, nx = c.shape
    C = c.reshape(nz // r, r, ny // r, r, nx // r, r).mean(axis=(1, 3, 5))
    U = u[:, :, ::r].reshape(nz // r, r, ny // r, r, nx // r).mean(axis=(1, 3))
    V = v[:, ::r, :].reshape(nz // r, r, ny // r, nx // r, r).mean(axis=(1, 4))
    W = w[::r].reshape(w[::r].shape[0], ny // r, r, nx // r, r).mean(axis=(2, 4))
    return U, V, W, C


def subgrid_fluxes(u, v, w, b, r, z_bounded=True):
    """Vertical subgrid fluxes at coarse centres: <q w> - <q><w> over each
    r^3 box, with u, v, w first averaged to fine cell centres."""
    uc = 0.5 * (u + np.roll(u, -1, axis=2))
    vc = 0.5 * (v + np.roll(v, -1, axis=1))
    wc = 0.5 * (w[:-1] + w[1:]) if z_bounded else 0.5 * (w + np.roll(w, -1, axis=0))
    nz, ny, nx = b.shape

    def box(a):
        return a.reshape(nz // r, r, ny // r, r, nx // r, r).mean(axis=(1, 3, 5))

    out = []
    for q in (uc, vc, wc, b):
        out.append(box(q * wc) - box(q) * box(wc))
    return np.stack(out)


# ---------------------------------------------------------------------------
# Features and the closure tendency
# ---------------------------------------------------------------------------

def features(s_pad, ph, mean, std):
    """(ncell, 500) standardised 5x5x5 neighbourhoods of u, v, w, b around
    every coarse cell, variable-major, offsets (dk, dj, di) in C order.
    s_pad: padded coarse fields 'u', 'v', 'w', 'b' (halos filled)."""
    cols = []
    for vi, name in enumerate(("u", "v", "w", "b")):
        a = s_pad[name]
        for dk in range(-2, 3):
            for dj in range(-2, 3):
                for di in range(-2, 3):
                    blk = view(a, di=di, dj=dj, dk=dk, ph=ph)
                    cols.append(((blk - mean[vi]) / std[vi]).ravel())
    return np.stack(cols, axis=1)


def closure_tendency(F, ph):
    """Tendencies of (u, v, w, T) from the physical vertical fluxes
    F = (tau_uw, tau_vw, tau_ww, J_bw) at coarse centres, shape (4, nz, ny, nx).

    u: the flux at (x face, z face) averages the four adjacent centres; v
    likewise in y; tracers: the two centres either side of each z face; w:
    tau_ww at centres differenced to the w faces.  Wall fluxes are zero, so
    every column integral is conserved.  J_bw is a buoyancy flux; the
    temperature flux is J_bw / (g alpha)."""
    nz = ph.nz
    dz = ph.spacing[2]
    tuw, tvw, tww, jb = F
    zf = np.zeros((1,) + tuw.shape[1:])

    def zfaces(a):  # centres -> interior z faces, zero at the walls
        mid = 0.5 * (a[1:] + a[:-1])
        return np.concatenate([zf, mid, zf], axis=0)

    fu = zfaces(0.5 * (tuw + np.roll(tuw, 1, axis=2)))
    fv = zfaces(0.5 * (tvw + np.roll(tvw, 1, axis=1)))
    ft = zfaces(jb / (ph.g * ph.alpha))
    G = {"u": -(fu[1:] - fu[:-1]) / dz, "v": -(fv[1:] - fv[:-1]) / dz,
         "T": -(ft[1:] - ft[:-1]) / dz}
    gw = np.zeros((nz + 1,) + tuw.shape[1:])
    gw[1:nz] = -(tww[1:] - tww[:-1]) / dz
    G["w"] = gw
    return G
