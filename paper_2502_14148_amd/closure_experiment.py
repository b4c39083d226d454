"""Learned vertical-flux closure for the free-convection LES, end to end on
the GPU through the C ABI.

1. Truth: two high-resolution free-convection runs (a training seed and a
   held-out seed) are spun up and then continued over an evaluation window;
   every `save_every` fine steps (the training run: every `train_every`)
   the state is coarse-grained by the ratio r (oc_coarse_grain:
   integral-preserving averages and the vertical subgrid fluxes
   <q w> - <q><w>, q = u, v, w, b).
2. Training: the network (500 -> 256 -> 256 -> 4, BF16 MFMA) is trained with
   Adam on the training run's coarse snapshots: oc_closure_features gives the
   standardised 5x5x5 neighbourhoods, the targets are the standardised
   subgrid fluxes.
3. Evaluation: coarse runs (time step r x the fine one) start from the
   held-out run's first coarse snapshot, with the learned closure, without
   it, and with constant nu = kappa; each is scored against the
   coarse-grained held-out truth at every snapshot time:
     * b error: relative L2 over (z, t) of the change of the horizontally
       averaged buoyancy b(z, t) - b(z, 0);
     * flux error: relative L2 of the horizontally averaged resolved vertical
       buoyancy flux <w'b'>(z, t) (w averaged to the cell centres).

   python -m paper_2502_14148_amd.closure_experiment [--fine 256] [--ratio 4]

prints one JSON object (errors, losses, cell-step counts, timings).
"""
import argparse
import json
import sys
import time

import numpy as np

from . import inputs, oc

FIELDS = ("u", "v", "w", "T", "S")


def _log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _buoyancy(ph, T, S):
    return ph.g * (ph.alpha * (T - ph.t_ref) - ph.beta * (S - ph.s_ref))


def _profiles(ph, st):
    """Horizontal means of b and of the resolved flux w'b' at the centres."""
    b = _buoyancy(ph, st["T"], st["S"])
    wc = 0.5 * (st["w"][1:] + st["w"][:-1])
    bm = b.mean(axis=(1, 2))
    wm = wc.mean(axis=(1, 2))
    flux = (wc * b).mean(axis=(1, 2)) - wm * bm
    return bm, flux


def _host_state(m):
    return {k: m.get_state(k, dtype=np.float32).astype(np.float64) for k in FIELDS}


def truth_run(fph, cph, seed, dt, spinup, window, save_every, keep_fluxes):
    """Fine run; coarse snapshots (device tensors), flux targets (host) and
    the coarse profiles at each snapshot time."""
    import torch
    m = oc.Model(fph, "fp32")
    m.set_states(inputs.convection_initial(fph, seed=seed))
    t0 = time.perf_counter()
    m.rk3_step(dt, spinup)
    c = oc.Model(cph, "fp32")
    flux = torch.empty((4, cph.nz, cph.ny, cph.nx), dtype=torch.float32, device="cuda")
    snaps, fluxes, prof = [], [], []
    for s in range(window // save_every + 1):
        if s:
            m.rk3_step(dt, save_every)
        c.coarse_grain_from(m, flux)
        snap = {}
        for k in FIELDS:
            snap[k] = torch.empty(c.shape_of(k), dtype=torch.float32, device="cuda")
            c.get_state(k, out=snap[k])
        snaps.append(snap)
        if keep_fluxes:
            fluxes.append(flux.cpu().numpy().reshape(4, -1).T.copy())
        prof.append(_profiles(cph, _host_state(c)))
    torch.cuda.synchronize()
    return snaps, fluxes, prof, time.perf_counter() - t0


def input_stats(cph, snaps):
    """Means and standard deviations of u, v, w, b over the snapshots."""
    acc = np.zeros((4, 2))
    n = 0
    for snap in snaps:
        st = {k: snap[k].cpu().numpy().astype(np.float64) for k in FIELDS}
        b = _buoyancy(cph, st["T"], st["S"])
        for q, a in enumerate((st["u"], st["v"], st["w"], b)):
            acc[q, 0] += a.mean()
            acc[q, 1] += (a * a).mean()
        n += 1
    mean = acc[:, 0] / n
    std = np.sqrt(np.maximum(acc[:, 1] / n - mean ** 2, 1e-30))
    return mean, std


def mlp_init(seed):
    """Weights ~ N(0, 1/fan_in), biases 0."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, shp in oc.MLP_SHAPES:
        p[k] = (rng.standard_normal(shp) / np.sqrt(shp[1])) if k.startswith("W") else np.zeros(shp)
    return p


def train(cph, snaps, fluxes, stats16, epochs, batch, lr, seed):
    import torch
    n = cph.nx * cph.ny * cph.nz
    net = oc.Mlp(max(n, batch))
    net.set_params(mlp_init(seed))
    cm = oc.Model(cph, "fp32")
    X = torch.empty((n, 500), dtype=torch.float32, device="cuda")
    om, osd = stats16[8:12], stats16[12:16]
    targets = [torch.from_numpy(((f - om) / osd).astype(np.float32)).cuda() for f in fluxes]
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(snaps))
        for s in order:
            for k in FIELDS:
                cm.set_state(k, snaps[s][k])
            cm.closure_features(stats16, out=X)
            nb = n // batch
            for b in range(nb):
                last = b == nb - 1
                l = net.train_step(X[b * batch:(b + 1) * batch],
                                   targets[s][b * batch:(b + 1) * batch], lr, want_loss=last)
                if last:
                    losses.append(l)
        _log(f"epoch {ep}: loss {np.mean(losses[-len(snaps):]):.4f}")
    torch.cuda.synchronize()
    return net, losses, time.perf_counter() - t0


def heldout_loss(cph, net, snaps, fluxes, stats16, every=25):
    import torch
    cm = oc.Model(cph, "fp32")
    n = cph.nx * cph.ny * cph.nz
    X = torch.empty((n, 500), dtype=torch.float32, device="cuda")
    om, osd = stats16[8:12], stats16[12:16]
    out = []
    for s in range(0, len(snaps), every):
        for k in FIELDS:
            cm.set_state(k, snaps[s][k])
        cm.closure_features(stats16, out=X)
        y = net.forward(X).cpu().numpy().astype(np.float64)
        out.append(float(np.mean((y - (fluxes[s] - om) / osd) ** 2)))
    return float(np.mean(out))


def coarse_run(cph, start, dt, nsnap, save_every, net=None, stats16=None, nu=None):
    import dataclasses
    ph = dataclasses.replace(cph)
    if nu is not None:
        ph.nu = ph.kappa = nu
    m = oc.Model(ph, "fp32")
    for k in FIELDS:
        m.set_state(k, start[k])
    if net is not None:
        m.set_closure(net, stats16)
    prof = [_profiles(ph, _host_state(m))]
    t0 = time.perf_counter()
    for _ in range(nsnap - 1):
        m.rk3_step(dt, save_every)
        prof.append(_profiles(ph, _host_state(m)))
    finite = bool(all(np.isfinite(p[0]).all() for p in prof))
    return prof, finite, time.perf_counter() - t0


def score(prof, truth):
    b = np.array([p[0] for p in prof])
    bt = np.array([p[0] for p in truth])
    fx = np.array([p[1] for p in prof])
    ft = np.array([p[1] for p in truth])
    db, dbt = b - b[:1], bt - bt[:1]
    return {"b_change_rel_l2": float(np.linalg.norm(db - dbt) / np.linalg.norm(dbt)),
            "flux_rel_l2": float(np.linalg.norm(fx - ft) / np.linalg.norm(ft))}


def experiment(fine=256, ratio=4, dt=10.0, spinup=8640, window=2000, save_every=4, epochs=2,
               batch=4096, lr=1e-3, train_seed=1, test_seed=2, nus=(1e-4, 1e-3, 1e-2),
               extent=None, train_every=None):
    """train_every: fine steps between the training run's snapshots (default
    save_every, the spacing of the held-out run's snapshots, which is also
    the coarse runs' time step in fine steps)."""
    train_every = train_every or save_every
    nc = fine // ratio
    L = extent or (2.0 * fine, 2.0 * fine, 1.0 * fine)
    fph = inputs.convection_physics((fine, fine, fine), L)
    cph = inputs.convection_physics((nc, nc, nc), L)
    cph.closure = True
    _log(f"truth runs {fine}^3 (train seed {train_seed}, held-out seed {test_seed})")
    tr_snaps, tr_flux, _, t_tr = truth_run(fph, cph, train_seed, dt, spinup, window, train_every,
                                           True)
    te_snaps, te_flux, te_prof, t_te = truth_run(fph, cph, test_seed, dt, spinup, window,
                                                 save_every, True)
    mean, std = input_stats(cph, tr_snaps[::max(1, len(tr_snaps) // 20)])
    F = np.concatenate(tr_flux[::max(1, len(tr_flux) // 20)])
    stats16 = np.concatenate([mean, std, F.mean(axis=0), F.std(axis=0) + 1e-30])
    _log("training")
    net, losses, t_train = train(cph, tr_snaps, tr_flux, stats16, epochs, batch, lr, train_seed)
    hl = heldout_loss(cph, net, te_snaps, te_flux, stats16)
    dtc = ratio * dt
    ns = len(te_snaps)
    res = {}
    _log("coarse runs")
    prof, ok, t = coarse_run(cph, te_snaps[0], dtc, ns, 1, net=net, stats16=stats16)
    res["learned"] = dict(score(prof, te_prof), finite=ok, seconds=t)
    prof, ok, t = coarse_run(cph, te_snaps[0], dtc, ns, 1)
    res["no_closure"] = dict(score(prof, te_prof), finite=ok, seconds=t, nu=cph.nu)
    for nu in nus:
        prof, ok, t = coarse_run(cph, te_snaps[0], dtc, ns, 1, nu=nu)
        res[f"nu_{nu:g}"] = dict(score(prof, te_prof), finite=ok, seconds=t)
    base = [v for k, v in res.items() if k != "learned" and v["finite"]]
    best = min(base, key=lambda v: v["b_change_rel_l2"]) if base else None
    fine_cs = fine ** 3 * window
    coarse_cs = nc ** 3 * (ns - 1)
    return {"fine": fine, "coarse": nc, "ratio": ratio, "dt_fine_s": dt, "dt_coarse_s": dtc,
            "spinup_steps": spinup, "window_fine_steps": window, "snapshots": ns,
            "training_snapshots": len(tr_snaps), "training_snapshot_every_fine_steps": train_every,
            "cell_step_ratio": fine_cs / coarse_cs,
            "train_loss_first": losses[0], "train_loss_last": float(np.mean(losses[-5:])),
            "heldout_loss": hl, "runs": res,
            "learned_vs_best_baseline_b": (res["learned"]["b_change_rel_l2"] /
                                           best["b_change_rel_l2"]) if best else None,
            "seconds": {"truth_train": t_tr, "truth_test": t_te, "training": t_train}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fine", type=int, default=256)
    ap.add_argument("--ratio", type=int, default=4)
    ap.add_argument("--dt", type=float, default=10.0)
    ap.add_argument("--spinup", type=int, default=8640)
    ap.add_argument("--window", type=int, default=2000)
    ap.add_argument("--save-every", type=int, default=4)
    ap.add_argument("--train-every", type=int, default=1,
                    help="fine steps between training snapshots (1: 2001 snapshots)")
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--lr", type=float, default=1e-3)
    a = ap.parse_args()
    out = experiment(fine=a.fine, ratio=a.ratio, dt=a.dt, spinup=a.spinup, window=a.window,
                     save_every=a.save_every, epochs=a.epochs, lr=a.lr, train_every=a.train_every)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
