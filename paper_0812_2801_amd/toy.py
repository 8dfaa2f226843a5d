"""Sweeps of the two-band toy model of sec. 6 (eq. L_toy) on the GPU: for a
set of masses (mu for the modified Ehrenfest scheme, mu_CP for CP) and a
ladder of RK4 time steps, every (mass, step) trajectory runs as one
work-item of one launch (me_toy_run).  The finest step of each mass is its
"exact" trajectory; me_toy_distance gives every other run's distance from
it, and Delta t_max(mass) is the largest step of the ladder that, with every
smaller step, stays below 0.1 (sec. 6: 0.1 % of the variation of each
dynamical variable, velocities included).  d_R and d_F (Fig. 1 a, b) come from the exact runs.

The default constants are those of the N2 molecule with a chosen gap
coordinate (workloads.TOY_N2).
"""
from __future__ import annotations

import math

import numpy as np

from . import binding as B


def params(**over) -> B.ToyParams:
    import workloads as W
    kw = dict(W.TOY_N2)
    kw.update(over)
    return B.toy_params(**kw)


def period_R(p: B.ToyParams) -> float:
    return 2.0 * math.pi / math.sqrt(p.K_R / p.M_R)


def electronic_period(p: B.ToyParams, scheme: str, mu: float) -> float:
    """Small-oscillation period of the angles about theta_i = R at G = G_0."""
    if scheme == "ehrenfest":
        return 4.0 * math.pi * mu / p.G0
    return 2.0 * math.pi * math.sqrt(2.0 * mu / p.G0)


def window(p: B.ToyParams, scheme: str, mu: float, t_sample: float) -> int:
    """Force-averaging window in samples: the geometric mean of the
    electronic and the nuclear period, at least one sample."""
    return max(1, int(round(math.sqrt(electronic_period(p, scheme, mu) * period_R(p)) / t_sample)))


def substep_ladder(n_steps: int = 28, finest: int = 2048, ratio: float = 2 ** (1 / 3)):
    """RK4 substeps per sample, ascending: a geometric ladder from finest / 4
    down to 1 (at most n_steps values) and `finest` itself, the reference."""
    out = {finest}
    s = float(finest) / 4.0
    for _ in range(n_steps):
        if s < 1.0:
            break
        out.add(int(round(s)))
        s /= ratio
    return sorted(out)


def sweep(scheme: str, mus, ladder, n_samples: int = 400, periods: float = 4.0, p: B.ToyParams = None,
          device="cuda:0", timer=None):
    """All (mu, substeps) trajectories of one scheme in one launch.  The
    trajectory index is ladder-major (consecutive work-items share a step
    count, so a wavefront does uniform work).  Returns per-mu d_R, d_F of the
    reference (finest) runs, the distance table [len(ladder), len(mus)] and
    Delta t_max per mu (NaN if even the coarsest-but-one step fails)."""
    import torch
    p = p or params()
    mus = np.asarray(mus, dtype=np.float64)
    ladder = sorted(int(s) for s in ladder)
    n_mu, n_l = mus.size, len(ladder)
    T = periods * period_R(p)
    t_s = T / n_samples
    mu_all = np.tile(mus, n_l)
    sub_all = np.repeat(np.array(ladder, dtype=np.int32), n_mu)
    win_all = np.tile(np.array([window(p, scheme, float(m), t_s) for m in mus], dtype=np.int32), n_l)
    if timer is not None:
        timer.start()
    out = B.toy_run(p, scheme, mu_all, sub_all, win_all, n_samples, T, max_substeps=max(ladder), device=device)
    if timer is not None:
        timer.stop()
    ref_row = n_l - 1                                   # the finest step
    ref = torch.as_tensor(np.tile(np.arange(n_mu, dtype=np.int32) + ref_row * n_mu, n_l), device=device)
    dist = B.toy_distance(out["samples"], ref).reshape(n_l, n_mu).cpu().numpy()
    d_R = out["d_R"].reshape(n_l, n_mu)[ref_row].cpu().numpy()
    d_F = out["d_F"].reshape(n_l, n_mu)[ref_row].cpu().numpy()
    dt = T / (n_samples * np.array(ladder, dtype=np.float64))
    dt_max = np.full(n_mu, np.nan)
    for m in range(n_mu):
        best = np.nan
        for r in range(n_l - 2, -1, -1):                # smallest step first, the reference excluded
            if not dist[r, m] < 0.1:
                break
            best = dt[r]
        dt_max[m] = best
    steps = int(np.sum(sub_all.astype(np.int64)) * n_samples)
    return {"scheme": scheme, "mu": mus, "ladder": ladder, "dt": dt, "d_R": d_R, "d_F": d_F, "dist": dist,
            "dt_max": dt_max, "rk4_steps": steps, "n_traj": int(mu_all.size), "t_total": T,
            "n_samples": n_samples}
