"""Largest stable time step of the modified-Ehrenfest step (AETRS with an
order-K Taylor exponential, sec. 5.1) and of the Car-Parrinello step against
the grid spacing -- the comparison of Fig. spacing: the Taylor propagator's
limit grows with h^2, CP's Verlet limit with h -- and against the mass
parameter: mu enters the Taylor exponent as dt / (2 mu), so its limit grows
as mu; CP's Verlet limit grows as sqrt(mu_CP).

A trial runs `steps` steps on the GPU from orbitals with a small white-noise
admixture (so that the highest-frequency modes, which go unstable first, are
populated) and frozen ions; it is unstable when the library reports a norm
growth (ME_EUNSTABLE), a non-finite energy, a change of the conserved
energy beyond `drift` (relative: below the limit a symplectic step keeps it
bounded, if by percents near the limit; above, it grows without bound), or
(CP) a constraint iteration that did not converge.  dt_max is bracketed by doubling from dt0
and bisected to `rel_tol`.
"""
from __future__ import annotations

import math
import sys

from . import binding as B


def noisy_orbitals(cfg, device="cuda:0", noise=1e-2, seed=99):
    """The workload's smooth orbitals plus a white-noise admixture of relative
    amplitude `noise`, Loewdin-orthonormalised again (FP64, on the device)."""
    import torch
    import workloads as W
    psi = W.initial_orbitals_device(cfg, device)
    g = torch.Generator(device=psi.device)
    g.manual_seed(seed)
    scale = noise * psi.abs().pow(2).mean().sqrt()
    z = torch.complex(torch.randn(psi.shape, generator=g, dtype=torch.float64, device=psi.device),
                      torch.randn(psi.shape, generator=g, dtype=torch.float64, device=psi.device))
    psi = psi + scale * z
    h3 = cfg.h ** 3
    s = h3 * (psi.conj() @ psi.T)
    s = 0.5 * (s + s.conj().T)
    w, v = torch.linalg.eigh(s)
    x = (v * (1.0 / w.sqrt())) @ v.conj().T
    return (x.T.contiguous() @ psi).contiguous()


def stable(cfg, psi0, scheme: str, dt: float, steps: int, mu: float, mu_cp: float, taylor: int = 4,
           precision: str = "f64", drift: float = 0.5) -> bool:
    import workloads as W
    p, keep = B.params_from_config(cfg, W.ion_positions(cfg), precision=precision, dt=dt, mu=mu,
                                   taylor_order=taylor, freeze_ions=True)
    s = B.System(p, keep, device=psi0.device)
    try:
        s.set_state(psi0)
        if scheme == "cp":
            s.cp_begin(mu_cp, dt)
            step = lambda rep: s.cp_step(report=rep)
        else:
            step = lambda rep: s.step(report=rep)
        e0 = None
        for k in range(steps):
            rep = step(k % 10 == 9 or k == 0)
            if rep is None:
                continue
            e = rep["e_total"]
            if not math.isfinite(e):
                return False
            if scheme == "cp" and not rep["cp_constraint_residual"] < 1e-8:
                return False                    # the RATTLE iteration no longer converges
            if e0 is None:
                e0 = e
            elif abs(e - e0) > drift * abs(e0):
                return False
        return True
    except B.ModehrError as err:
        if err.status == B.ME_EUNSTABLE:
            return False
        raise
    finally:
        s.close()


def dt_max(cfg, psi0, scheme: str, mu: float, mu_cp: float, dt0: float, taylor: int = 4, steps: int = 150,
           rel_tol: float = 0.01, precision: str = "f64") -> float:
    lo = _dt_max(cfg, psi0, scheme, mu, mu_cp, dt0, taylor, steps, rel_tol, precision)
    print(f"# dt_max {scheme} n={cfg.n} taylor={taylor} mu={mu:g} mu_cp={mu_cp:g}: {lo:.5g}", file=sys.stderr,
          flush=True)
    return lo


def _dt_max(cfg, psi0, scheme, mu, mu_cp, dt0, taylor, steps, rel_tol, precision) -> float:
    lo, hi = 0.0, dt0
    while stable(cfg, psi0, scheme, hi, steps, mu, mu_cp, taylor, precision):
        lo, hi = hi, 2.0 * hi
        if hi > 1e3 * dt0:
            raise RuntimeError("no instability found")
    if lo == 0.0:
        lo = hi / 2.0
        while not stable(cfg, psi0, scheme, lo, steps, mu, mu_cp, taylor, precision):
            hi, lo = lo, lo / 2.0
            if lo < 1e-6 * dt0:
                raise RuntimeError("unstable at every time step tried")
    while hi - lo > rel_tol * lo:
        mid = 0.5 * (lo + hi)
        if stable(cfg, psi0, scheme, mid, steps, mu, mu_cp, taylor, precision):
            lo = mid
        else:
            hi = mid
    return lo


def spacing_config(n: int, L: float = 12.0, n_orb: int = 8, n_ions: int = 4):
    """An L-bohr periodic box on an n^3 grid (h = L / n) with a few ions."""
    import workloads as W
    return W.C2.replace(name=f"dt{n}", n=n, h=L / n, n_orb=n_orb, n_ions=n_ions, placement="uniform",
                        min_sep=2.5, seed=4242)


def spacing_series(ns=(32, 40, 48, 60), mu: float = 4.0, mu_cp: float = 200.0, steps: int = 150):
    """dt_max of Taylor-4 and Taylor-8 AETRS and of CP on each grid, and the
    log-log slopes of dt_max against h."""
    rows = []
    for n in ns:
        cfg = spacing_config(n)
        psi0 = noisy_orbitals(cfg)
        row = {"n": n, "h": cfg.h,
               "ehrenfest_t4": dt_max(cfg, psi0, "ehrenfest", mu, mu_cp, 0.05, 4, steps),
               "ehrenfest_t8": dt_max(cfg, psi0, "ehrenfest", mu, mu_cp, 0.05, 8, steps),
               "cp": dt_max(cfg, psi0, "cp", mu, mu_cp, 0.5, 4, steps)}
        rows.append(row)
        del psi0

    def slope(key):
        xs = [math.log(r["h"]) for r in rows]
        ys = [math.log(r[key]) for r in rows]
        mx, my = sum(xs) / len(xs), sum(ys) / len(ys)
        return sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sum((x - mx) ** 2 for x in xs)

    return {"mu": mu, "mu_cp": mu_cp, "steps": steps, "rows": rows,
            "slope_ehrenfest_t4": slope("ehrenfest_t4"), "slope_ehrenfest_t8": slope("ehrenfest_t8"),
            "slope_cp": slope("cp")}


def _slope(xs, ys):
    lx = [math.log(x) for x in xs]
    ly = [math.log(y) for y in ys]
    mx, my = sum(lx) / len(lx), sum(ly) / len(ly)
    return sum((a - mx) * (b - my) for a, b in zip(lx, ly)) / sum((a - mx) ** 2 for a in lx)


def mass_series(n: int = 40, mus=(2.0, 4.0, 8.0), mus_cp=(50.0, 200.0, 800.0), steps: int = 150):
    """dt_max of Taylor-4 AETRS against mu and of CP against mu_CP on one
    grid, with the log-log slopes (1 and 1/2 expected)."""
    cfg = spacing_config(n)
    psi0 = noisy_orbitals(cfg)
    e = [dt_max(cfg, psi0, "ehrenfest", mu, 200.0, 0.05 * mu / 4.0, 4, steps) for mu in mus]
    c = [dt_max(cfg, psi0, "cp", 4.0, mc, 0.5 * math.sqrt(mc / 200.0), 4, steps) for mc in mus_cp]
    del psi0
    return {"n": n, "h": cfg.h, "steps": steps,
            "ehrenfest_t4": [{"mu": m, "dt_max": d} for m, d in zip(mus, e)],
            "cp": [{"mu_cp": m, "dt_max": d} for m, d in zip(mus_cp, c)],
            "slope_ehrenfest_t4_vs_mu": _slope(mus, e), "slope_cp_vs_mu_cp": _slope(mus_cp, c)}
