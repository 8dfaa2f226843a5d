#!/usr/bin/env python3
"""Benchmark of the modified-Ehrenfest MD step on one MI355X.

Workload (default): the single-system configuration -- periodic 96^3 grid,
h = 0.25 bohr, 64 Z=4 ions placed uniformly with minimum separation 2.5 bohr,
128 complex orbitals (seeded random smoothed fields, Loewdin-orthonormalised),
mu = 4, dt = 0.08 au, AETRS with fourth-order Taylor exponentials.  One
"step" is one full MD step: ion update, V_loc and projector tables at the new
positions, both exponentials (8 H psi per orbital), density, Hartree +
exchange, local / nonlocal / Ewald forces and velocities.

The headline value is the FP32 run's orbital*gridpoint*H psi per second over
the whole step (N_orb * N * 8 per step); the same workload in FP64 is timed
beside it and the speed-up reported, together with each precision's
one-step error against the FP64 CPU oracle on sampled orbitals.

A second workload is timed beside it (``batched``): 16 systems of uneven
grid size (32^3 to 96^3) and orbital count (8 to 256), FP32, advanced
together, every Horner stage one launch over all systems, steps replayed
from a captured hipGraph, launch shape from the autotuner.

A third workload (``cp``) times the paper's comparison scheme on the same
96^3 system: Car-Parrinello with RATTLE / velocity Verlet (one H psi and five
O(N_W^2 N_C) GEMMs per step), mu_cp = 200 and dt_cp = 0.184 au, and reports
the cost of one atomic unit of simulated time for both schemes.
``--cp-series`` adds the system-size series (grids 48^3 to 128^3, orbitals
and ions in proportion to the volume) behind the cost crossover.

A fourth (``precision_study_128``) times the 128^3 x 432-orbital workload of
the precision study in FP32, FP32 with the split-bf16 projector contraction
and FP64 (its errors against the FP64 oracle are a GPU test).

Prints one JSON line.  --gpus N > 1 is refused: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "orbital·gridpts Hψ/s + ms/MD step, FP32/batched vs FP64 GPU at stated error"
STENCIL_SRC = os.path.join(ROOT, "paper_0812_2801_amd", "csrc", "stencil.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stencil_traffic_c2.json")


def stencil_hash() -> str:
    with open(STENCIL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def run_precision(cfg, inp, prec, steps, warmup, sample):
    import numpy as np
    import torch
    from paper_0812_2801_amd import binding as B
    p, keep = B.params_from_config(cfg, inp["pos"], precision=prec)
    s = B.System(p, keep, device="cuda:0")
    psi0 = torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1))
    s.set_state(psi0)
    del psi0
    e_start = s.report()["e_total"]
    # one step from the initial state: the sampled orbitals for the error check
    s.step()
    got = s.get_state()[list(sample)].cpu().numpy()
    for _ in range(warmup):
        s.step()
    s.sync()
    s.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.sync()                      # raises if an orbital norm became unstable
    launches, kms, kbytes = s.timing_read()
    kinds = {k: s.timing_read(k) for k in (2, 3)}
    s.timing_enable(False)
    rep = s.report()
    s.close()
    del s
    torch.cuda.empty_cache()
    ms = (t1 - t0) * 1e3 / steps
    return {"ms_per_step": ms, "launches": launches, "kernel_ms": kms, "kernel_bytes": kbytes,
            "kinds": kinds, "psi_sample": got, "report": rep, "energy_drift": rep["e_total"] - e_start,
            "e_start": e_start, "steps_total": 1 + warmup + steps}


def run_batch(steps, warmup, eager_steps, autotune):
    """The batched workload: 16 uneven FP32 systems advanced together, each
    Horner stage one launch over all systems, 6-step graphs replayed."""
    import tempfile
    import torch
    import workloads as W
    from paper_0812_2801_amd import binding as B
    cfgs = W.batch_configs(16)
    params, keep = [], []
    for c in cfgs:
        p, k = B.params_from_config(c, W.ion_positions(c), precision="f32")
        params.append(p)
        keep.append(k)
    b = B.Batch(params, keep, device="cuda:0")
    t0 = time.perf_counter()
    for s, c in zip(b.systems, cfgs):
        psi = W.initial_orbitals_device(c, "cuda:0")
        s.set_state(psi)
        del psi
    torch.cuda.synchronize()
    print(f"# batch inputs on the device in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    cache = os.environ.get("MODEHR_TUNE_CACHE",
                           os.path.join(tempfile.gettempdir(), "modehr_batch_tuning.json"))
    tuning = b.autotune(cache) if autotune else b.tuning()
    b.propagate(warmup, use_graph=True)            # includes the graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.propagate(steps, use_graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # eager steps: per-launch timing of the persistent stencil
    b.timing_enable(True)
    t2 = time.perf_counter()
    b.propagate(eager_steps, use_graph=False)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    launches, kms, kbytes = b.timing_read()
    n3, ms3, by3 = b.timing_read(3)
    n2, ms2, by2 = b.timing_read(2)
    b.timing_enable(False)
    norm_dev = max(s.report()["max_norm_dev"] for s in b.systems)
    work = sum(c.n_orb * c.n_points * 8 for c in cfgs)
    b.close()
    del b
    torch.cuda.empty_cache()
    ms = (t1 - t0) * 1e3 / steps
    avg_ms = kms / max(1, launches)
    avg_bytes = kbytes / max(1, launches)

    def rate(n, kms_, by):
        return (by / max(1, n)) / (kms_ / max(1, n) * 1e-3) / 1e9 if n else None
    # as for one system: the three-stream Horner stage (six of the eight
    # launches of a step) is the dominant kernel; the first stages and the
    # average over all launches are reported beside it
    achieved = rate(n3, ms3, by3)
    return {
        "workload": "16 uneven systems: grids {32..96}^3 h=0.25, 4-64 ions (jittered lattice), "
                    "8-256 orbitals each (934 M orbital points in all), mu=4, dt=0.08, FP32, whole MD steps",
        "value": work / (ms * 1e-3), "unit": "orbital·gridpt·Hψ/s", "ms_per_step": ms, "steps": steps,
        "graph": True, "eager_ms_per_step": (t3 - t2) * 1e3 / eager_steps,
        "tuning": tuning,
        "stencil": {"kernel": "batch_stencil_kernel (all systems in one launch), three-stream Horner stage",
                    "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "kernel_avg_ms": ms3 / max(1, n3), "algorithmic_bytes_per_launch": by3 / max(1, n3),
                    "first_stage": {"kernel_avg_ms": ms2 / max(1, n2), "achieved": rate(n2, ms2, by2)},
                    "all_stages": {"kernel_avg_ms": avg_ms, "algorithmic_bytes_per_launch": avg_bytes,
                                   "achieved": rate(launches, kms, kbytes),
                                   "frac": rate(launches, kms, kbytes) / HBM_PEAK_GBS}},
        "max_norm_dev": norm_dev,
    }


# Car-Parrinello parameters: the paper's benzene comparison uses mu = 15,
# dt = 3.15 for the modified Ehrenfest scheme and mu_cp = 750, dt = 7.26 for
# CP; the same ratios on this workload's mu = 4, dt = 0.08 give these.
CP_MU = 4.0 * 750.0 / 15.0
CP_DT = 0.08 * 7.26 / 3.15


def cp_config(n: int):
    """The single-system workload scaled to an n^3 grid: orbitals and ions in
    proportion to the volume (multiples of 8 orbitals)."""
    import workloads as W
    f = (n / 96.0) ** 3
    return W.C2.replace(name=f"cp{n}", n=n, n_orb=max(8, int(round(128 * f / 8.0)) * 8),
                        n_ions=max(2, int(round(64 * f))), seed=812 + 7 + n)


def time_scheme(cfg, scheme: str, steps: int, warmup: int = 2, **over) -> float:
    """ms per step of 'ehrenfest' or 'cp' on cfg (FP32, device-generated
    orbitals); `over` goes to the parameters (ETRS, force form)."""
    import torch
    import workloads as W
    from paper_0812_2801_amd import binding as B
    p, keep = B.params_from_config(cfg, W.ion_positions(cfg), precision="f32", **over)
    s = B.System(p, keep, device="cuda:0")
    psi = W.initial_orbitals_device(cfg, "cuda:0")
    s.set_state(psi)
    del psi
    if scheme == "cp":
        s.cp_begin(CP_MU, CP_DT)
        step = s.cp_step
    else:
        step = s.step
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    rep = s.report()
    s.close()
    del s
    torch.cuda.empty_cache()
    if not math.isfinite(rep["e_total"]):
        raise RuntimeError(f"{scheme} on {cfg.name}: non-finite energy")
    return ms


def run_cp(steps: int, ehrenfest_ms: float, series: bool):
    """CP on the 96^3 workload; the cost per atomic unit of simulated time of
    both schemes (ms per step / dt); with `series`, the same over system size."""
    import workloads as W
    cp_ms = time_scheme(W.C2, "cp", steps)
    out = {"workload": "96^3 h=0.25, 64 ions, 128 FP32 orbitals; Car-Parrinello with RATTLE / velocity Verlet, "
                       f"mu_cp={CP_MU:g}, dt_cp={CP_DT:.4f}",
           "ms_per_step": cp_ms, "dt": CP_DT, "ms_per_au": cp_ms / CP_DT,
           "ehrenfest_ms_per_au": ehrenfest_ms / 0.08,
           "ehrenfest_over_cp_cost_per_au": (ehrenfest_ms / 0.08) / (cp_ms / CP_DT)}
    if series:
        rows = []
        for n in (48, 64, 80, 96, 112, 128):
            cfg = cp_config(n)
            e_ms = time_scheme(cfg, "ehrenfest", 10)
            c_ms = time_scheme(cfg, "cp", 10)
            row = {"n": n, "n_orb": cfg.n_orb, "n_ions": cfg.n_ions, "ehrenfest_ms_per_step": e_ms,
                   "cp_ms_per_step": c_ms, "ehrenfest_over_cp_cost_per_au": (e_ms / 0.08) / (c_ms / CP_DT)}
            print(f"# cp series {row}", file=sys.stderr, flush=True)
            rows.append(row)
        out["series"] = rows
    return out


def run_adjoint(every: int = 10):
    """The adjoint workload: 64^3, 32 frozen ions, 64 FP32 orbitals, 50 steps
    with per-step field amplitudes and a 16^3 static perturbation; the final
    dipole and its gradient with respect to both through the checkpointed
    adjoint (checkpoints every `every` steps)."""
    import torch
    import workloads as W
    from paper_0812_2801_amd import binding as B
    from paper_0812_2801_amd.autograd import DipoleObjective
    cfg = W.C5
    pos = W.ion_positions(cfg)
    rngs = W.rngs(cfg)
    ctrl = W.controls(cfg, rngs[2])
    psi0 = W.initial_orbitals_device(cfg, "cuda:0")
    p, keep = B.params_from_config(cfg, pos, precision="f32", enable_adjoint=True)
    s = B.System(p, keep)
    c = torch.tensor(ctrl, dtype=torch.float64, requires_grad=True)
    dv = torch.zeros((cfg.coarse_n,) * 3, dtype=torch.float64, requires_grad=True)
    J = DipoleObjective.apply(c, dv, s, psi0, every)          # warm-up (plans, code objects)
    J.backward()
    c.grad = None
    dv.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = DipoleObjective.apply(c, dv, s, psi0, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.close()
    del s, psi0
    torch.cuda.empty_cache()
    return {"workload": "64^3 h=0.25, 32 frozen ions, 64 FP32 orbitals, mu=1, dt=0.02, 50 steps with "
                        "field amplitudes; dJ/d(eps_n) and dJ/d(dV 16^3) of the final dipole",
            "forward_ms": (t1 - t0) * 1e3, "backward_ms": (t2 - t1) * 1e3,
            "backward_over_forward": (t2 - t1) / (t1 - t0), "checkpoint_every": every,
            "J": float(J), "grad_eps_norm": float(c.grad.norm())}


def run_c4(steps: int = 6, warmup: int = 2, precisions=("f32", "f32_bf16x3", "f64")) -> dict:
    """The precision-study workload (128^3 grid, 216 ions on a jittered
    lattice, 432 orbitals, mu = 4, dt = 0.08, moving ions): time per MD step
    in each precision and the three-stream Horner stage's rate.  Orbitals
    drawn on the device (same recipe, torch's generator)."""
    import torch
    import workloads as W
    from paper_0812_2801_amd import binding as B
    cfg = W.C4
    psi = W.initial_orbitals_device(cfg, "cuda:0")
    pos = W.ion_positions(cfg)
    out = {"workload": "128^3 grid h=0.25, 216 ions Z=4 (jittered 6^3 lattice), 432 complex orbitals, mu=4, "
                       "dt=0.08, AETRS+Taylor-4, moving ions, whole MD step"}
    work = cfg.n_orb * cfg.n_points * 8
    for prec in precisions:
        p, keep = B.params_from_config(cfg, pos, precision=prec)
        s = B.System(p, keep, device="cuda:0")
        s.set_state(psi)
        for _ in range(warmup):
            s.step()
        s.sync()
        s.timing_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.sync()
        n3, ms3, by3 = s.timing_read(3)
        s.timing_enable(False)
        s.close()
        del s
        torch.cuda.empty_cache()
        ms = (t1 - t0) * 1e3 / steps
        out[prec] = {"ms_per_step": ms, "value": work / (ms * 1e-3),
                     "stencil_three_stream": {"kernel_avg_ms": ms3 / max(1, n3),
                                              "achieved_GBps": (by3 / max(1, n3)) / (ms3 / max(1, n3) * 1e-3) / 1e9}}
        print(f"# c4 {prec}: {ms:.2f} ms/step", file=sys.stderr, flush=True)
    del psi
    torch.cuda.empty_cache()
    if "f64" in out and "f32" in out:
        out["speedup_f32_vs_f64"] = out["f64"]["ms_per_step"] / out["f32"]["ms_per_step"]
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample(cfg, inp, n_sample):
    """FP64 oracle: one AETRS propagation (both exponentials) of the first
    n_sample orbitals from the initial state, the orbitals split over P worker
    processes (P = the cores this process may run on, at most 16), one
    BLAS/OpenMP thread each, by the oracle's orbital-parallel driver; H(t)
    and H(t+dt) are built from all orbitals (not timed).  Returns the
    propagated orbitals, the wall time and P."""
    from oracle import Model, dynamics
    from oracle.parallel import Driver
    m = Model.from_config(cfg)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    _, h0, h1 = dynamics.step_hamiltonians(m, st)
    workers = max(1, min(16, len(os.sched_getaffinity(0)), n_sample))
    with Driver(m, n_sample, workers=workers, orbitals_per_task=max(1, n_sample // workers)) as d:
        d.psi[...] = inp["psi"][:n_sample]
        t0 = time.perf_counter()
        d.propagate(h0, h1)
        t1 = time.perf_counter()
        out = d.psi.copy()
    return out, t1 - t0, workers


def traffic_entry(kernel: str):
    """Measured HBM bytes per launch of one stencil instantiation (FETCH_SIZE +
    WRITE_SIZE, copy-calibrated), or None when no measurement of the current
    stencil source exists."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        d = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if d.get("stencil_sha256_16") != stencil_hash():
        return None
    k = d.get("by_kernel", {}).get(kernel)
    if not k:
        return None
    return 1024.0 * (d["fetch_scale"] * k["fetch_KiB"] + d["write_scale"] * k["write_KiB"])


def device_streams(n_bytes: int, reps: int = 20) -> dict:
    """HBM rate of plain torch streams over buffers of n_bytes each: a copy
    (1 read, 1 write) and a + b (2 reads, 1 write, the stencil's mix)."""
    import torch
    n = n_bytes // 4
    a = torch.ones(n, device="cuda:0")
    b = torch.ones(n, device="cuda:0")
    c = torch.empty(n, device="cuda:0")

    def rate(fn, moved):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return moved / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

    out = {"copy": rate(lambda: c.copy_(a), 2 * n * 4), "add": rate(lambda: torch.add(a, b, out=c), 3 * n * 4)}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def calibrate_copy(gib: float = 2.0, reps: int = 5):
    """A plain device copy of known size, for scaling HBM counters."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each": 2 * n * 4, "reps": reps}))


def run_toy(oracle_sample: bool = True) -> dict:
    """The Fig. 1 (c, d) sweep of the two-band toy model (eq. L_toy): every
    (mass, RK4 step) trajectory of a scheme in one launch, timed with HIP
    events on the launch stream; d_R, d_F and Delta t_max per mass.  With
    oracle_sample, the oracle integrates one trajectory of the sweep (its
    RK4 steps per second on one core)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_0812_2801_amd import toy
    S = W.TOY_SWEEP
    ladder = toy.substep_ladder(S["ladder_steps"], S["finest"], S["ratio"])

    class Timer:
        def start(self):
            self.e0 = torch.cuda.Event(enable_timing=True)
            self.e1 = torch.cuda.Event(enable_timing=True)
            self.e0.record()

        def stop(self):
            self.e1.record()

        def ms(self):
            self.e1.synchronize()
            return self.e0.elapsed_time(self.e1)

    out = {"workload": f"{S['n_mu']} masses x {len(ladder)} RK4 steps per scheme, {S['periods']:g} gsBO periods, "
                       f"{S['n_samples']} samples", "ladder": ladder}
    for scheme in ("ehrenfest", "cp"):
        mus = np.geomspace(*S["mu_" + scheme], S["n_mu"])
        toy.sweep(scheme, mus[:2], ladder[:2], S["n_samples"], S["periods"])     # warm-up
        tm = Timer()
        r = toy.sweep(scheme, mus, ladder, S["n_samples"], S["periods"], timer=tm)
        ms = tm.ms()
        pick = slice(None, None, max(1, S["n_mu"] // 16))
        out[scheme] = {
            "kernel_ms": round(ms, 3), "n_traj": r["n_traj"], "rk4_steps": r["rk4_steps"],
            "rk4_steps_per_s": r["rk4_steps"] / (ms * 1e-3),
            "longest_trajectory_steps": S["n_samples"] * ladder[-1],
            "mu": [round(float(x), 5) for x in r["mu"][pick]],
            "d_R": [float(f"{x:.4g}") for x in r["d_R"][pick]],
            "d_F": [float(f"{x:.4g}") for x in r["d_F"][pick]],
            "dt_max": [None if not np.isfinite(x) else float(f"{x:.4g}") for x in r["dt_max"][pick]],
        }
    if oracle_sample:
        from oracle import toy as T
        P = T.ToyParams(**W.TOY_N2)
        t_total = S["periods"] * P.period_R
        sub = 16
        t0 = time.perf_counter()
        T.run(P, "ehrenfest", [1.0], sub, S["n_samples"], t_total)
        el = time.perf_counter() - t0
        out["cpu_oracle"] = {"rk4_steps_per_s": S["n_samples"] * sub / el, "cores": 1, "kind": "oracle",
                             "sample": f"one Ehrenfest trajectory, {S['n_samples'] * sub} RK4 steps"}
    return out


def run_variants(steps: int = 20) -> dict:
    """The propagator and force variants on the 96^3 x 128 FP32 workload:
    AETRS, ETRS with one and two corrections, the wave-function-gradient
    nonlocal force."""
    import workloads as W
    out = {"workload": "96^3 h=0.25, 64 ions, 128 FP32 orbitals", "steps": steps}
    for name, over in (("aetrs", {}), ("etrs_1", {"etrs_iterations": 1}), ("etrs_2", {"etrs_iterations": 2}),
                       ("aetrs_gradient_force", {"nl_force_form": 1})):
        out[name + "_ms_per_step"] = round(time_scheme(W.C2, "ehrenfest", steps, **over), 4)
    return out


def run_finite(steps: int = 50) -> dict:
    """The finite-box workload (the 72^3 ring box): ms per MD step in FP32 and
    FP64, beside the same grid run as a periodic cube."""
    import torch
    import workloads as W
    from paper_0812_2801_amd import binding as B
    cfg = W.F3
    inp = W.make_inputs(cfg)
    out = {"workload": f"{cfg.n}^3 h={cfg.h}, {cfg.n_ions}-atom ring, {cfg.n_orb} orbitals, box of "
                       f"{cfg.finite_radius} b spheres",
           "box_fraction": float(W.box_mask(cfg, inp["pos"]).mean()), "steps": steps}
    psi = torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1))
    for prec in ("f32", "f64"):
        for kind, c in (("finite", cfg), ("periodic", cfg.replace(finite_radius=0.0))):
            p, keep = B.params_from_config(c, inp["pos"], precision=prec)
            s = B.System(p, keep, device="cuda:0")
            s.set_state(psi)
            e0 = s.report()["e_total"]
            for _ in range(3):
                s.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                s.step()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            rep = s.report()
            s.close()
            out[f"{kind}_{prec}_ms_per_step"] = round(ms, 4)
            out[f"{kind}_{prec}_energy_change"] = rep["e_total"] - e0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sample", type=int, default=4, help="orbitals in the oracle sample")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--precision", default="f32", choices=["f32", "f32_bf16x3", "f64"])
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 16-system run")
    ap.add_argument("--batch-steps", type=int, default=48)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched workload (profiling)")
    ap.add_argument("--no-cp", action="store_true", help="skip the Car-Parrinello comparison")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the finite-box and toy-model summaries of the default run")
    ap.add_argument("--cp-steps", type=int, default=20)
    ap.add_argument("--cp-series", action="store_true", help="add the system-size series of both schemes")
    ap.add_argument("--cp-only", action="store_true",
                    help="only the Car-Parrinello comparison (Ehrenfest timed at the same sizes)")
    ap.add_argument("--dt-scan", action="store_true",
                    help="only the largest stable time step against the grid spacing (Taylor-4, Taylor-8, CP)")
    ap.add_argument("--variants", action="store_true",
                    help="only the propagator / force variants (ETRS, gradient-form force) on the 96^3 workload")
    ap.add_argument("--finite", action="store_true",
                    help="only the finite-box workload (union of atom-centred spheres, free-space Hartree)")
    ap.add_argument("--c4-only", action="store_true",
                    help="run only the 128^3 x 432 precision-study workload (profiling)")
    ap.add_argument("--no-c4", action="store_true", help="skip the 128^3 x 432 workload")
    ap.add_argument("--c4-precisions", default="f32,f32_bf16x3,f64",
                    help="comma-separated precisions of the 128^3 x 432 workload")
    ap.add_argument("--toy", action="store_true",
                    help="only the two-band toy-model sweep (d_R, d_F, Delta t_max against the mass)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.batch_only:           # profiling aid: the batched workload alone
        print(json.dumps({"batched": run_batch(args.batch_steps, 8, 6, not args.no_autotune)}))
        return
    if args.variants:
        print(json.dumps({"variants": run_variants()}))
        return
    if args.finite:
        print(json.dumps({"finite_box": run_finite()}))
        return
    if args.toy:
        print(json.dumps({"toy_model": run_toy(not args.no_cpu)}))
        return
    if args.c4_only:
        print(json.dumps({"precision_study_128": run_c4(args.steps, args.warmup,
                                                        tuple(args.c4_precisions.split(",")))}))
        return
    if args.dt_scan:
        from paper_0812_2801_amd import scan
        print(json.dumps({"dt_max_vs_spacing": scan.spacing_series(), "dt_max_vs_mass": scan.mass_series()}))
        return
    if args.cp_only:
        import workloads as W
        e_ms = time_scheme(W.C2, "ehrenfest", args.cp_steps)
        print(json.dumps({"cp": run_cp(args.cp_steps, e_ms, args.cp_series)}))
        return

    import numpy as np
    import torch
    import workloads as W
    cfg = W.C2
    t_gen = time.perf_counter()
    inp = W.make_inputs(cfg)
    t_gen = time.perf_counter() - t_gen
    print(f"# inputs generated in {t_gen:.1f} s", file=sys.stderr, flush=True)
    sample = list(range(min(args.sample, cfg.n_orb)))
    work = cfg.n_orb * cfg.n_points * 8          # orbital*gridpoint*H psi per step

    main_run = run_precision(cfg, inp, args.precision, args.steps, args.warmup, sample)
    print(f"# {args.precision}: {main_run['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    f64_run = None
    if not args.no_fp64 and args.precision != "f64":
        f64_run = run_precision(cfg, inp, "f64", max(10, args.steps // 4), args.warmup, sample)
        print(f"# f64: {f64_run['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    bf_run = None
    if not args.no_fp64 and args.precision == "f32":
        bf_run = run_precision(cfg, inp, "f32_bf16x3", max(10, args.steps // 4), args.warmup, sample)
        print(f"# f32_bf16x3: {bf_run['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    batch = None
    if not args.no_batch:
        batch = run_batch(args.batch_steps, 8, 6, not args.no_autotune)
        print(f"# batch: {batch['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    cp_run = None
    if not args.no_cp:
        cp_run = run_cp(args.cp_steps, main_run["ms_per_step"], args.cp_series)
        print(f"# cp: {cp_run['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    c4 = None
    if not args.no_c4:
        c4 = run_c4()

    adj = None
    if not args.no_adjoint:
        adj = run_adjoint()
        print(f"# adjoint: forward {adj['forward_ms']:.1f} ms, backward {adj['backward_ms']:.1f} ms",
              file=sys.stderr, flush=True)

    extras = {}
    if not args.no_extras:
        # the finite-box and toy-model studies, summarised; a failure there is
        # recorded and does not cost the headline line
        for key, fn in (("finite_box", lambda: run_finite(20)), ("toy_model", lambda: run_toy(not args.no_cpu))):
            try:
                extras[key] = fn()
            except Exception as e:          # noqa: BLE001
                extras[key] = {"error": f"{type(e).__name__}: {e}"}
            print(f"# {key} done", file=sys.stderr, flush=True)

    cpu = None
    errors = {}
    if not args.no_cpu:
        n_cpu = min(cfg.n_orb, max(len(sample), 2 * min(16, len(os.sched_getaffinity(0)))))
        ref_all, t_cpu, cores = oracle_sample(cfg, inp, n_cpu)
        ref = ref_all[:len(sample)].reshape(len(sample), -1)
        errors[args.precision] = float(np.abs(main_run["psi_sample"] - ref).max())
        if f64_run is not None:
            errors["f64"] = float(np.abs(f64_run["psi_sample"] - ref).max())
        if bf_run is not None:
            errors["f32_bf16x3"] = float(np.abs(bf_run["psi_sample"] - ref).max())
        cpu_work = n_cpu * cfg.n_points * 8
        cpu = {"value": cpu_work / t_cpu, "unit": "orbital·gridpt·Hψ/s", "cores": cores,
               "kind": "oracle", "cpu": cpu_model(),
               "sample": f"one AETRS propagation (8 H psi) of {n_cpu} of the 128 orbitals of the 96^3 "
                         f"workload, FP64 NumPy, {cores} worker processes of one thread each "
                         f"(orbital-parallel oracle driver), {t_cpu:.1f} s wall, "
                         f"{cores * t_cpu:.0f} core-s"}

    ms = main_run["ms_per_step"]
    value = work / (ms * 1e-3)
    # the dominant kernel: the three-stream Horner stage (six of the eight
    # stencil launches of a step); the two-stream first stages beside it
    n3, ms3, by3 = main_run["kinds"][3]
    n2, ms2, by2 = main_run["kinds"][2]
    avg_ms = ms3 / max(1, n3)
    avg_bytes = by3 / max(1, n3)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    tname = "void me::stencil_kernel<float, 1, 8, 1, false>" if args.precision != "f64" else \
        "void me::stencil_kernel<double, 1, 8, 1, false>"
    traffic = traffic_entry(tname)
    all_ms = main_run["kernel_ms"] / max(1, main_run["launches"])
    all_bytes = main_run["kernel_bytes"] / max(1, main_run["launches"])
    streams = device_streams(cfg.n_orb * cfg.n_points * 8)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "orbital·gridpt·Hψ/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": "single system: 96^3 grid h=0.25, 64 ions Z=4 (uniform, min sep 2.5), "
                               "128 complex orbitals, mu=4, dt=0.08, AETRS+Taylor-4, whole MD step",
                   "precision": args.precision, "grid": 96, "n_orb": cfg.n_orb, "n_ions": cfg.n_ions,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "stencil_kernel, three-stream Horner stage (read u_k and psi, write u_k-1; "
                               "6 of the 8 stencil launches of a step)",
                     "kernel_avg_ms": avg_ms, "algorithmic_bytes_per_launch": avg_bytes, "launches": n3,
                     "first_stage": {"kernel_avg_ms": ms2 / max(1, n2),
                                     "algorithmic_bytes_per_launch": by2 / max(1, n2),
                                     "achieved": (by2 / max(1, n2)) / (ms2 / max(1, n2) * 1e-3) / 1e9 if n2 else None},
                     "all_stages": {"kernel_avg_ms": all_ms, "achieved": all_bytes / (all_ms * 1e-3) / 1e9},
                     "device_streams_GBps": streams},
        "cpu_baseline": cpu,
        "errors_vs_fp64_oracle_one_step": errors,
        "energy_drift": {"total": main_run["energy_drift"], "e_start": main_run["e_start"],
                         "steps": main_run["steps_total"],
                         "max_norm_dev": main_run["report"]["max_norm_dev"]},
    }
    if f64_run is not None:
        out["fp64"] = {"ms_per_step": f64_run["ms_per_step"],
                       "value": work / (f64_run["ms_per_step"] * 1e-3),
                       "stencil_avg_ms": f64_run["kernel_ms"] / max(1, f64_run["launches"])}
        out["speedup_vs_fp64"] = f64_run["ms_per_step"] / ms
    if bf_run is not None:
        out["f32_bf16x3"] = {"ms_per_step": bf_run["ms_per_step"],
                             "value": work / (bf_run["ms_per_step"] * 1e-3),
                             "stencil_avg_ms": bf_run["kernel_ms"] / max(1, bf_run["launches"])}
    if adj is not None:
        out["adjoint"] = adj
    if c4 is not None:
        out["precision_study_128"] = c4
    if cp_run is not None:
        out["cp"] = cp_run
    if batch is not None:
        out["batched"] = batch
        out["batched_vs_single_system"] = batch["value"] / value
    if "toy_model" in extras and "error" not in extras["toy_model"]:
        t = extras["toy_model"]
        extras["toy_model"] = {k: t[k] for k in ("workload", "cpu_oracle") if k in t}
        for sch in ("ehrenfest", "cp"):
            extras["toy_model"][sch] = {k: t[sch][k] for k in ("kernel_ms", "n_traj", "rk4_steps", "rk4_steps_per_s")}
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
