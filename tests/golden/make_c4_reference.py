"""Write tests/golden/c4_oracle_trajectory.npz: the FP64 oracle's trajectory
of the precision workload (128^3 grid, h = 0.25, 216 ions on a jittered
lattice, 432 orbitals from per-orbital streams, mu = 4, dt = 0.08, AETRS
with Taylor-4, moving ions, 20 steps).

For the state after every step n = 0..20 it stores the energy parts and the
total energy (eq. E_KS, eq. E_new), the forces, positions and velocities of
the ions, and the orbitals at a seeded sample of (orbital, point) pairs, so a
GPU run of the same inputs can be compared with the oracle step by step.

Calls only the oracle (its orbital-parallel driver) and the input
generators.  About two hours on 8 cores; the file is rewritten after every
step.  Usage: python tests/golden/make_c4_reference.py [workers]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import Model  # noqa: E402
from oracle.parallel import Driver  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_oracle_trajectory.npz")
SAMPLE_ORBITALS = (0, 144, 288, 431)
POINTS_PER_ORBITAL = 192
PARTS = ("kinetic", "local", "hartree", "xc", "nonlocal", "ion", "ion_kinetic")


def sample_points(cfg):
    rng = np.random.default_rng(np.random.SeedSequence([cfg.seed, 555]))
    return np.stack([np.sort(rng.choice(cfg.n_points, POINTS_PER_ORBITAL, replace=False))
                     for _ in SAMPLE_ORBITALS])


def main(workers=None):
    cfg = W.C4
    m = Model.from_config(cfg)
    pts = sample_points(cfg)
    orbs = np.array(SAMPLE_ORBITALS)
    rec = {k: [] for k in ("e_total", "e_ks", "e_parts", "force", "pos", "vel", "psi", "max_abs_psi")}
    t0 = time.time()
    with Driver(m, cfg.n_orb, workers=workers) as d:
        W.initial_orbitals_streamed(cfg, out=d.psi)
        print(f"inputs: {time.time() - t0:.0f} s", flush=True)
        st = d.init_state(d.psi, W.ion_positions(cfg))
        for n in range(cfg.steps + 1):
            if n > 0:
                st = d.aetrs_step(st)
            e = d.total_energy(st)
            flat = d.psi.reshape(cfg.n_orb, -1)
            rec["e_total"].append(e["total"])
            rec["e_ks"].append(e["ks"])
            rec["e_parts"].append([e[k] for k in PARTS])
            rec["force"].append(st.force.copy())
            rec["pos"].append(st.pos.copy())
            rec["vel"].append(st.vel.copy())
            rec["psi"].append(np.stack([flat[a, pts[i]] for i, a in enumerate(orbs)]))
            rec["max_abs_psi"].append(float(np.abs(flat[orbs]).max()))
            np.savez_compressed(
                OUT + ".tmp.npz", sample_orbitals=orbs, sample_points=pts, parts=np.array(PARTS),
                n=cfg.n, h=cfg.h, n_orb=cfg.n_orb, n_ions=cfg.n_ions, mu=cfg.mu, dt=cfg.dt,
                seed=cfg.seed, recipe=np.array("initial_orbitals_streamed"),
                steps_done=n, **{k: np.array(v) for k, v in rec.items()})
            os.replace(OUT + ".tmp.npz", OUT)
            print(f"step {n}: E = {e['total']:.10f}, max|F| = {np.abs(st.force).max():.6f}, "
                  f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else None)
