"""Precision study at the full 128^3 shape (216 ions on a jittered lattice,
432 orbitals, mu = 4, dt = 0.08, moving ions, 20 AETRS steps) against the
FP64 CPU oracle, step by step.

The oracle's trajectory of the same seeded inputs is stored in
tests/golden/c4_oracle_trajectory.npz (written by make_c4_reference.py
beside it, which calls only the oracle): after every step the energy, the
forces and the orbitals at 4 x 192 sampled (orbital, point) pairs.  The GPU
runs the workload in FP64, FP32 and FP32 with the split-bf16 projector
contraction, each from the same FP64 orbitals, and after every step reports
max|dpsi| at the sampled pairs, the total-energy error dE and max|dF|
against the oracle, and the distance of all 432 orbitals from the FP64 GPU
run.

Gates (per step n, errors that may grow with n):
  FP64        max|dpsi| <= 1e-10, |dE| <= 1e-8 |E|, max|dF| <= 1e-8
  FP32, bf16  max|dpsi| <= 1e-4 (the one-step bound, not compounded),
              |dE| <= 1e-5 |E| (n * 8 stages * 2^-24 is 1e-5 at n = 20),
              max|dF| <= 1e-4 (forces are O(0.3) hartree/bohr)
"""
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import note

pytestmark = pytest.mark.gpu

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_oracle_trajectory.npz")
PRECS = ("f64", "f32", "f32_bf16x3")
GATE = {"f64": (1e-10, 1e-8, 1e-8), "f32": (1e-4, 1e-5, 1e-4), "f32_bf16x3": (1e-4, 1e-5, 1e-4)}


def test_c4_precision_study_against_oracle():
    import torch
    from paper_0812_2801_amd import binding as B
    cfg = W.C4
    ref = np.load(REF, allow_pickle=False)
    n_ref = int(ref["steps_done"])
    assert (int(ref["n"]), int(ref["n_orb"]), int(ref["n_ions"])) == (cfg.n, cfg.n_orb, cfg.n_ions)
    orbs = ref["sample_orbitals"]
    pts = torch.from_numpy(ref["sample_points"]).to("cuda:0")
    note(f"c4: orbitals on the device (reference: {n_ref} steps)")
    psi = W.initial_orbitals_streamed_device(cfg, "cuda:0")
    pos = W.ion_positions(cfg)
    systems = {}
    for prec in PRECS:
        p, keep = B.params_from_config(cfg, pos, precision=prec)
        s = B.System(p, keep)
        s.set_state(psi)
        systems[prec] = s
    del psi
    torch.cuda.empty_cache()

    def sampled(st):
        rows = st[torch.from_numpy(orbs).to(st.device)]
        return torch.gather(rows, 1, pts).cpu().numpy().astype(np.complex128)

    rows = []
    worst = {p: [0.0, 0.0, 0.0] for p in PRECS}
    for n in range(n_ref + 1):
        states, line = {}, [n]
        for prec, s in systems.items():
            rep = s.report() if n == 0 else s.step(report=True)
            st = s.get_state()
            dpsi = float(np.abs(sampled(st) - ref["psi"][n]).max())
            de = rep["e_total"] - float(ref["e_total"][n])
            df = float(np.abs(s.forces() - ref["force"][n]).max())
            states[prec] = st
            line += [dpsi, de, df]
            g = GATE[prec]
            scale_e = abs(float(ref["e_total"][n]))
            assert dpsi <= g[0] and abs(de) <= g[1] * scale_e and df <= g[2], (n, prec, dpsi, de, df)
            w = worst[prec]
            worst[prec] = [max(w[0], dpsi), max(w[1], abs(de)), max(w[2], df)]
        d64 = states["f64"].to(torch.complex128)
        line += [float((states[p].to(torch.complex128) - d64).abs().max()) for p in ("f32", "f32_bf16x3")]
        del states, d64
        rows.append(line)
        note(f"  step {n:2d} | " + " | ".join(
            f"{p}: dpsi {line[1 + 3 * i]:.1e} dE {line[2 + 3 * i]:+.1e} dF {line[3 + 3 * i]:.1e}"
            for i, p in enumerate(PRECS)) + f" | all orbitals vs f64 GPU: f32 {line[-2]:.1e} bf16x3 {line[-1]:.1e}")
    for prec in PRECS:
        note(f"  worst {prec}: max|dpsi| {worst[prec][0]:.2e}, max|dE| {worst[prec][1]:.2e}, "
             f"max|dF| {worst[prec][2]:.2e} (max|psi| {float(np.max(ref['max_abs_psi'])):.2e}, "
             f"E {float(ref['e_total'][0]):.4f})")
    for s in systems.values():
        s.close()
    assert n_ref == cfg.steps, f"the stored oracle trajectory holds {n_ref} of {cfg.steps} steps"
