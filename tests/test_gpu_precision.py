"""Precision study at the full 128^3 shape (216 ions on a jittered lattice,
432 orbitals, mu = 4, dt = 0.08).

1. One AETRS step in FP32 and in FP32 with the split-bf16 projector
   contraction, against the FP64 CPU oracle on sampled orbitals.  The oracle
   builds H(t) and H(t+dt) from the density of all 432 orbitals and
   propagates the sampled ones; the ions are frozen so that the step needs no
   forces of the full set.
2. Twenty steps with moving ions in FP32, FP32 + bf16x3 and FP64 on the GPU
   (each timed): the per-step distance of the sampled orbitals from the FP64
   run (a report of how the reduced-precision error grows, bounded loosely).

The oracle part alone takes about two minutes of one CPU core, so the test
runs only with MODEHR_FULL_SHAPE=1."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("MODEHR_FULL_SHAPE") != "1",
                                 reason="full 128^3 x 432 shape: set MODEHR_FULL_SHAPE=1 (about 4 minutes)")]

SAMPLE = [0, 431]


def _system(cfg, pos, prec, psi_dev):
    from paper_0812_2801_amd import binding as B
    p, keep = B.params_from_config(cfg, pos, precision=prec)
    s = B.System(p, keep)
    s.set_state(psi_dev)
    return s


def _sample(s):
    return to_np(s.get_state()[SAMPLE])


def test_c4_shape_precision():
    import torch
    from oracle import Model, dynamics
    cfg = W.C4
    note("c4 shape: orbitals on the device")
    psi_dev = W.initial_orbitals_device(cfg, "cuda:0")
    pos = W.ion_positions(cfg)

    # 2. twenty steps, moving ions, each precision on its own (timed), the
    #    sampled orbitals kept after every step
    import time
    traj = {}
    for prec in ("f64", "f32", "f32_bf16x3"):
        s = _system(cfg, pos, prec, psi_dev)
        s.step()                                  # first step: code objects, plans
        torch.cuda.synchronize()
        samples = [_sample(s)]
        elapsed = 0.0
        for n in range(cfg.steps - 1):
            t0 = time.perf_counter()
            s.step()
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            samples.append(_sample(s))
        note(f"  {prec}: {1e3 * elapsed / (cfg.steps - 1):.2f} ms per MD step")
        traj[prec] = samples
        s.close()
        del s
        torch.cuda.empty_cache()
    worst = {}
    for prec in ("f32", "f32_bf16x3"):
        d = [float(np.abs(a - b).max()) for a, b in zip(traj[prec], traj["f64"])]
        worst[prec] = max(d)
        note(f"  {prec} vs f64, steps 1..{cfg.steps}: " + " ".join(f"{x:.1e}" for x in d))
    assert max(worst.values()) < 1e-3

    # 1. one step against the oracle, frozen ions
    frozen = cfg.replace(freeze_ions=True)
    got = {}
    for prec in ("f32", "f32_bf16x3"):
        s = _system(frozen, pos, prec, psi_dev)
        s.step()
        got[prec] = _sample(s)
        s.close()
        del s
        torch.cuda.empty_cache()
    note("  oracle: H(t), H(t+dt) from all 432 orbitals")
    psi = to_np(psi_dev).reshape(cfg.n_orb, cfg.n, cfg.n, cfg.n)
    del psi_dev
    torch.cuda.empty_cache()
    m = Model.from_config(frozen)
    st = dynamics.init_state(m, psi, pos)
    _, h0, h1 = dynamics.step_hamiltonians(m, st)
    ref = dynamics.propagate_orbitals(m, psi[SAMPLE], h0, h1).reshape(len(SAMPLE), -1)
    for prec, g in got.items():
        err = float(np.abs(g - ref).max())
        note(f"  one step vs oracle, {prec}: max|dpsi| {err:.3e} (max|psi| {np.abs(ref).max():.3e})")
        assert err < 1e-4
