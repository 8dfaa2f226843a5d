"""Parity at the benchmark's own configuration: the 96^3 system with 64 ions
and 128 FP32 orbitals, one AETRS step in the launch configuration bench.py
times, against the FP64 CPU oracle on two sampled orbitals.  The oracle
builds H(t) and H(t+dt) from the density of all 128 orbitals and propagates
the sampled ones; the ions are frozen so that the step needs no forces of
the full set (about half a minute of one CPU core)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu

SAMPLE = [0, 127]


def test_bench_shape_one_step_vs_oracle():
    import torch
    from oracle import Model, dynamics
    from paper_0812_2801_amd import binding as B
    cfg = W.C2.replace(freeze_ions=True)
    psi_dev = W.initial_orbitals_device(cfg, "cuda:0")
    pos = W.ion_positions(cfg)
    got = {}
    for prec in ("f32", "f32_bf16x3"):
        note(f"bench shape {cfg.n}^3 x {cfg.n_orb} {prec}: one step on the GPU")
        p, keep = B.params_from_config(cfg, pos, precision=prec)
        s = B.System(p, keep)
        s.set_state(psi_dev)
        s.step()
        got[prec] = to_np(s.get_state()[SAMPLE])
        s.close()
        del s
    psi = to_np(psi_dev).reshape(cfg.n_orb, cfg.n, cfg.n, cfg.n)
    del psi_dev
    torch.cuda.empty_cache()
    note("  oracle: density of all orbitals, H(t), H(t+dt)")
    m = Model.from_config(cfg)
    st = dynamics.init_state(m, psi, pos)
    _, h0, h1 = dynamics.step_hamiltonians(m, st)
    note("  oracle: propagating the sampled orbitals")
    ref = dynamics.propagate_orbitals(m, psi[SAMPLE], h0, h1).reshape(len(SAMPLE), -1)
    for prec, g in got.items():
        err = float(np.abs(g - ref).max())
        note(f"  {prec}: max|dpsi| {err:.3e} (max|psi| {np.abs(ref).max():.3e})")
        assert err < 1e-4
