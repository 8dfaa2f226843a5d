"""The 16-system batched workload at its own scale (grids 32^3-96^3, 8-256
orbitals, 934 M orbital points, FP32, frozen ions) against the FP64 oracle.

* One eager step of the whole batch (one persistent stencil launch per
  Horner stage over every system): sampled orbitals of the largest grid
  (96^3, 200 orbitals) and of the smallest (32^3, 256 orbitals, 54 ions)
  against the oracle's step of those orbitals, H(t) and H(t+dt) built from
  the density of all of that system's orbitals.
* Seven more steps, six of them replayed from the captured hipGraph: every
  orbital of the 32^3 system against the oracle's full eight-step
  trajectory (the orbital-parallel oracle driver).

The orbitals come from the input generator on the device in FP64 and are
rounded once to FP32; the oracle starts from the same FP32 values."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu

LARGE, SMALL = 1, 13          # c3_sys01_96 (96^3, 200 orbitals), c3_sys13_32 (32^3, 256 orbitals)
SAMPLE = {LARGE: [0, 199], SMALL: [0, 137, 255]}


def _oracle_one_step(cfg, psi, sample):
    from oracle import Model, dynamics
    m = Model.from_config(cfg)
    st = dynamics.init_state(m, psi, W.ion_positions(cfg))
    _, h0, h1 = dynamics.step_hamiltonians(m, st)
    return dynamics.propagate_orbitals(m, psi[sample], h0, h1).reshape(len(sample), -1)


def test_batch_full_scale_against_oracle():
    import os
    import torch
    from oracle import Model
    from oracle.parallel import Driver
    from paper_0812_2801_amd import binding as B
    cfgs = [c.replace(freeze_ions=True) for c in W.batch_configs(16)]
    assert (cfgs[LARGE].n, cfgs[LARGE].n_orb) == (96, 200) and (cfgs[SMALL].n, cfgs[SMALL].n_orb) == (32, 256)
    params, keep = [], []
    for c in cfgs:
        p, k = B.params_from_config(c, W.ion_positions(c), precision="f32")
        params.append(p)
        keep.append(k)
    b = B.Batch(params, keep, device="cuda:0")
    psi0 = {}
    for i, (s, c) in enumerate(zip(b.systems, cfgs)):
        psi = W.initial_orbitals_device(c, "cuda:0").to(torch.complex64)
        if i in SAMPLE:
            psi0[i] = to_np(psi).astype(np.complex128).reshape((c.n_orb,) + (c.n,) * 3)
        s.set_state(psi)
        del psi
    note("c3 batch: 16 systems on the device, one eager step")
    b.propagate(1, use_graph=False)
    got1 = {i: to_np(b.systems[i].get_state()[SAMPLE[i]]) for i in SAMPLE}
    for i in SAMPLE:
        ref = _oracle_one_step(cfgs[i], psi0[i], SAMPLE[i])
        err = float(np.abs(got1[i] - ref).max())
        note(f"  {cfgs[i].name}: one step, orbitals {SAMPLE[i]}: max|dpsi| {err:.2e} "
             f"(max|psi| {np.abs(ref).max():.2e})")
        assert err < 1e-4

    note("c3 batch: seven more steps (six from the graph)")
    b.propagate(7, use_graph=True)
    got8 = to_np(b.systems[SMALL].get_state())
    c = cfgs[SMALL]
    m = Model.from_config(c)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with Driver(m, c.n_orb, workers=workers, orbitals_per_task=4) as d:
        st = d.init_state(psi0[SMALL], W.ion_positions(c))
        for _ in range(8):
            st = d.aetrs_step(st)
        ref = d.psi.reshape(c.n_orb, -1).copy()
    err = float(np.abs(got8 - ref).max())
    note(f"  {c.name}: eight steps (graph replay), all {c.n_orb} orbitals: max|dpsi| {err:.2e} "
         f"(max|psi| {np.abs(ref).max():.2e})")
    assert err < 8e-4
    b.close()
