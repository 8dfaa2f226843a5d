"""A batch with a row wider than 192 points: a 200^3 system (x-tiles of 64
points in the persistent stencil) beside a 24^3 one (whole rows).  Each
system after two steps against the same system run alone (the same
arithmetic per point, so the orbitals agree to rounding), and the 200^3
system after one FP64 step against the oracle."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu

WIDE = W.C1.replace(name="wide200", n=200, h=0.25, n_ions=8, n_orb=2, placement="lattice", jitter=0.5,
                    seed=20001)
SMALL = W.C1.replace(name="small24", n=24, h=0.3, n_ions=3, n_orb=3, placement="lattice", jitter=0.2,
                     seed=20002)


def _run(cfgs, prec, steps, batch):
    import torch
    from paper_0812_2801_amd import binding as B
    out = []
    params, keep, psis = [], [], []
    for c in cfgs:
        p, k = B.params_from_config(c, W.ion_positions(c), precision=prec)
        params.append(p)
        keep.append(k)
        psis.append(W.initial_orbitals_device(c, "cuda:0"))
    if batch:
        b = B.Batch(params, keep, device="cuda:0")
        assert b.tuning()["block"] >= 64
        for s, psi in zip(b.systems, psis):
            s.set_state(psi)
        b.propagate(steps, use_graph=False)
        out = [(to_np(s.get_state()), s.forces()) for s in b.systems]
        b.close()
    else:
        for p, k, psi in zip(params, keep, psis):
            s = B.System(p, k)
            s.set_state(psi)
            for _ in range(steps):
                s.step()
            out.append((to_np(s.get_state()), s.forces()))
            s.close()
    return out, [to_np(p) for p in psis]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_wide_row_batch_matches_systems_alone(prec):
    note(f"wide-row batch {prec}")
    got, _ = _run([WIDE, SMALL], prec, 2, batch=True)
    want, _ = _run([WIDE, SMALL], prec, 2, batch=False)
    tol = 1e-12 if prec == "f64" else 2e-6
    for c, (pg, fg), (pw, fw) in zip((WIDE, SMALL), got, want):
        d = float(np.abs(pg - pw).max())
        df = float(np.abs(fg - fw).max())
        note(f"  {c.name}: batch vs alone max|dpsi| {d:.2e} max|dF| {df:.2e}")
        assert d <= tol and df <= 1e3 * tol


def test_wide_row_batch_step_matches_oracle():
    from oracle import Model, dynamics
    note("wide-row batch f64, one frozen-ion step vs the oracle (orbital 0)")
    c = WIDE.replace(freeze_ions=True)
    got, psi0 = _run([c, SMALL], "f64", 1, batch=True)
    psi = psi0[0].reshape((c.n_orb,) + (c.n,) * 3)
    m = Model.from_config(c)
    pos = W.ion_positions(c)
    rho = m.density(psi)
    # the step's Hamiltonians need the density of both orbitals; the ions do
    # not move, so no forces are needed to build them
    st = dynamics.State(psi=psi, pos=pos, vel=np.zeros_like(pos), force=np.zeros_like(pos), rho=rho,
                        hist=[m.v_hxc(rho)])
    _, h0, h1 = dynamics.step_hamiltonians(m, st)
    ref = dynamics.propagate_orbitals(m, psi[:1], h0, h1).reshape(-1)
    d = float(np.abs(got[0][0][0] - ref).max())
    note(f"  {c.name}: orbital 0 max|dpsi| {d:.2e} (max|psi| {np.abs(ref).max():.2e})")
    assert d <= 1e-10
