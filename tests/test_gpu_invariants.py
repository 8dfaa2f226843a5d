"""Invariants of the method on the GPU path (FP64), the same properties the
oracle is pinned to in test_oracle_dynamics.py:

* the orthonormality defect (eq. escpro) and the total-energy drift
  (eq. E_new) shrink with dt at the orders of Taylor-4 / AETRS;
* AETRS is time-reversible up to the Taylor truncation: dt steps followed by
  -dt steps return close to the start, closer for smaller dt, and the GPU's
  residual equals the oracle's.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu


def _system(cfg, dt=None):
    import torch
    from paper_0812_2801_amd import binding as B
    inp = W.make_inputs(cfg)
    over = {} if dt is None else {"dt": dt}
    p, keep = B.params_from_config(cfg, inp["pos"], precision="f64", **over)
    s = B.System(p, keep)
    s.set_state(torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1)))
    return s, inp


def _overlap_defect(s, h):
    import torch
    psi = s.get_state()
    S = (h ** 3) * (psi.conj() @ psi.T)
    return float((S - torch.eye(S.shape[0], dtype=S.dtype, device=S.device)).abs().max())


def test_orthonormality_and_energy_drift_shrink_with_dt():
    cfg = W.C2.replace(n=32, n_ions=8, n_orb=16, mu=1.0, seed=4242, precision="f64")
    errs, drifts = [], []
    for dt, ns in ((0.02, 10), (0.01, 20)):
        s, _ = _system(cfg, dt=dt)
        e0 = s.report()["e_total"]
        worst = 0.0
        for _ in range(ns):
            s.step()
            worst = max(worst, _overlap_defect(s, cfg.h))
        drift = abs(s.report()["e_total"] - e0)
        note(f"  dt {dt}: max orthonormality defect {worst:.3e}, |energy drift| {drift:.3e}")
        errs.append(worst)
        drifts.append(drift)
        s.close()
    # Taylor-4 leaves a norm defect ~ (tau |H|)^6 per step on the fastest
    # components: small, and at least 8x smaller at half the step
    assert errs[0] < 1e-5
    assert errs[1] < errs[0] / 8
    assert drifts[1] < drifts[0] / 3


def test_time_reversal_matches_the_oracle():
    from oracle import Model, dynamics
    res = []
    for dt in (0.02, 0.01):
        cfg = W.C1.replace(dt=dt, seed=4343)
        fwd, inp = _system(cfg)
        for _ in range(4):
            fwd.step()
        buf = fwd.new_checkpoint()
        fwd.save_checkpoint(buf)
        back, _ = _system(cfg, dt=-dt)
        back.load_checkpoint(buf)
        for _ in range(4):
            back.step()
        psi = to_np(back.get_state()).reshape(inp["psi"].shape)
        pos, _ = back.ions()
        d_psi = float(np.abs(psi - inp["psi"]).max())
        d_pos = float(np.abs(pos - inp["pos"]).max())
        # the same round trip in the oracle
        m = Model.from_config(cfg)
        st = dynamics.init_state(m, inp["psi"], inp["pos"])
        for _ in range(4):
            st = dynamics.aetrs_step(m, st)
        mb = Model.from_config(cfg, dt=-dt)
        sb = dynamics.State(psi=st.psi, pos=st.pos, vel=st.vel, force=st.force, rho=st.rho, hist=list(st.hist))
        for _ in range(4):
            sb = dynamics.aetrs_step(mb, sb)
        note(f"  dt {dt}: GPU return error psi {d_psi:.3e} pos {d_pos:.3e}; "
             f"oracle psi {np.abs(sb.psi - inp['psi']).max():.3e}; |GPU - oracle| {np.abs(psi - sb.psi).max():.2e}")
        assert np.abs(psi - sb.psi).max() < 1e-9
        assert np.abs(pos - sb.pos).max() < 1e-11
        res.append((d_psi, d_pos))
        fwd.close()
        back.close()
    assert res[0][0] < 1e-2 and res[1][0] < res[0][0] / 2
    assert res[1][1] < res[0][1]
