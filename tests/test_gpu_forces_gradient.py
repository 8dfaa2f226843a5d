"""The wave-function-gradient form of the nonlocal force (the footnote of
sec. 5.1, nl_force_form = 1) on the GPU against the oracle's, and its
distance from the analytic projector derivative."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_gradient_form_forces_match_oracle(prec, tol):
    import torch
    from oracle import Model, dynamics
    from paper_0812_2801_amd import binding as B
    cfg = W.C1.replace(name="g32", n=32, h=0.25, n_orb=12, n_ions=6, placement="lattice", jitter=0.2, seed=321)
    inp = W.make_inputs(cfg)
    out = {}
    for form in (0, 1):
        p, keep = B.params_from_config(cfg, inp["pos"], precision=prec, nl_force_form=form)
        s = B.System(p, keep)
        s.set_state(torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1)))
        out[form] = s.forces()
        s.close()
    m = Model.from_config(cfg)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    want = m.forces(st.pos, st.psi, st.rho, nl_form="gradient")["total"]
    d = np.abs(out[1].reshape(want.shape) - want).max()
    dab = np.abs(out[1] - out[0]).max()
    note(f"{prec}: gradient form max|dF| vs oracle {d:.2e}; gradient vs analytic form {dab:.2e}")
    assert d < tol
    assert 0.0 < dab < 0.1 * np.abs(want).max()
