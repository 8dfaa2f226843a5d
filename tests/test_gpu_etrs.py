"""ETRS on the GPU (etrs_iterations > 0: the second exponential of the step
redone with v_Hxc of the density it produces, sec. 5.1) against the oracle's
etrs_step, under a field and with moving ions.  The ETRS-AETRS difference is
printed beside the error so that the tolerance visibly separates the two."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu

CFG = W.C1.replace(name="e32", n=32, h=0.25, n_orb=5, n_ions=6, placement="lattice", jitter=0.3, seed=3202)


@pytest.mark.parametrize("prec,tol_psi,tol_f", [("f64", 1e-10, 1e-9), ("f32", 1e-4, 1e-3)])
@pytest.mark.parametrize("iterations", [1, 3])
def test_etrs_steps_match_oracle(prec, tol_psi, tol_f, iterations):
    import torch
    from oracle import Model, dynamics
    from paper_0812_2801_amd import binding as B
    note(f"etrs {prec} iterations={iterations}")
    inp = W.make_inputs(CFG)
    p, keep = B.params_from_config(CFG, inp["pos"], precision=prec, etrs_iterations=iterations)
    s = B.System(p, keep)
    s.set_state(torch.from_numpy(inp["psi"].reshape(CFG.n_orb, -1)))
    m = Model.from_config(CFG)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    ae = st
    for n in range(3):
        eps = 0.01 * (n + 1)
        rep = s.step(ctrl=eps, report=True)
        st = dynamics.etrs_step(m, st, eps, iterations=iterations)
        ae = dynamics.aetrs_step(m, ae, eps)
        psi = to_np(s.get_state()).reshape(st.psi.shape)
        dpsi = np.abs(psi - st.psi).max()
        df = np.abs(s.forces() - st.force).max()
        e = dynamics.total_energy(m, st)
        note(f"  step {n}: max|dpsi| {dpsi:.2e} max|dF| {df:.2e} dE {abs(rep['e_total'] - e['total']):.2e}; "
             f"ETRS-AETRS {np.abs(st.psi - ae.psi).max():.2e}")
        assert dpsi < tol_psi
        assert df < tol_f
        if prec == "f64":
            assert abs(rep["e_total"] - e["total"]) < 1e-9 * max(1.0, abs(e["total"]))
    s.close()


def test_etrs_refused_where_unsupported():
    from paper_0812_2801_amd import binding as B
    inp = W.make_inputs(W.C1)
    p, keep = B.params_from_config(W.C1, inp["pos"], etrs_iterations=1, enable_adjoint=True)
    with pytest.raises(B.ModehrError):
        B.System(p, keep)
    p, keep = B.params_from_config(W.C1, inp["pos"], etrs_iterations=9)
    with pytest.raises(B.ModehrError):
        B.System(p, keep)
