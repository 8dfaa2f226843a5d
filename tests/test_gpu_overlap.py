"""The MD step on two streams (the ion-side work of a step and the nonlocal
forces on a second stream, ordered by events) against the same step on the
caller's stream alone (MODEHR_OVERLAP=0): the kernels and their inputs are
the same, so orbitals, forces, positions and the energy report must agree
bit for bit after several steps with moving ions, and both against the FP64
oracle within the usual gates.  ETRS (the second exponential redone) takes
the same fork and join."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu

CFG = W.C1.replace(n=24, h=0.3, n_orb=5, n_ions=5, placement="lattice", jitter=0.2, seed=2411)


def _run(prec, overlap, steps, **over):
    import torch
    from paper_0812_2801_amd import binding as B
    old = os.environ.get("MODEHR_OVERLAP")
    os.environ["MODEHR_OVERLAP"] = "1" if overlap else "0"
    try:
        inp = W.make_inputs(CFG)
        p, keep = B.params_from_config(CFG, inp["pos"], precision=prec, **over)
        s = B.System(p, keep)
    finally:
        if old is None:
            os.environ.pop("MODEHR_OVERLAP", None)
        else:
            os.environ["MODEHR_OVERLAP"] = old
    s.set_state(torch.from_numpy(inp["psi"].reshape(CFG.n_orb, -1)))
    reps = [s.step(report=True) for _ in range(steps)]
    pos, vel = s.ions()
    out = (to_np(s.get_state()), s.forces().copy(), np.concatenate([pos, vel]), [r["e_total"] for r in reps])
    s.close()
    return out, inp


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_bf16x3"])
def test_two_stream_step_is_bit_identical(prec):
    from oracle import Model, dynamics
    (psi_a, f_a, pos_a, e_a), inp = _run(prec, True, 4)
    (psi_b, f_b, pos_b, e_b), _ = _run(prec, False, 4)
    note(f"{prec}: two streams vs one: max|dpsi| {np.abs(psi_a - psi_b).max():.1e}, "
         f"max|dF| {np.abs(f_a - f_b).max():.1e}, dE {max(abs(x - y) for x, y in zip(e_a, e_b)):.1e}")
    assert np.array_equal(psi_a, psi_b)
    assert np.array_equal(f_a, f_b)
    assert e_a == e_b
    assert np.array_equal(pos_a, pos_b)
    # and the step itself against the oracle
    m = Model.from_config(CFG)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    for _ in range(4):
        st = dynamics.aetrs_step(m, st)
    d = np.abs(psi_a - st.psi.reshape(CFG.n_orb, -1)).max()
    df = np.abs(f_a - st.force).max()
    note(f"  vs oracle after 4 steps: max|dpsi| {d:.1e}, max|dF| {df:.1e}")
    tol = {"f64": (1e-10, 1e-9), "f32": (1e-4, 1e-4), "f32_bf16x3": (1e-4, 1e-4)}[prec]
    assert d <= tol[0] and df <= tol[1]


def test_two_stream_etrs_is_bit_identical():
    (psi_a, f_a, _, e_a), _ = _run("f64", True, 3, etrs_iterations=1)
    (psi_b, f_b, _, e_b), _ = _run("f64", False, 3, etrs_iterations=1)
    note(f"ETRS: two streams vs one: max|dpsi| {np.abs(psi_a - psi_b).max():.1e}")
    assert np.array_equal(psi_a, psi_b)
    assert np.array_equal(f_a, f_b)
    assert e_a == e_b
