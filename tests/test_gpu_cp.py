"""GPU Car-Parrinello comparison step (eq. EoM_CP, RATTLE / velocity Verlet)
through the C ABI against the FP64 oracle, and its invariants at a larger
size: orthonormality held by the constraint, the conserved energy."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu


def _system(cfg, prec):
    import torch
    from paper_0812_2801_amd import binding as B
    inp = W.make_inputs(cfg)
    p, keep = B.params_from_config(cfg, inp["pos"], precision=prec)
    s = B.System(p, keep)
    s.set_state(torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1)))
    return s, inp


@pytest.mark.parametrize("prec,tol", [("f64", 1e-11), ("f32", 2e-6)])
def test_cp_steps_follow_the_oracle(prec, tol):
    from oracle import Model, cp
    for cfg in (W.C1, W.C1.replace(name="odd", n=20, n_orb=5, n_ions=5, placement="lattice", jitter=0.2, seed=77)):
        note(f"cp vs oracle {prec} {cfg.name}")
        mu_cp, dt = 50.0, 0.25
        s, inp = _system(cfg, prec)
        s.cp_begin(mu_cp, dt)
        m = Model.from_config(cfg)
        st = cp.init_state(m, inp["psi"], inp["pos"])
        for _ in range(4):
            rep = s.cp_step(report=True)
            st = cp.cp_step(m, st, mu_cp, dt)
        psi = to_np(s.get_state()).reshape(st.psi.shape)
        e = cp.energy(m, st, mu_cp)
        d = np.abs(psi - st.psi).max()
        df = np.abs(s.forces().reshape(st.force.shape) - st.force).max()
        note(f"  max|dpsi| {d:.2e} max|dF| {df:.2e} dE {abs(rep['e_total'] - e['total']):.2e} "
             f"residual {rep['cp_constraint_residual']:.1e}")
        assert d < tol
        assert df < (1e-9 if prec == "f64" else 1e-4)
        assert abs(rep["e_total"] - e["total"]) < (1e-9 if prec == "f64" else 1e-3) * abs(e["total"])
        assert abs(rep["e_fictitious"] - e["fictitious"]) < (1e-9 if prec == "f64" else 1e-3) * e["fictitious"]
        assert 0.0 <= rep["cp_constraint_residual"] < 1e-11
        s.close()


def test_cp_invariants_at_64_cubed():
    """64^3, 32 moving ions, 48 FP32 orbitals: the constraint keeps the
    orbitals orthonormal to the accuracy of the FP32 overlaps (sums over
    262144 points, partial sums added in FP64: measured 1.3e-7 after 21
    steps) and E_CP stays put (the FP32 Ehrenfest step drifts by about 1e-4
    of E as well)."""
    import torch
    from oracle import Model
    cfg = W.C5.replace(name="cp64", n_orb=48, freeze_ions=False, seed=515)
    note("cp invariants 64^3 f32")
    s, inp = _system(cfg, "f32")
    s.cp_begin(200.0, 0.184)
    e0 = s.cp_step(report=True)["e_total"]
    worst = 0.0
    for _ in range(20):
        worst = max(worst, abs(s.cp_step(report=True)["e_total"] - e0))
    psi = to_np(s.get_state()).astype(np.complex128)
    m = Model.from_config(cfg)
    ov = m.overlaps(psi.reshape((cfg.n_orb,) + m.grid.shape))
    dev = np.abs(ov - np.eye(cfg.n_orb)).max()
    note(f"  max|S - I| {dev:.2e}  max|E - E0| {worst:.2e} of {abs(e0):.3e}")
    assert dev < 1e-3
    assert worst < 5e-4 * abs(e0)
    s.close()


def test_cp_invariants_at_the_benchmark_shape():
    """96^3, 64 moving ions, 128 FP32 orbitals, mu_CP = 200, dt = 0.1844 (the
    benchmark's CP leg): after 10 steps the orbitals are orthonormal to the
    accuracy of the FP32 overlaps and E_CP has not moved beyond the FP32
    step's own drift."""
    import torch
    cfg = W.C2
    note("cp invariants 96^3 x 128 f32")
    from paper_0812_2801_amd import binding as B
    p, keep = B.params_from_config(cfg, W.ion_positions(cfg), precision="f32")
    s = B.System(p, keep)
    s.set_state(W.initial_orbitals_device(cfg, "cuda:0"))
    s.cp_begin(200.0, 0.08 * 7.26 / 3.15)
    e0 = s.cp_step(report=True)["e_total"]
    worst, res = 0.0, 0.0
    for _ in range(9):
        rep = s.cp_step(report=True)
        worst = max(worst, abs(rep["e_total"] - e0))
        res = max(res, rep["cp_constraint_residual"])
    psi = s.get_state().to(torch.complex128)
    ov = cfg.h ** 3 * (psi.conj() @ psi.T)
    dev = (ov - torch.eye(cfg.n_orb, dtype=torch.complex128, device=ov.device)).abs().max().item()
    note(f"  max|S - I| {dev:.2e}  max|E - E0| {worst:.2e} of {abs(e0):.3e}  constraint residual {res:.1e}")
    assert dev < 1e-3
    assert worst < 5e-4 * abs(e0)
    assert res < 1e-8
    s.close()


def test_cp_needs_begin_after_a_state_change():
    from paper_0812_2801_amd import binding as B
    s, _ = _system(W.C1, "f64")
    with pytest.raises(B.ModehrError) as e:
        s.cp_step()
    assert e.value.status == B.ME_ESTATE
    s.cp_begin(50.0, 0.25)
    s.cp_step()
    s.step()                                  # an Ehrenfest step ends the CP run
    with pytest.raises(B.ModehrError) as e:
        s.cp_step()
    assert e.value.status == B.ME_ESTATE
    with pytest.raises(B.ModehrError) as e:
        s.cp_begin(-1.0, 0.25)
    assert e.value.status == B.ME_EINVAL
    s.close()
