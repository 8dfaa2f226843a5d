"""GPU parity: the HIP library through its C ABI against the FP64 CPU oracle
on the same seeded inputs.  Tolerances: FP64 max|dpsi| <= 1e-10 per step
(absolute, orbitals normalised to h^3 sum |psi|^2 = 1); FP32 <= 1e-4."""
import numpy as np
import pytest

import workloads as W
from gpu_common import make_pair, note, to_np

pytestmark = pytest.mark.gpu

SMALL = [
    ("c1", W.C1),
    # ragged: n = 18 leaves x runs of 1 point (FP32) and 2-row y tiles
    ("n18", W.C1.replace(n=18, h=0.3, n_orb=3, seed=1801)),
    # several stencil tiles and z chunks, 6 ions on a lattice
    ("n32", W.C1.replace(n=32, h=0.25, n_ions=6, n_orb=5, placement="lattice",
                         jitter=0.3, seed=3201)),
]


def _veff(m, st):
    return m.vloc(st.pos) + st.hist[-1]


@pytest.mark.parametrize("name,cfg", SMALL)
@pytest.mark.parametrize("prec", ["f64", "f32", "f32_bf16x3"])
def test_apply_H_matches_oracle(name, cfg, prec):
    note(f"apply_H {name} {prec}")
    sysm, m, st, inp, cfg = make_pair(cfg, precision=prec)
    rng = np.random.default_rng(5)
    shape = (3,) + m.grid.shape
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * 0.05
    got = to_np(sysm.apply_H(x.reshape(3, -1))).reshape(shape)
    want = m.apply_H(x, _veff(m, st), m.spheres(st.pos))
    # FP32 rounding ~6e-8 per operation; split-bf16 products keep ~16 mantissa bits
    tol = {"f64": 1e-11, "f32": 3e-6, "f32_bf16x3": 2e-5}[prec]
    err = np.abs(got - want).max() / np.abs(want).max()
    note(f"  rel err {err:.3e}")
    assert err < tol
    sysm.close()


@pytest.mark.parametrize("name,cfg", SMALL)
def test_initial_potentials_and_forces(name, cfg):
    note(f"potentials/forces {name}")
    sysm, m, st, inp, cfg = make_pair(cfg)
    vloc = to_np(sysm.potential(0)).reshape(m.grid.shape)
    vhxc = to_np(sysm.potential(1)).reshape(m.grid.shape)
    assert np.abs(vloc - m.vloc(st.pos)).max() < 1e-11 * max(1, np.abs(vloc).max())
    assert np.abs(vhxc - st.hist[-1]).max() < 1e-11 * max(1, np.abs(vhxc).max())
    rho = to_np(sysm.density()).reshape(m.grid.shape)
    assert np.abs(rho - st.rho).max() < 1e-13 * st.rho.max()
    f = sysm.forces()
    note(f"  force err {np.abs(f - st.force).max():.3e}")
    assert np.abs(f - st.force).max() < 1e-9 * max(1, np.abs(st.force).max())
    sysm.close()


@pytest.mark.parametrize("name,cfg", SMALL)
def test_energy_report_matches_oracle(name, cfg):
    from oracle import dynamics
    note(f"energy {name}")
    sysm, m, st, inp, cfg = make_pair(cfg)
    rep = sysm.report()
    e = dynamics.total_energy(m, st)
    for k, kk in (("e_kinetic", "kinetic"), ("e_local", "local"), ("e_hartree", "hartree"),
                  ("e_xc", "xc"), ("e_nonlocal", "nonlocal"), ("e_ion", "ion"),
                  ("e_total", "total")):
        assert abs(rep[k] - e[kk]) < 1e-10 * max(1.0, abs(e[kk])), (k, rep[k], e[kk])
    assert abs(rep["charge"] - cfg.occ * cfg.n_orb) < 1e-9
    sysm.close()


@pytest.mark.parametrize("name,cfg", SMALL)
def test_trajectory_f64(name, cfg):
    from oracle import dynamics
    steps = 10 if name == "c1" else 3
    note(f"trajectory f64 {name} steps={steps}")
    sysm, m, st, inp, cfg = make_pair(cfg)
    for n in range(steps):
        rep = sysm.step(report=True)
        st = dynamics.aetrs_step(m, st)
        psi = to_np(sysm.get_state()).reshape(st.psi.shape)
        pos, vel = sysm.ions()
        dpsi = np.abs(psi - st.psi).max()
        e = dynamics.total_energy(m, st)
        note(f"  step {n}: max|dpsi| {dpsi:.2e} dpos {np.abs(pos - st.pos).max():.2e} "
             f"dE {abs(rep['e_total'] - e['total']):.2e}")
        assert dpsi < 1e-10
        assert np.abs(pos - st.pos).max() < 1e-12
        assert np.abs(vel - st.vel).max() < 1e-12
        assert np.abs(sysm.forces() - st.force).max() < 1e-9
        assert abs(rep["e_total"] - e["total"]) < 1e-9 * max(1, abs(e["total"]))
    sysm.close()


@pytest.mark.parametrize("name,cfg", SMALL)
@pytest.mark.parametrize("prec", ["f32", "f32_bf16x3"])
def test_step_f32_within_gate(name, cfg, prec):
    from oracle import dynamics
    note(f"step {prec} {name}")
    sysm, m, st, inp, cfg = make_pair(cfg, precision=prec)
    for n in range(3):
        sysm.step()
        st = dynamics.aetrs_step(m, st)
        psi = to_np(sysm.get_state()).reshape(st.psi.shape)
        dpsi = np.abs(psi - st.psi).max()
        note(f"  step {n}: max|dpsi| {dpsi:.2e} (max|psi| {np.abs(st.psi).max():.2e})")
        assert dpsi < 1e-4
    sysm.close()


@pytest.mark.parametrize("order", [1, 2, 6])
def test_other_taylor_orders(order):
    from oracle import dynamics
    note(f"taylor order {order}")
    sysm, m, st, inp, cfg = make_pair(W.C1, taylor_order=order)
    sysm.step()
    st = dynamics.aetrs_step(m, st)
    psi = to_np(sysm.get_state()).reshape(st.psi.shape)
    assert np.abs(psi - st.psi).max() < 1e-10
    sysm.close()


def test_no_ions_and_frozen_field_step():
    from oracle import dynamics
    note("no ions, field")
    cfg = W.C1.replace(n_ions=0, placement="lattice", n_orb=2, seed=77)
    sysm, m, st, inp, cfg = make_pair(cfg)
    for eps in (0.01, -0.02):
        rep = sysm.step(ctrl=eps, report=True)
        st = dynamics.aetrs_step(m, st, eps)
    psi = to_np(sysm.get_state()).reshape(st.psi.shape)
    assert np.abs(psi - st.psi).max() < 1e-10
    e = dynamics.total_energy(m, st)
    note(f"  E {rep['e_total']:.12f} oracle {e['total']:.12f}, E_ion {rep['e_ion']}")
    assert rep["e_ion"] == 0.0
    assert abs(rep["e_total"] - e["total"]) < 1e-9 * max(1.0, abs(e["total"]))
    sysm.close()


def test_frozen_ions_with_field_and_static_potential():
    import torch
    from oracle import Model, dynamics, adjoint
    from paper_0812_2801_amd import binding as B
    note("frozen, field, static potential")
    cfg = W.C1.replace(freeze_ions=True, coarse_n=4, seed=4401)
    inp = W.make_inputs(cfg)
    dv = 0.05 * np.random.default_rng(2).standard_normal((4, 4, 4))
    fine = adjoint.coarse_to_fine(dv, cfg.n)
    p, keep = B.params_from_config(cfg, inp["pos"])
    sysm = B.System(p, keep)
    sysm.set_static_potential(torch.from_numpy(fine.reshape(-1)))
    sysm.set_state(torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1)))
    m = Model.from_config(cfg, vstatic=fine)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    for eps in (0.01, 0.03, -0.01):
        sysm.step(ctrl=eps)
        st = dynamics.aetrs_step(m, st, eps)
    psi = to_np(sysm.get_state()).reshape(st.psi.shape)
    assert np.abs(psi - st.psi).max() < 1e-10
    pos, _ = sysm.ions()
    assert np.abs(pos - inp["pos"]).max() == 0.0
    sysm.close()


def test_invalid_arguments_return_codes():
    import torch
    from paper_0812_2801_amd import binding as B
    note("invalid args")
    cfg = W.C1
    inp = W.make_inputs(cfg)
    p, keep = B.params_from_config(cfg, inp["pos"])
    sysm = B.System(p, keep)
    with pytest.raises(B.ModehrError) as e:
        sysm.step()
    assert e.value.status == B.ME_ESTATE
    x = torch.zeros((cfg.n_orb, cfg.n ** 3), dtype=torch.complex128, device="cuda")
    st = sysm.lib.me_apply_H(sysm.h, None, None, 1, cfg.n ** 3)
    assert st in (B.ME_EINVAL, B.ME_ESTATE)
    sysm.set_state(x + 1e-3)
    st = sysm.lib.me_apply_H(sysm.h, x.data_ptr(), x.data_ptr(), cfg.n_orb, cfg.n ** 3)
    assert st == B.ME_EINVAL
    sysm.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_orbital_steps(prec):
    # one orbital: the 8-orbital contraction blocks, the norm partials and the
    # density reduce over a single member
    from oracle import dynamics
    note(f"single orbital {prec}")
    sysm, m, st, inp, cfg = make_pair(W.C1.replace(n_orb=1, seed=1901), precision=prec)
    for _ in range(2):
        sysm.step()
        st = dynamics.aetrs_step(m, st)
    psi = to_np(sysm.get_state()).reshape(st.psi.shape)
    err = np.abs(psi - st.psi).max()
    note(f"  max|dpsi| {err:.2e}")
    assert err < (1e-10 if prec == "f64" else 1e-4)
    assert np.abs(sysm.forces() - st.force).max() < (1e-9 if prec == "f64" else 1e-3)
    sysm.close()
