"""The finite box on the GPU (finite_radius > 0: the union of atom-centred
spheres with a zero boundary condition, free-space Hartree by doubled-grid
FFTs, isolated ions) against the oracle's plain sums: trajectories of the
small box in FP64 and FP32; at the 72^3 ring box, v_Hxc at sampled points,
V_loc and the forces everywhere, and the invariants of a 20-step FP32 run."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu


def _pair(cfg, prec, oracle_state=True):
    import torch
    from oracle import dynamics, finite
    from paper_0812_2801_amd import binding as B
    inp = W.make_inputs(cfg)
    p, keep = B.params_from_config(cfg, inp["pos"], precision=prec)
    s = B.System(p, keep)
    s.set_state(torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1)))
    m = finite.FiniteModel.from_config(cfg, pos0=inp["pos"], radius=cfg.finite_radius)
    st = dynamics.init_state(m, inp["psi"], inp["pos"]) if oracle_state else None
    return s, m, st, inp


@pytest.mark.parametrize("prec,tol_psi,tol_f", [("f64", 1e-10, 1e-9), ("f32", 1e-4, 1e-3)])
def test_small_box_trajectory(prec, tol_psi, tol_f):
    from oracle import dynamics
    note(f"finite box {W.F0.name} {prec}")
    s, m, st, inp = _pair(W.F0, prec)
    out = ~m.mask.astype(bool)
    for n in range(3):
        rep = s.step(report=True)
        st = dynamics.aetrs_step(m, st)
        psi = to_np(s.get_state()).reshape(st.psi.shape)
        dpsi = np.abs(psi - st.psi).max()
        df = np.abs(s.forces() - st.force).max()
        e = dynamics.total_energy(m, st)
        note(f"  step {n}: max|dpsi| {dpsi:.2e} max|dF| {df:.2e} dE {abs(rep['e_total'] - e['total']):.2e}")
        assert dpsi < tol_psi and df < tol_f
        assert np.abs(psi[:, out]).max() == 0.0
        if prec == "f64":
            assert abs(rep["e_total"] - e["total"]) < 1e-9 * max(1.0, abs(e["total"]))
    s.close()


def test_ring_box_fields_forces_and_invariants():
    from oracle import finite
    from paper_0812_2801_amd import binding as B
    cfg = W.F3
    note(f"finite box {cfg.name}: {cfg.n}^3, {cfg.n_orb} orbitals, {cfg.n_ions} ions")
    s, m, _, inp = _pair(cfg, "f32", oracle_state=False)
    # the oracle's v_H everywhere would be a 10^10-term sum: density, V_loc
    # and forces in full, v_Hxc at sampled points
    rho = m.density(inp["psi"])
    force = m.forces(inp["pos"], inp["psi"], rho)["total"]
    rng = np.random.default_rng(7)
    inside = np.nonzero(m.mask.ravel())[0]
    pts = np.concatenate([rng.choice(inside, 48, replace=False), rng.choice(m.grid.N, 16, replace=False)])
    vhxc = to_np(s.potential(1)).ravel()
    from oracle import potentials
    want = finite.hartree_free(m.grid, rho, points=pts) + potentials.slater_potential(rho.ravel()[pts])
    dv = np.abs(vhxc[pts] - want).max() / np.abs(want).max()
    note(f"  v_Hxc at 64 sampled points: rel err {dv:.2e}")
    assert dv < 1e-5
    vloc = to_np(s.potential(0)).reshape(m.grid.shape)
    assert np.abs(vloc - m.vloc(inp["pos"])).max() < 1e-11 * np.abs(vloc).max()
    df = np.abs(s.forces() - force).max()
    note(f"  forces: max|dF| {df:.2e} (max|F| {np.abs(force).max():.2e})")
    assert df < 1e-3 * max(1.0, np.abs(force).max())
    e0 = s.report()["e_total"]
    out = ~m.mask.astype(bool).ravel()
    for n in range(20):
        rep = s.step(report=(n == 19))
    psi = to_np(s.get_state())
    norms = cfg.h ** 3 * (np.abs(psi) ** 2).sum(axis=1)
    note(f"  20 steps: dE {rep['e_total'] - e0:.2e} (E {e0:.5f}), max|norm-1| {np.abs(norms - 1).max():.2e}")
    assert np.abs(psi[:, out]).max() == 0.0
    assert np.abs(norms - 1.0).max() < 1e-4
    assert abs(rep["e_total"] - e0) < 1e-3 * abs(e0)
    with pytest.raises(B.ModehrError):
        s.step(ctrl=0.01)
    s.close()
    p, keep = B.params_from_config(cfg, inp["pos"], finite_radius=10.0)
    with pytest.raises(B.ModehrError):
        B.System(p, keep)


def test_small_box_etrs():
    # the finite box with the ETRS propagator (v_Hxc of the predicted density
    # from the free-space Poisson solve) against the oracle
    import torch
    from oracle import dynamics, finite
    from paper_0812_2801_amd import binding as B
    cfg = W.F0
    note(f"finite box {cfg.name} ETRS")
    inp = W.make_inputs(cfg)
    p, keep = B.params_from_config(cfg, inp["pos"], precision="f64", etrs_iterations=1)
    s = B.System(p, keep)
    s.set_state(torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1)))
    m = finite.FiniteModel.from_config(cfg, pos0=inp["pos"], radius=cfg.finite_radius)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    for n in range(2):
        s.step()
        st = dynamics.etrs_step(m, st, 0.0, iterations=1)
        dpsi = np.abs(to_np(s.get_state()).reshape(st.psi.shape) - st.psi).max()
        note(f"  step {n}: max|dpsi| {dpsi:.2e}")
        assert dpsi < 1e-10
    s.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_box_with_many_ions_forces(prec, tol):
    # 20 ions on a ring: the local-force kernel takes the ions in groups of 8
    cfg = W.F3.replace(name="ring20", n=56, h=0.4, n_ions=20, n_orb=8, ring_radius=4.0, finite_radius=4.5,
                       seed=2020)
    note(f"finite box {cfg.name}: {cfg.n_ions} ions {prec}")
    s, m, _, inp = _pair(cfg, prec, oracle_state=False)
    want = m.forces(inp["pos"], inp["psi"], m.density(inp["psi"]))["total"]
    df = np.abs(s.forces() - want).max()
    note(f"  forces max|dF| {df:.2e} (max|F| {np.abs(want).max():.2e})")
    assert df < tol * max(1.0, np.abs(want).max())
    s.close()
