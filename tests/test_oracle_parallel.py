"""The orbital-parallel driver of the oracle (used for the full-size FP64
reference trajectories and the CPU baseline) reproduces the serial oracle:
the same steps, forces and energies up to the order of the sums over
orbitals."""
import numpy as np

import workloads as W
from oracle import Model, dynamics
from oracle.parallel import Driver


def _close(a, b, rel=1e-13):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max()) <= rel * max(1e-300, float(np.abs(b).max()))


def test_parallel_steps_equal_serial_steps():
    cfg = W.C1.replace(n_orb=5, n_ions=3, placement="uniform", min_sep=1.5, seed=4711)
    inp = W.make_inputs(cfg)
    m = Model.from_config(cfg)
    ser = dynamics.init_state(m, inp["psi"], inp["pos"])
    with Driver(m, cfg.n_orb, workers=2, orbitals_per_task=2) as d:
        par = d.init_state(inp["psi"], inp["pos"])
        assert _close(par.force, ser.force) and _close(par.rho, ser.rho)
        for n in range(3):
            eps = 0.01 * (n - 1)
            ser = dynamics.aetrs_step(m, ser, eps)
            par = d.aetrs_step(par, eps)
            assert _close(d.psi, ser.psi), n
            assert _close(par.pos, ser.pos) and _close(par.vel, ser.vel), n
            assert _close(par.force, ser.force, 1e-11), n
            assert _close(par.rho, ser.rho), n
            assert all(_close(a, b) for a, b in zip(par.hist, ser.hist)), n
        e_ser = dynamics.total_energy(m, ser)
        e_par = d.total_energy(par)
        for k, v in e_ser.items():
            assert abs(e_par[k] - v) <= 1e-12 * max(1.0, abs(v)), k


def test_streamed_orbitals_are_orthonormal_and_reproducible():
    cfg = W.C1.replace(n_orb=7, seed=99)
    a = W.initial_orbitals_streamed(cfg)
    b = W.initial_orbitals_streamed(cfg, chunk=3)
    assert np.array_equal(a, b)
    flat = a.reshape(cfg.n_orb, -1)
    s = cfg.h ** 3 * (flat.conj() @ flat.T)
    assert np.abs(s - np.eye(cfg.n_orb)).max() < 1e-13
    # each orbital's fields come from its own stream
    f_all = W.orbital_fields(cfg, 0, 7)
    f_mid = W.orbital_fields(cfg, 3, 5)
    assert np.array_equal(f_all[3:5], f_mid)
