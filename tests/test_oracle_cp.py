"""Pins of the oracle's Car-Parrinello step (eq. L_CP, eq. EoM_CP; electrons
by RATTLE / velocity Verlet): closed-form stationary eigenstates, the two
constraints, second-order energy conservation and time reversibility."""
import numpy as np

import workloads as W
from oracle import Model, cp


def _plane_waves(m, ks):
    """Normalised plane waves exp(i 2 pi k.r / L) on the (z, y, x) grid."""
    x, y, z = m.grid.coords()
    out = []
    for kx, ky, kz in ks:
        ph = 2.0 * np.pi / m.grid.L * (kx * x + ky * y + kz * z)
        out.append(np.exp(1j * ph) / np.sqrt(m.grid.L ** 3))
    return np.array(out)


def test_plane_wave_eigenstates_are_stationary():
    # no ions: rho of plane waves is uniform, so v_Hxc is constant and plane
    # waves are exact eigenvectors of the finite-difference H; with zero
    # orbital velocity the constraint force cancels H psi exactly
    m = Model(n=10, h=0.4, zval=np.zeros(0), mass=np.zeros(0))
    psi0 = _plane_waves(m, [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 2, 1)])
    assert np.abs(m.overlaps(psi0) - np.eye(4)).max() < 1e-13
    st = cp.init_state(m, psi0, np.zeros((0, 3)))
    for _ in range(5):
        st = cp.cp_step(m, st, mu_cp=50.0, dt=0.3)
    assert np.abs(st.psi - psi0).max() < 1e-12
    assert np.abs(st.psidot).max() < 1e-11


def _c1_state(mu_cp=50.0, seed=7):
    c = W.C1.replace(seed=seed)
    inp = W.make_inputs(c)
    m = Model.from_config(c)
    return m, cp.init_state(m, inp["psi"], inp["pos"])


def test_constraints_hold_after_each_step():
    m, st = _c1_state()
    for _ in range(4):
        st = cp.cp_step(m, st, mu_cp=50.0, dt=0.25)
        s = m.overlaps(st.psi)
        assert np.abs(s - np.eye(len(s))).max() < 1e-12
        q = cp._gram(m, st.psi, st.psidot)
        assert np.abs(q + q.conj().T).max() < 1e-12
        assert np.abs(st.psidot).max() > 1e-3         # the orbitals do move


def _drift(dt, t_end=1.2, mu_cp=50.0):
    m, st = _c1_state(mu_cp)
    e0 = cp.energy(m, st, mu_cp)["total"]
    worst = 0.0
    for _ in range(int(round(t_end / dt))):
        st = cp.cp_step(m, st, mu_cp, dt)
        worst = max(worst, abs(cp.energy(m, st, mu_cp)["total"] - e0))
    return worst, st


def test_energy_conservation_is_second_order():
    d1, st1 = _drift(0.2)
    d2, st2 = _drift(0.1)
    ratio = d1 / d2
    assert 2.5 < ratio < 6.0, ratio
    assert d2 < 1e-3
    # the ions moved and the orbitals carry fictitious kinetic energy
    m, _ = _c1_state()
    assert np.abs(st2.pos - W.make_inputs(W.C1.replace(seed=7))["pos"]).max() > 1e-6
    assert cp.energy(m, st2, 50.0)["fictitious"] > 1e-6


def test_velocity_verlet_with_rattle_is_time_reversible():
    m, st0 = _c1_state()
    st = st0
    for _ in range(5):
        st = cp.cp_step(m, st, mu_cp=50.0, dt=0.25)
    st.psidot = -st.psidot
    st.vel = -st.vel
    for _ in range(5):
        st = cp.cp_step(m, st, mu_cp=50.0, dt=0.25)
    assert np.abs(st.psi - st0.psi).max() < 1e-10
    assert np.abs(st.pos - st0.pos).max() < 1e-10
    assert np.abs(st.psidot + st0.psidot).max() < 1e-9


def test_constraint_solver_reaches_tolerance_on_a_perturbed_rotation():
    rng = np.random.default_rng(5)
    n = 6
    g = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = np.eye(n) + 0.02 * g                         # <Psi|Psi~>
    a = b.conj().T @ b + 0.01 * np.eye(n)            # a Hermitian <Psi~|Psi~>
    x, it, res = cp.solve_position_constraint(a, b, tol=1e-14)
    assert res < 1e-14 and it < 100
    assert np.abs(x - x.conj().T).max() < 1e-15
