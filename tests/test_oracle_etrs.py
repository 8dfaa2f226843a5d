"""Pins of the oracle's ETRS step (the propagator AETRS approximates, sec.
5.1): zero corrections is AETRS, a density-independent H makes the two equal,
the corrections converge to the self-consistent second exponential, and
ETRS run forward then backward returns much closer to the start than AETRS."""
import copy

import numpy as np

import workloads as W
from oracle import Model, dynamics


def _c1(**over):
    c = W.C1.replace(freeze_ions=True, **over)
    inp = W.make_inputs(c)
    m = Model.from_config(c)
    return m, dynamics.init_state(m, inp["psi"], inp["pos"])


def test_zero_corrections_is_aetrs():
    m, st = _c1()
    a = dynamics.aetrs_step(m, st)
    e = dynamics.etrs_step(m, st, iterations=0)
    assert np.array_equal(a.psi, e.psi)


def test_density_independent_hamiltonian_gives_aetrs():
    # occupation 0: rho = 0, v_Hxc = 0 at every step, so the extrapolated and
    # the self-consistent potentials coincide; with moving ions and a field,
    # the corrected exponential must still use V_loc(R(t+dt)) and the field
    c = W.C1.replace(freeze_ions=False)
    inp = W.make_inputs(c)
    m = Model.from_config(c)
    m.occ = 0.0
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    a = dynamics.aetrs_step(m, st, 0.05)
    e = dynamics.etrs_step(m, st, 0.05, iterations=3)
    assert np.abs(a.pos - st.pos).max() > 1e-9          # the ions do move (heavy ions, short step)
    assert np.abs(a.psi - e.psi).max() < 1e-14


def test_corrections_converge_to_the_self_consistent_step():
    m, st = _c1()
    tau = m.dt / (2.0 * m.mu)
    pos1, h0, h1 = dynamics.step_hamiltonians(m, st)
    half = dynamics.taylor(m, tau, h0[0], h0[1], st.psi)
    prev = None
    for k in (1, 2, 3, 4):
        psi1 = dynamics.etrs_step(m, st, iterations=k).psi
        resid = np.abs(psi1 - dynamics.taylor(m, tau, m.vloc(pos1) + m.v_hxc(m.density(psi1)), h1[1], half)).max()
        if prev is not None:
            assert resid < 0.2 * prev or resid < 1e-14
        prev = resid
    assert prev < 1e-12


def test_etrs_is_far_more_time_reversible_than_aetrs():
    def round_trip(step, n=4):
        m, st0 = _c1(dt=0.02, mu=1.0)       # tau E_max = 1.1, well inside the Taylor-4 limit
        st = st0
        for _ in range(n):
            st = step(m, st)
        mb = copy.copy(m)
        mb.dt = -m.dt
        for _ in range(n):
            st = step(mb, st)
        return np.abs(st.psi - st0.psi).max()

    e_aetrs = round_trip(lambda m, s: dynamics.aetrs_step(m, s))
    e_etrs = round_trip(lambda m, s: dynamics.etrs_step(m, s, iterations=6))
    assert e_etrs < 0.1 * e_aetrs, (e_etrs, e_aetrs)
