"""Pins of reading R3: the Hamiltonian of the second AETRS exponential,
H(t+dt), is built from previous steps (sec. 5.1, eq. aetrs).  The ionic part
is exact at R(t+dt); the Hartree-exchange potential is extrapolated from the
last three stored levels by the quadratic through them, from two levels by
the line, from one by the constant.

The pins fix that reading without re-typing its coefficients: the
extrapolation must be exact for every polynomial history of the degree its
level count allows and must fail for the next degree; the adjoint's weights
must reproduce the same extrapolation; one AETRS step must propagate with
exactly that potential; and on a real trajectory the extrapolation error must
fall with the third power of the step."""
import numpy as np

import workloads as W
from oracle import Model, adjoint, dynamics


def _fields(seed, k, shape=(4, 5, 6)):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(shape) for _ in range(k)]


def _poly_history(coef, levels):
    """levels values q(0..levels-1) and the next one q(levels), with
    q(j) = sum_d coef[d] j^d evaluated directly."""
    def q(j):
        return sum(c * float(j) ** d for d, c in enumerate(coef))
    return [q(j) for j in range(levels)], q(levels)


def test_extrapolation_exact_for_quadratic_history():
    for seed in range(4):
        hist, want = _poly_history(_fields(seed, 3), 3)
        got = dynamics.extrapolate(hist)
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_extrapolation_not_exact_for_cubic_history():
    # a cubic term is the first one the three-level rule cannot follow:
    # j^3 at 0, 1, 2 extrapolates to 3*8 - 3*1 + 0 = 21 instead of 27
    a = _fields(9, 1)[0]
    hist, want = _poly_history([0 * a, 0 * a, 0 * a, a], 3)
    got = dynamics.extrapolate(hist)
    assert np.abs(got - want).max() > 5.9 * np.abs(a).max()
    assert np.abs((want - got) - 6.0 * a).max() < 1e-12 * np.abs(a).max()


def test_extrapolation_two_levels_linear_one_level_constant():
    for seed in range(3):
        hist, want = _poly_history(_fields(10 + seed, 2), 2)
        got = dynamics.extrapolate(hist)
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # the two-level rule is not exact for a quadratic
    hist, want = _poly_history(_fields(20, 3), 2)
    assert np.abs(dynamics.extrapolate(hist) - want).max() > 1e-3
    one = _fields(30, 1)
    got = dynamics.extrapolate(one)
    assert np.array_equal(got, one[0]) and got is not one[0]


def test_adjoint_weights_reproduce_the_forward_extrapolation():
    # vt = sum_j a_j v_{n-j} in the reverse sweep: the weights must extrapolate
    # the same polynomials exactly, newest level first
    for levels, deg in ((3, 2), (2, 1), (1, 0)):
        a = adjoint._extrap_coeffs(levels)
        assert len(a) == levels
        hist, want = _poly_history(_fields(40 + levels, deg + 1), levels)
        got = sum(a[j] * hist[levels - 1 - j] for j in range(levels))
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
        assert np.abs(got - dynamics.extrapolate(hist)).max() < 1e-12 * np.abs(want).max()


def _tiny_model():
    pos = np.array([[0.7, 1.1, 0.9], [2.0, 1.9, 2.3]])
    m = Model(n=8, h=0.35, zval=np.full(2, 4.0), mass=np.full(2, W.BE9_MASS),
              freeze_ions=True, dt=0.02, mu=1.0)
    return m, pos


def test_aetrs_step_propagates_with_the_extrapolated_potential():
    m, pos = _tiny_model()
    rng = np.random.default_rng(5)
    shape = (2,) + m.grid.shape
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    psi /= np.sqrt(m.grid.dv * np.sum(np.abs(psi) ** 2, axis=(1, 2, 3)))[:, None, None, None]
    st = dynamics.init_state(m, psi, pos)
    # a prescribed history: quadratic in the level index, small in size
    coef = [0.05 * f for f in _fields(6, 3, m.grid.shape)]
    hist, v_next = _poly_history(coef, 3)
    st = dynamics.State(psi=st.psi, pos=st.pos, vel=st.vel, force=st.force, rho=st.rho,
                        hist=list(hist))
    got = dynamics.aetrs_step(m, st).psi
    tau = m.dt / (2.0 * m.mu)
    vloc = m.vloc(pos)
    sph = m.spheres(pos)
    half = dynamics.taylor(m, tau, vloc + hist[-1], sph, psi)
    want = dynamics.taylor(m, tau, vloc + v_next, sph, half)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
    # the potential of the second exponential matters at this size: the
    # newest level alone (no extrapolation) gives a visibly different step
    other = dynamics.taylor(m, tau, vloc + hist[-1], sph, half)
    assert np.abs(other - want).max() > 1e3 * np.abs(got - want).max()


def test_extrapolation_error_is_third_order_on_a_trajectory():
    # along the oracle's own c1 dynamics v_Hxc(t) is smooth, so the quadratic
    # through three levels misses v_Hxc(t + dt) by O(dt^3): halving dt cuts
    # the miss by about 8 (7.4 here; the linear rule gives 3.9)
    miss = []
    for dt in (0.02, 0.01):
        m = Model.from_config(W.C1, dt=dt)
        inp = W.make_inputs(W.C1)
        s = dynamics.init_state(m, inp["psi"], inp["pos"])
        steps = int(round(0.12 / dt))
        for _ in range(steps):
            s = dynamics.aetrs_step(m, s)
        pred = dynamics.extrapolate(s.hist)
        s = dynamics.aetrs_step(m, s)
        miss.append(float(np.abs(pred - s.hist[-1]).max()))
    ratio = miss[0] / miss[1]
    assert 6.0 < ratio < 10.0, (miss, ratio)
