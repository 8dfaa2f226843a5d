"""Pins of the two-band toy model (eq. L_toy): the equations of motion
against the Euler-Lagrange equations of the printed Lagrangian (by finite
differences of the Lagrangian itself), RK4 against its defining polynomial on
linear systems, the small electronic oscillation against its closed form,
energy conservation at fourth order, the gsBO closed form against direct
integration, and the mu -> 0 limit of d_R and d_F."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import toy

P = toy.ToyParams()


def test_n2_constants():
    # harmonic wavenumber of N2 back from K_R and M_R; R_0 = 1.0977 A
    assert abs(P.omega_R * 219474.6313632 - 2358.57) < 1e-6
    assert abs(P.R0 - 2.0743) < 1e-3
    assert abs(P.M_R / 1822.888486 - 7.0015) < 1e-3


def test_workload_constants_are_the_oracles():
    import workloads as W
    for k, v in W.TOY_N2.items():
        assert abs(getattr(P, k) - v) <= 1e-15 * abs(v), k


def test_rk4_is_the_fourth_order_polynomial_on_linear_systems():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 6))
    y = rng.standard_normal(6)
    h = 0.13
    got = toy.rk4_step(lambda v: A @ v, y, h)
    M = np.eye(6)
    term = np.eye(6)
    for k in range(1, 5):
        term = term @ (h * A) / k
        M = M + term
    assert np.abs(got - M @ y).max() < 1e-14 * np.abs(M @ y).max()


def _grad(fn, x, eps):
    g = np.zeros(len(x))
    for k in range(len(x)):
        e = np.zeros(len(x))
        e[k] = eps
        g[k] = (fn(x + e) - fn(x - e)) / (2 * eps)
    return g


@pytest.mark.parametrize("scheme,mu", [("ehrenfest", 0.7), ("cp", 40.0)])
def test_equations_of_motion_follow_the_lagrangian(scheme, mu):
    # Euler-Lagrange residual d/dt dL/dqdot - dL/dq at random states, with the
    # accelerations from rhs(); every derivative of L by central differences
    rng = np.random.default_rng(11)
    for _ in range(4):
        q = np.array([2.1, 2.4, 2.2, 0.35]) + 0.3 * rng.standard_normal(4)
        if scheme == "ehrenfest":
            Rd, Gd = 1e-3 * rng.standard_normal(2)
            y = np.array([q[0], q[1], q[2], Rd, q[3], Gd])
            d = toy.rhs(P, scheme, mu, y)
            qd = np.array([d[0], d[1], Rd, Gd])
            qdd = np.array([0.0, 0.0, d[3], d[5]])          # theta'' does not enter: L is linear in theta'
        else:
            vel = np.concatenate([0.05 * rng.standard_normal(2), 1e-3 * rng.standard_normal(2)])
            y = np.array([q[0], q[1], vel[0], vel[1], q[2], vel[2], q[3], vel[3]])
            d = toy.rhs(P, scheme, mu, y)
            qd = vel
            qdd = np.array([d[2], d[3], d[5], d[7]])
        L = lambda a, b: toy.lagrangian(P, scheme, mu, a, b)
        p_of = lambda a, b: _grad(lambda v: L(a, v), b, 1e-4)
        dLdq = _grad(lambda v: L(v, qd), q, 1e-5)
        eps = 1e-4
        dpdt = (p_of(q + eps * qd, qd + eps * qdd) - p_of(q - eps * qd, qd - eps * qdd)) / (2 * eps)
        res = dpdt - dLdq
        scale = np.abs(dLdq).max() + np.abs(dpdt).max()
        assert np.abs(res).max() < 1e-5 * scale, (scheme, res, scale)


@pytest.mark.parametrize("scheme,mu", [("ehrenfest", 0.5), ("cp", 30.0)])
def test_small_electronic_oscillation(scheme, mu):
    # ions frozen (infinite masses): theta_i - R oscillates at 2 pi / electronic_period
    p = toy.ToyParams(M_R=1e30, M_G=1e30)
    a = 1e-4
    y = toy.initial_state(p, scheme)
    y[0, 0] += a
    T = toy.electronic_period(p, scheme, mu)
    G = y[0, 4] if scheme == "ehrenfest" else y[0, 6]
    # the frequency is G / (2 mu) for the first-order angles, sqrt(G / (2 mu)) for CP
    w = 2 * math.pi / T * ((G / p.G0) if scheme == "ehrenfest" else math.sqrt(G / p.G0))
    dt = T / 2000
    f = lambda v: toy.rhs(p, scheme, mu, v)
    t = 0.0
    for _ in range(1300):
        y = toy.rk4_step(f, y, dt)
        t += dt
    c = toy.coords(scheme, y)[0]
    R = c[2]
    assert abs((c[0] - R) - a * math.cos(w * t)) < 1e-6 * a
    if scheme == "ehrenfest":
        assert abs((c[1] - R) + a * math.sin(w * t)) < 1e-6 * a
    else:
        assert abs(c[1] - R) < 1e-12


@pytest.mark.parametrize("scheme,mu", [("ehrenfest", 0.5), ("cp", 60.0)])
def test_energy_conserved_at_fourth_order(scheme, mu):
    # the energy of the Lagrangian is conserved by the exact flow; RK4 loses
    # it at a power of dt between 4 and 6 (dt^5 for a harmonic mode)
    T = 0.5 * P.period_R
    drift = []
    for n in (200, 400):
        y = toy.initial_state(P, scheme)
        e0 = toy.energy(P, scheme, mu, y)[0]
        f = lambda v: toy.rhs(P, scheme, mu, v)
        for _ in range(n):
            y = toy.rk4_step(f, y, T / n)
        drift.append(abs(toy.energy(P, scheme, mu, y)[0] - e0))
    ratio = drift[0] / drift[1]
    assert drift[0] < 1e-8 * abs(e0) and 16.0 < ratio < 64.0, (drift, ratio)


def test_gsbo_closed_form():
    # M_R R'' = -K_R (R - R_0) from 1.1 R_0 at rest, integrated by RK4
    dt = P.period_R / 4000
    y = np.array([1.1 * P.R0, 0.0])
    f = lambda v: np.array([v[1], -P.K_R * (v[0] - P.R0) / P.M_R])
    for _ in range(3000):
        y = toy.rk4_step(f, y, dt)
    assert abs(y[0] - toy.gsbo_R(P, 3000 * dt)) < 1e-10
    t0, t1 = 123.0, 171.5
    num = quad(lambda t: -P.K_R * (toy.gsbo_R(P, t) - P.R0), t0, t1)[0] / (t1 - t0)
    assert abs(toy.gsbo_force_mean(P, t0, t1) - num) < 1e-12


def test_trajectory_distance_of_an_offset():
    rng = np.random.default_rng(2)
    ref = rng.standard_normal((50, 4))
    span = ref.max(axis=0) - ref.min(axis=0)
    c = np.array([0.0, 0.0, 0.01, 0.0])
    got = toy.trajectory_distance(ref + c, ref)
    assert abs(got - 100 * 0.01 / span[2]) < 1e-12


def test_distances_vanish_as_mu_goes_to_zero():
    T = 2 * P.period_R
    out = {}
    for scheme, mus, sub in (("ehrenfest", [2.0, 0.5, 0.125], 4), ("cp", [400.0, 100.0, 25.0], 4)):
        r = toy.run(P, scheme, mus, sub, 400, T)
        out[scheme] = r
        d_R, d_F = r["d_R"], r["d_F"]
        assert d_R[0] > d_R[1] > d_R[2], (scheme, d_R)
        assert d_F[0] > d_F[1] > d_F[2], (scheme, d_F)
    # at the smallest mass the Ehrenfest R(t) follows the gsBO motion closely
    assert out["ehrenfest"]["d_R"][2] < 1.0
    assert out["cp"]["d_R"][2] < 1.0


def test_dt_max_is_the_threshold_of_the_ladder():
    # the selected step passes (with every smaller one) and the next coarser
    # step of the ladder fails the 0.1 distance criterion
    T = P.period_R
    ladder = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32]
    for scheme, mu in (("ehrenfest", 0.3), ("cp", 5.0)):
        best = toy.dt_max(P, scheme, mu, 60, T, ladder, 128)
        assert best is not None
        s_best = int(round(T / (60 * best)))
        ref = toy.run(P, scheme, [mu], 128, 60, T)["samples"][0]
        d = {s: toy.trajectory_distance(toy.run(P, scheme, [mu], s, 60, T)["samples"][0], ref) for s in ladder}
        assert all(d[s] < 0.1 for s in ladder if s >= s_best), (scheme, d)
        coarser = [s for s in ladder if s < s_best]
        assert coarser and d[max(coarser)] >= 0.1, (scheme, d)
