"""Pins of the oracle's propagator: fourth-order Taylor exponential and AETRS
(sec. 5.1, eq. aetrs), the mu time rescaling (eq. transf), the invariants of
sec. 4.2 (eq. E_new energy, eq. escpro overlaps, basis-rotation symmetry
eq. symmetry1) and velocity-Verlet time reversibility."""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import Model, dynamics


def tiny(n=8, h=0.35):
    pos = np.array([[0.7, 1.1, 0.9], [2.0, 1.9, 2.3]])
    m = Model(n=n, h=h, zval=np.full(2, 4.0), mass=np.full(2, W.BE9_MASS))
    return m, pos


def test_taylor_equals_dense_matrix_polynomial():
    m, pos = tiny()
    rng = np.random.default_rng(2)
    veff = rng.standard_normal(m.grid.shape)
    sph = m.spheres(pos)
    H = m.dense_H(veff, sph)
    tau = 0.013
    A = -1j * tau * H
    P = np.eye(len(H), dtype=complex)
    Ak = np.eye(len(H), dtype=complex)
    for k in range(1, 5):
        Ak = Ak @ A
        P = P + Ak / math.factorial(k)
    psi = rng.standard_normal((3,) + m.grid.shape) + 1j * rng.standard_normal((3,) + m.grid.shape)
    got = dynamics.taylor(m, tau, veff, sph, psi).reshape(3, -1)
    want = (P @ psi.reshape(3, -1).T).T
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_taylor_is_close_to_exact_exponential_within_truncation_bound():
    m, pos = tiny()
    rng = np.random.default_rng(3)
    veff = rng.standard_normal(m.grid.shape)
    sph = m.spheres(pos)
    H = m.dense_H(veff, sph)
    nrm = np.linalg.norm(H, 2)
    for tau in (0.002, 0.005, 0.01):
        U = scipy.linalg.expm(-1j * tau * H)
        psi = rng.standard_normal(m.grid.N) + 1j * rng.standard_normal(m.grid.N)
        psi /= np.linalg.norm(psi)
        got = dynamics.taylor(m, tau, veff, sph, psi.reshape((1,) + m.grid.shape)).ravel()
        x = tau * nrm
        bound = sum(x ** k / math.factorial(k) for k in range(5, 30))
        err = np.linalg.norm(got - U @ psi)
        assert err <= bound * 1.0001 + 1e-14
        assert err > 1e-3 * bound        # the bound is not vacuous


def test_taylor4_amplification_closed_form_on_eigenvectors():
    # for an eigenvector with eigenvalue lam, theta = tau*lam:
    # |T4|^2 = 1 - theta^6/72 + theta^8/576; contractive iff theta < 2 sqrt 2
    m, _ = tiny(n=10, h=0.3)
    g = m.grid
    x, y, z = g.coords()
    k = 2 * np.pi * np.array([3, -2, 4]) / g.L
    f = (np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) * np.ones(g.shape))[None]
    v0 = 0.25
    lam = -0.5 * sum(float(g.fd_symbol(np.array(kk))) for kk in k) + v0
    for theta in (0.3, 1.0, 2.0, 2.8, 2.9, 3.5):
        tau = theta / lam
        out = dynamics.taylor(m, tau, np.full(g.shape, v0), [], f)
        amp = float(np.mean(np.abs(out) ** 2))
        closed = 1 - theta ** 6 / 72 + theta ** 8 / 576
        assert abs(amp - closed) < 1e-12 * max(1, closed)
        assert (amp < 1.0) == (theta < 2 * math.sqrt(2))
        # reversal with -tau multiplies each eigencomponent by |T4|^2 as well
        back = dynamics.taylor(m, -tau, np.full(g.shape, v0), [], out)
        assert np.abs(back - closed * f).max() < 1e-12 * max(1, closed)


def c1_state(**over):
    cfg = W.C1
    inp = W.make_inputs(cfg)
    m = Model.from_config(cfg, **over)
    return m, dynamics.init_state(m, inp["psi"], inp["pos"])


def test_mu_enters_only_as_electronic_time():
    m1, s1 = c1_state(freeze_ions=True, mu=1.0, dt=0.02)
    m4, s4 = c1_state(freeze_ions=True, mu=4.0, dt=0.08)
    for _ in range(3):
        s1 = dynamics.aetrs_step(m1, s1)
        s4 = dynamics.aetrs_step(m4, s4)
    assert np.abs(s1.psi - s4.psi).max() < 1e-14


def test_basis_rotation_covariance():
    m, s = c1_state()
    rng = np.random.default_rng(7)
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    U = scipy.linalg.expm(-1j * 0.5 * (A + A.conj().T))     # exp(-iS), S Hermitian
    rot = np.einsum("ab,bzyx->azyx", U, s.psi)
    sr = dynamics.init_state(m, rot, s.pos)
    for _ in range(3):
        s = dynamics.aetrs_step(m, s)
        sr = dynamics.aetrs_step(m, sr)
    assert np.abs(np.einsum("ab,bzyx->azyx", U, s.psi) - sr.psi).max() < 1e-12
    assert np.abs(s.rho - sr.rho).max() < 1e-12 * s.rho.max()
    assert np.abs(s.pos - sr.pos).max() < 1e-12


def test_orthonormality_and_energy_drift_shrink_with_dt():
    errs, drifts = [], []
    for dt, ns in ((0.02, 10), (0.01, 20)):
        m, s = c1_state(dt=dt)
        e0 = dynamics.total_energy(m, s)["total"]
        worst = 0.0
        for _ in range(ns):
            s = dynamics.aetrs_step(m, s)
            S = m.overlaps(s.psi)
            worst = max(worst, float(np.abs(S - np.eye(len(S))).max()))
        errs.append(worst)
        drifts.append(abs(dynamics.total_energy(m, s)["total"] - e0))
    assert errs[0] < 1e-6
    assert errs[1] < errs[0] / 8          # Taylor-4 norm defect ~ tau^6 per step
    assert drifts[1] < drifts[0] / 3      # second-order energy error


def test_time_reversal_returns_close_to_start():
    res = []
    for dt in (0.02, 0.01):
        m, s0 = c1_state(dt=dt)
        s = s0
        for _ in range(4):
            s = dynamics.aetrs_step(m, s)
        mb = Model.from_config(W.C1, dt=-dt)
        sb = dynamics.State(psi=s.psi, pos=s.pos, vel=s.vel, force=s.force, rho=s.rho,
                            hist=list(s.hist))
        for _ in range(4):
            sb = dynamics.aetrs_step(mb, sb)
        res.append((np.abs(sb.psi - s0.psi).max(), np.abs(sb.pos - s0.pos).max()))
    assert res[0][0] < 1e-2 and res[1][0] < res[0][0] / 2
    assert res[1][1] < res[0][1]


def test_frozen_density_evolution_is_linear():
    # with v_eff fixed the map psi -> T4 T4 psi is linear (sec. 4.2 footnote)
    m, s = c1_state(freeze_ions=True)
    pos1, h0, h1 = dynamics.step_hamiltonians(m, s)
    a = s.psi[:2]
    b = s.psi[2:]
    la = dynamics.propagate_orbitals(m, a + 0.3j * b, h0, h1)
    lb = dynamics.propagate_orbitals(m, a, h0, h1) + 0.3j * dynamics.propagate_orbitals(m, b, h0, h1)
    assert np.abs(la - lb).max() < 1e-13
