"""Pins of the oracle's reverse-mode gradient of the final dipole with respect
to per-step control amplitudes and a coarse static potential: central finite
differences of the oracle's own forward trajectory, along random and
coordinate directions, and exhaustively on a tiny grid."""
import numpy as np
import pytest

import workloads as W
from oracle import Model, adjoint


def small_problem(n=16, h=0.3, n_orb=4, steps=4, coarse=4, seed=0):
    cfg = W.C1.replace(n=n, h=h, n_orb=n_orb, freeze_ions=True, coarse_n=coarse,
                       control_sigma=0.01, steps=steps, seed=900 + seed)
    inp = W.make_inputs(cfg)
    m = Model.from_config(cfg)
    rng = np.random.default_rng(seed)
    dv = 0.01 * rng.standard_normal((coarse,) * 3)
    return m, inp["psi"], inp["pos"], inp["ctrl"], dv


def test_interpolation_adjoint_is_transpose():
    rng = np.random.default_rng(1)
    c = rng.standard_normal((4, 4, 4))
    f = rng.standard_normal((16, 16, 16))
    lhs = np.sum(adjoint.coarse_to_fine(c, 16) * f)
    rhs = np.sum(c * adjoint.fine_to_coarse_adjoint(f, 4))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # interpolation reproduces coarse values at coincident points and constants exactly
    fine = adjoint.coarse_to_fine(c, 16)
    assert np.abs(fine[::4, ::4, ::4] - c).max() < 1e-15
    assert np.abs(adjoint.coarse_to_fine(np.ones((4, 4, 4)), 16) - 1).max() < 1e-15


def test_gradient_matches_directional_finite_differences():
    m, psi, pos, ctrl, dv = small_problem()
    J, ge, gv = adjoint.gradient(m, psi, pos, ctrl, dv)
    rng = np.random.default_rng(5)
    for trial in range(3):
        de = rng.standard_normal(ctrl.shape)
        dd = rng.standard_normal(dv.shape)
        if trial == 1:
            dd[:] = 0          # controls only
        if trial == 2:
            de[:] = 0          # static potential only
        h = 1e-4
        jp = adjoint.forward(m, psi, pos, ctrl + h * de, dv + h * dd)
        jm = adjoint.forward(m, psi, pos, ctrl - h * de, dv - h * dd)
        fd = (jp - jm) / (2 * h)
        an = float(np.dot(ge, de) + np.sum(gv * dd))
        assert abs(fd - an) < 1e-6 * max(1e-3, abs(fd)), (trial, fd, an)


def test_gradient_every_control_tiny_grid():
    m, psi, pos, ctrl, dv = small_problem(n=8, h=0.35, n_orb=2, steps=5, coarse=4, seed=3)
    J, ge, gv = adjoint.gradient(m, psi, pos, ctrl, dv)
    h = 1e-4
    for n in range(len(ctrl)):
        e = np.zeros_like(ctrl); e[n] = h
        fd = (adjoint.forward(m, psi, pos, ctrl + e, dv)
              - adjoint.forward(m, psi, pos, ctrl - e, dv)) / (2 * h)
        assert abs(fd - ge[n]) < 1e-7 * max(1e-2, abs(fd)), (n, fd, ge[n])
    for idx in [(0, 0, 0), (1, 2, 3), (3, 3, 1)]:
        e = np.zeros_like(dv); e[idx] = h
        fd = (adjoint.forward(m, psi, pos, ctrl, dv + e)
              - adjoint.forward(m, psi, pos, ctrl, dv - e)) / (2 * h)
        assert abs(fd - gv[idx]) < 1e-7 * max(1e-2, abs(fd)), (idx, fd, gv[idx])
