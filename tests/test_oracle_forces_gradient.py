"""Pins of the wave-function-gradient form of the nonlocal force (the
footnote of sec. 5.1): the first-difference coefficients, the FD gradient of
a plane wave in closed form, agreement with the analytic projector derivative
for smooth orbitals, and finite differences of the energy."""
from fractions import Fraction

import numpy as np

import workloads as W
from oracle import Model, kb
from oracle.grid import Grid, central_first_difference_coeffs


def test_first_difference_coefficients():
    # the textbook 8th-order central first difference
    assert central_first_difference_coeffs(8) == [Fraction(4, 5), Fraction(-1, 5), Fraction(4, 105),
                                                  Fraction(-1, 280)]
    # exact on polynomials up to degree 8
    g = Grid(24, 0.1)
    x = np.arange(24) * 0.1
    for deg in range(1, 9):
        f = np.broadcast_to((x - 1.2) ** deg, g.shape).copy()
        d = g.gradient(f)[0]
        want = deg * (x - 1.2) ** (deg - 1)
        assert np.abs(d[0, 0, 8:16] - want[8:16]).max() < 1e-9 * max(1.0, np.abs(want).max())


def test_plane_wave_gradient_closed_form():
    g = Grid(12, 0.3)
    x, y, z = g.coords()
    k = 2 * np.pi * np.array([2, -1, 3]) / g.L
    f = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    a = [0.8, -0.2, 4 / 105, -1 / 280]
    for c in range(3):
        kt = sum(2 * a[m - 1] * np.sin(m * k[c] * g.h) for m in range(1, 5)) / g.h
        assert np.abs(g.gradient(f)[c] - 1j * kt * f).max() < 1e-12


def test_gradient_form_close_to_projector_derivative_for_smooth_orbitals():
    c = W.C1
    inp = W.make_inputs(c)
    m = Model.from_config(c)
    rho = m.density(inp["psi"])
    fa = m.forces(inp["pos"], inp["psi"], rho)["nonlocal"]
    fg = m.forces(inp["pos"], inp["psi"], rho, nl_form="gradient")["nonlocal"]
    # the same continuum derivative; on the grid they differ by the
    # discretisation and by the step of the projector at its cutoff (3 sigma,
    # where p is 1 % of its peak), which the integration by parts drops:
    # 7.5 % of the largest force at h = 0.3, 2 % at h = 0.2
    assert np.abs(fg - fa).max() < 0.1 * np.abs(fa).max()
    assert np.abs(fg - fa).max() > 0.0


def test_gradient_form_against_finite_difference_of_energy_on_fine_grid():
    # finer grid: the gradient form approaches -dE/dR.  Ion 1 of this
    # configuration has no grid point within 1e-4 of its cutoff sphere, so its
    # E_NL(R) is smooth there (ion 0's is not: a point crosses the cutoff)
    c = W.C1.replace(n=24, h=0.2)
    inp = W.make_inputs(c)
    m = Model.from_config(c)
    psi, pos = inp["psi"], inp["pos"]
    rho = m.density(psi)
    fa = m.forces(pos, psi, rho)["nonlocal"]
    fg = m.forces(pos, psi, rho, nl_form="gradient")["nonlocal"]
    eps, J = 1e-4, 1
    fd = np.zeros(3)
    for ax in range(3):
        e = []
        for s in (+1, -1):
            p2 = pos.copy()
            p2[J, ax] += s * eps
            e.append(kb.energy(kb.contract(m.grid, m.spheres(p2), psi), m.kb_energy, m.occ))
        fd[ax] = -(e[0] - e[1]) / (2 * eps)
    assert np.abs(fa[J] - fd).max() < 1e-6 * np.abs(fd).max()       # the analytic form is exact
    assert np.abs(fg[J] - fd).max() < 0.03 * np.abs(fd).max()        # the gradient form approximates
