"""Pins of the oracle's finite-difference kinetic operator (sec. 5: real-space
grid with finite-difference derivatives; 8th-order, 25-point star)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.grid import Grid, FD8, central_second_difference_coeffs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constants.json")))


def test_fd8_matches_published_table():
    want = [Fraction(s) for s in GOLD["fd8_second_derivative"]["values"]]
    assert central_second_difference_coeffs(8) == want


@pytest.mark.parametrize("p", range(0, 12))
def test_1d_stencil_polynomial_exactness(p):
    # the 9-point stencil differentiates x^p exactly for p <= 9 and not for p = 10
    h = 0.37
    x0 = 0.81
    xs = x0 + h * np.arange(-4, 5)
    f = xs.astype(np.float64) ** p
    c = FD8
    approx = (c[0] * f[4] + sum(c[m] * (f[4 + m] + f[4 - m]) for m in range(1, 5))) / h ** 2
    exact = p * (p - 1) * x0 ** (p - 2) if p >= 2 else 0.0
    if p <= 9:
        assert abs(approx - exact) <= 1e-9 * max(1.0, abs(exact))
    else:
        assert abs(approx - exact) > 1e-6


def test_symbol_is_eighth_order():
    g = Grid(16, 0.3)
    # symbol(k) + k^2 ~ C k^10 h^8 for small k h
    k1, k2 = 2.0, 1.0
    e1 = g.fd_symbol(np.array(k1)) + k1 ** 2
    e2 = g.fd_symbol(np.array(k2)) + k2 ** 2
    assert 2 ** 10 * 0.8 < e1 / e2 < 2 ** 10 * 1.2


def test_plane_waves_are_eigenvectors_of_the_laplacian():
    g = Grid(12, 0.3)
    x, y, z = g.coords()
    rng = np.random.default_rng(3)
    for _ in range(5):
        m = rng.integers(-6, 6, size=3)
        k = 2 * np.pi * m / g.L
        f = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) * np.ones(g.shape)
        lam = sum(float(g.fd_symbol(np.array(kk))) for kk in k)
        assert np.abs(g.laplacian(f) - lam * f).max() < 1e-12 * max(1.0, abs(lam))


def test_dense_laplacian_spectrum_equals_closed_form():
    g = Grid(6, 0.4)
    N = g.N
    e = np.eye(N).reshape((N,) + g.shape)
    D = g.laplacian(e).reshape(N, N)
    ev = np.sort(np.linalg.eigvalsh(0.5 * (D + D.T)))
    m = np.fft.fftfreq(g.n) * g.n
    s = np.array([float(g.fd_symbol(np.array(2 * np.pi * mm / g.L))) for mm in m])
    closed = np.sort((s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel())
    assert np.abs(ev - closed).max() < 1e-10 * np.abs(closed).max()


def test_largest_kinetic_eigenvalue():
    # at the Nyquist wave number each axis contributes -6.50159/h^2 to the Laplacian
    for h in (0.3, 0.25):
        g = Grid(8, h)
        s = float(g.fd_symbol(np.array(np.pi / h)))
        assert abs(s * h * h + 6.501587301587) < 1e-9
        tmax = 0.5 * 3 * (-s)
        assert abs(tmax * h * h - 9.752380952) < 1e-7
