"""Pins of the oracle's potentials: local ionic potential (eq. ionicpotential)
and its forces (eq. ionicforces, read as -dE/dR), Hartree, Slater exchange and
the Ewald ion-ion term of eq. E_KS."""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import erf

from oracle import potentials
from oracle.grid import Grid

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constants.json")))


def test_hartree_of_a_cosine_is_exact():
    g = Grid(16, 0.3)
    x, y, z = g.coords()
    k = 2 * np.pi * np.array([1, -2, 3]) / g.L
    rho = np.cos(k[0] * x + k[1] * y + k[2] * z) * np.ones(g.shape)
    vh = potentials.hartree(g, rho)
    assert np.abs(vh - 4 * np.pi * rho / (k @ k)).max() < 1e-12


def test_hartree_of_a_constant_is_zero_and_energy_positive():
    g = Grid(12, 0.3)
    assert np.abs(potentials.hartree(g, np.full(g.shape, 0.7))).max() < 1e-13
    rho = np.random.default_rng(0).random(g.shape)
    vh = potentials.hartree(g, rho)
    assert potentials.hartree_energy(g, rho, vh) > 0


def test_slater_matches_uniform_gas_exchange():
    eps_coeff = GOLD["lda_exchange_per_electron"]["value"]
    for rho in (1e-3, 0.05, 0.7, 3.0):
        rs = (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)
        per_e = float(potentials.slater_energy_density(np.array(rho))) / rho
        assert abs(per_e - eps_coeff / rs) < 1e-12 * abs(per_e)


def test_slater_potential_is_derivative_of_energy():
    rho = np.array([1e-3, 0.02, 0.3, 2.5])
    d = 1e-6 * rho
    fd = (potentials.slater_energy_density(rho + d) - potentials.slater_energy_density(rho - d)) / (2 * d)
    assert np.abs(fd - potentials.slater_potential(rho)).max() < 1e-8 * np.abs(fd).max()


def _vloc_reference(L, r, R, Z, a, b):
    """-Z erf(|r-R|/a)/|r-R|, periodically summed with a neutralising background
    and its cell average removed, by a different Ewald split (parameter b):
    explicit reciprocal sum with exp(-G^2 b^2/4) plus a real-space sum of the
    short-ranged difference [erf(s/b) - erf(s/a)]/s."""
    omega = L ** 3
    mmax = int(math.ceil(2 * 6.0 / b * L / (2 * np.pi))) + 1
    mr = np.arange(-mmax, mmax + 1)
    mm = np.array(np.meshgrid(mr, mr, mr, indexing="ij")).reshape(3, -1).T
    mm = mm[np.any(mm != 0, axis=1)]
    G = 2 * np.pi * mm / L
    g2 = (G * G).sum(1)
    d = r - R
    rec = np.sum(-4 * np.pi * Z / g2 * np.exp(-g2 * b * b / 4) * np.cos(G @ d)) / omega
    nmax = 3
    sr = np.arange(-nmax, nmax + 1)
    T = np.array(np.meshgrid(sr, sr, sr, indexing="ij")).reshape(3, -1).T * L
    s = np.sqrt(((d + T) ** 2).sum(1))
    real = Z * np.sum((erf(s / b) - erf(s / a)) / s)
    return rec + real - Z * np.pi * (a * a - b * b) / omega


def test_vloc_matches_independent_ewald_split_sum():
    g = Grid(16, 0.3)
    a = 1.0    # wide enough that the FFT box truncation is below 1e-12
    pos = np.array([[1.234, 2.1, 0.77], [3.9, 0.4, 4.4]])
    Z = np.array([4.0, 2.5])
    v = potentials.vloc(g, pos, Z, a)
    rng = np.random.default_rng(1)
    for _ in range(12):
        i = rng.integers(0, g.n, size=3)          # (ix, iy, iz)
        r = g.h * i.astype(float)
        ref = sum(_vloc_reference(g.L, r, pos[J], Z[J], a, 0.55) for J in range(2))
        assert abs(v[i[2], i[1], i[0]] - ref) < 1e-11


def test_local_forces_are_minus_energy_gradient():
    g = Grid(16, 0.3)
    rng = np.random.default_rng(2)
    rho = rng.random(g.shape)
    pos = np.array([[1.3, 2.2, 0.9], [3.7, 1.1, 4.0], [2.5, 4.1, 2.2]])
    Z = np.array([4.0, 4.0, 3.0])
    f = potentials.local_forces(g, pos, Z, 0.5, rho)
    d = 1e-4
    for J in range(3):
        for c in range(3):
            pp = pos.copy(); pp[J, c] += d
            pm = pos.copy(); pm[J, c] -= d
            ep = g.dv * np.sum(rho * potentials.vloc(g, pp, Z, 0.5))
            em = g.dv * np.sum(rho * potentials.vloc(g, pm, Z, 0.5))
            assert abs(-(ep - em) / (2 * d) - f[J, c]) < 1e-6 * max(1.0, abs(f[J, c]))


def test_ewald_single_charge_madelung():
    zeta = GOLD["madelung_sc_jellium"]["value"]
    for L, Z in ((1.0, 1.0), (4.8, 4.0), (24.0, 4.0)):
        e, f = potentials.ewald(L, np.array([[0.3, 0.1, 0.2]]) * L, np.array([Z]))
        assert abs(e + zeta * Z * Z / (2 * L)) < 1e-11 * zeta * Z * Z / L
        assert np.abs(f).max() < 1e-11


def test_ewald_is_independent_of_splitting_and_forces_are_gradient():
    L = 6.0
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, L, size=(4, 3))
    Z = np.array([4.0, 4.0, 2.0, 1.0])
    e1, f1 = potentials.ewald(L, pos, Z, eta=0.6)
    e2, f2 = potentials.ewald(L, pos, Z, eta=1.3)
    assert abs(e1 - e2) < 1e-10 * abs(e1)
    assert np.abs(f1 - f2).max() < 1e-9
    assert np.abs(f1.sum(0)).max() < 1e-9         # Newton's third law
    d = 1e-5
    for J in range(4):
        for c in range(3):
            pp = pos.copy(); pp[J, c] += d
            pm = pos.copy(); pm[J, c] -= d
            fd = -(potentials.ewald(L, pp, Z)[0] - potentials.ewald(L, pm, Z)[0]) / (2 * d)
            assert abs(fd - f1[J, c]) < 1e-6 * max(1.0, abs(f1[J, c]))
