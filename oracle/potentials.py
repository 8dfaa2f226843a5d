"""Local ionic potential, Hartree, Slater exchange and Ewald ion-ion terms.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper regenerates the ionic potential V_ion = sum_J V_J^loc(r - R_J) at
every step (sec. 5.2, eq. ionicpotential) and takes the local-potential
forces from it (eq. ionicforces).  Here V_J^loc = -Z_J erf(|r-R_J|/a)/|r-R_J|
in a periodic cube with a neutralising background, evaluated as its Fourier
series over the FFT box (G = 0 dropped).  The printed sign of eq.
ionicforces is ambiguous; the force here is the exact negative derivative of
the discrete energy h^3 sum_i rho_i V_loc(r_i) with respect to R_J.

Hartree: V_H(G) = 4 pi rho(G)/G^2 (G != 0).  Exchange: Slater (LDA exchange
of the spin-unpolarised uniform gas).  Ion-ion: the Ewald energy of point
charges with a neutralising background (the last term of eq. E_KS made
periodic).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .grid import Grid


# ------------------------------------------------------------------ V_loc
def structure_factor(grid: Grid, pos: np.ndarray, zval: np.ndarray) -> np.ndarray:
    """S(G) = sum_J Z_J exp(-i G.R_J) on the FFT box."""
    gx, gy, gz, _ = grid.gvectors()
    s = np.zeros(grid.shape, dtype=np.complex128)
    for J in range(len(pos)):
        x, y, z = pos[J]
        s += zval[J] * np.exp(-1j * (gx * x + gy * y + gz * z))
    return s


def vloc_form_factor(grid: Grid, a: float) -> np.ndarray:
    """v(G) = -(4 pi / G^2) exp(-G^2 a^2 / 4) per unit charge, 0 at G = 0:
    the Fourier transform of -erf(r/a)/r."""
    _, _, _, g2 = grid.gvectors()
    with np.errstate(divide="ignore", invalid="ignore"):
        v = -4.0 * np.pi / g2 * np.exp(-g2 * a * a / 4.0)
    v[0, 0, 0] = 0.0
    return v


def vloc(grid: Grid, pos: np.ndarray, zval: np.ndarray, a: float) -> np.ndarray:
    """V_loc(r_i) = Re[(1/Omega) sum_G v(G) S(G) exp(i G.r_i)] (eq. ionicpotential)."""
    vg = vloc_form_factor(grid, a) * structure_factor(grid, pos, zval)
    # numpy's ifftn carries 1/N; (1/Omega) sum_G = (N/Omega) * ifftn = ifftn / h^3
    return np.real(np.fft.ifftn(vg)) / grid.dv


def rho_g(grid: Grid, rho: np.ndarray) -> np.ndarray:
    """rho(G) = h^3 sum_i rho_i exp(-i G.r_i)."""
    return grid.dv * np.fft.fftn(rho)


def local_forces(grid: Grid, pos: np.ndarray, zval: np.ndarray, a: float,
                 rho: np.ndarray) -> np.ndarray:
    """F_J = -d/dR_J [h^3 sum_i rho_i V_loc(r_i)]
           = (1/Omega) Re sum_G conj(rho(G)) (i G) v(G) Z_J exp(-i G.R_J)."""
    gx, gy, gz, _ = grid.gvectors()
    v = vloc_form_factor(grid, a)
    w = np.conj(rho_g(grid, rho)) * v
    f = np.zeros((len(pos), 3))
    for J in range(len(pos)):
        x, y, z = pos[J]
        t = w * zval[J] * np.exp(-1j * (gx * x + gy * y + gz * z))
        for c, g in enumerate((gx, gy, gz)):
            f[J, c] = np.real(np.sum(1j * g * t)) / grid.omega
    return f


# ---------------------------------------------------------------- Hartree
def hartree(grid: Grid, rho: np.ndarray) -> np.ndarray:
    """V_H with V_H(G) = 4 pi rho(G) / G^2 for G != 0 and 0 at G = 0."""
    _, _, _, g2 = grid.gvectors()
    rg = np.fft.fftn(rho)
    with np.errstate(divide="ignore", invalid="ignore"):
        k = 4.0 * np.pi / g2
    k[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(rg * k))


def hartree_energy(grid: Grid, rho: np.ndarray, vh: np.ndarray) -> float:
    return 0.5 * grid.dv * float(np.sum(rho * vh))


# ---------------------------------------------------------------- Slater
SLATER_CX = 0.75 * (3.0 / np.pi) ** (1.0 / 3.0)


def slater_energy_density(rho: np.ndarray) -> np.ndarray:
    """e_x(rho) = -(3/4)(3/pi)^(1/3) rho^(4/3) (energy per volume)."""
    return -SLATER_CX * np.cbrt(rho) * rho


def slater_potential(rho: np.ndarray) -> np.ndarray:
    """v_x = d e_x / d rho = -(3 rho / pi)^(1/3)."""
    return -np.cbrt(3.0 * rho / np.pi)


def slater_energy(grid: Grid, rho: np.ndarray) -> float:
    return grid.dv * float(np.sum(slater_energy_density(rho)))


def v_hxc(grid: Grid, rho: np.ndarray) -> np.ndarray:
    return hartree(grid, rho) + slater_potential(rho)


# ---------------------------------------------------------------- Ewald
def _ewald_parts(L: float, pos: np.ndarray, zval: np.ndarray, eta: float,
                 tol: float = 1e-17):
    omega = L ** 3
    npos = len(pos)
    # real-space cutoff: erfc(eta r) < tol
    rc = 1.0
    while erfc(eta * rc) > tol:
        rc *= 1.1
    nmax = int(math.ceil(rc / L)) + 1
    e_real = 0.0
    f_real = np.zeros((npos, 3))
    rng = range(-nmax, nmax + 1)
    shifts = np.array([(i, j, k) for i in rng for j in rng for k in rng], dtype=float) * L
    for J in range(npos):
        for K in range(npos):
            d = pos[J] - pos[K] + shifts          # R_J - R_K + T
            r = np.sqrt((d * d).sum(1))
            m = (r > 1e-12) & (r < rc)
            rr = r[m]
            e_real += 0.5 * zval[J] * zval[K] * float(np.sum(erfc(eta * rr) / rr))
            g = (erfc(eta * rr) / rr ** 2
                 + 2.0 * eta / math.sqrt(math.pi) * np.exp(-(eta * rr) ** 2) / rr)
            f_real[J] += zval[J] * zval[K] * ((g / rr)[:, None] * d[m]).sum(0)
    # reciprocal space: exp(-G^2/(4 eta^2)) < tol
    gc = 2.0 * eta * math.sqrt(-math.log(tol))
    mmax = int(math.ceil(gc * L / (2.0 * math.pi)))
    mr = np.arange(-mmax, mmax + 1)
    mm = np.array(np.meshgrid(mr, mr, mr, indexing="ij")).reshape(3, -1).T
    mm = mm[np.any(mm != 0, axis=1)]
    G = 2.0 * np.pi * mm / L
    g2 = (G * G).sum(1)
    keep = g2 < gc * gc
    G, g2 = G[keep], g2[keep]
    w = np.exp(-g2 / (4.0 * eta * eta)) / g2
    phase = np.exp(1j * (G @ pos.T))                   # [nG, N] e^{i G.R_J}
    S = phase @ zval
    e_rec = 2.0 * math.pi / omega * float(np.sum(w * np.abs(S) ** 2))
    f_rec = np.zeros((npos, 3))
    for J in range(npos):
        im = np.imag(phase[:, J] * np.conj(S))
        f_rec[J] = 4.0 * math.pi * zval[J] / omega * ((w * im)[:, None] * G).sum(0)
    e_self = -eta / math.sqrt(math.pi) * float(np.sum(zval ** 2))
    e_bg = -math.pi * float(np.sum(zval)) ** 2 / (2.0 * omega * eta * eta)
    return e_real + e_rec + e_self + e_bg, f_real + f_rec


def ewald(L: float, pos: np.ndarray, zval: np.ndarray, eta: float | None = None):
    """Ewald energy and forces of point charges Z_J at R_J in a periodic cube of
    side L with a uniform neutralising background.  Returns (E, F[N,3])."""
    if eta is None:
        eta = 5.0 / L
    return _ewald_parts(L, np.asarray(pos, float), np.asarray(zval, float), eta)
