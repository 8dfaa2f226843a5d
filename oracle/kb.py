"""Gaussian s-channel Kleinman-Bylander nonlocal projector.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's Hamiltonian contains the nonlocal part of norm-conserving
pseudopotentials (sec. 5); the workloads replace it by one s-channel
projector per ion,
    p_J(r) = (pi sigma^2)^(-3/4) exp(-|d|^2 / (2 sigma^2)),  |d| < r_cut,
with d the minimum-image vector r - R_J, normalised analytically so that the
continuum integral of p_J^2 is one, and V_NL = E_KB sum_J |p_J><p_J| with the
grid quadrature h^3 sum as the inner product:
    c_JA = h^3 sum_k p_J(r_k) psi_A(r_k),   (V_NL psi_A)(r_k) = E_KB sum_J p_J(r_k) c_JA.
Overlapping spheres simply add.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from .grid import Grid


@dataclass
class Sphere:
    idx: np.ndarray     # flat indices into the (z, y, x) grid
    p: np.ndarray       # projector values
    d: np.ndarray       # [K, 3] minimum-image r_k - R_J


def spheres(grid: Grid, pos: np.ndarray, sigma: float, rcut: float) -> List[Sphere]:
    """Grid points strictly inside r_cut of each ion (minimum image)."""
    x, y, z = grid.coords()
    X = np.broadcast_to(x, grid.shape).ravel()
    Y = np.broadcast_to(y, grid.shape).ravel()
    Z = np.broadcast_to(z, grid.shape).ravel()
    norm = (np.pi * sigma * sigma) ** (-0.75)
    out = []
    for J in range(len(pos)):
        dx = grid.min_image(X - pos[J, 0])
        dy = grid.min_image(Y - pos[J, 1])
        dz = grid.min_image(Z - pos[J, 2])
        d2 = dx * dx + dy * dy + dz * dz
        m = d2 < rcut * rcut
        idx = np.nonzero(m)[0]
        p = norm * np.exp(-d2[m] / (2.0 * sigma * sigma))
        out.append(Sphere(idx, p, np.stack([dx[m], dy[m], dz[m]], axis=1)))
    return out


def contract(grid: Grid, sph: List[Sphere], psi: np.ndarray) -> np.ndarray:
    """c[J, A] = h^3 sum_k p_J(r_k) psi_A(r_k) for psi of shape [n_orb, z, y, x]."""
    flat = psi.reshape(psi.shape[0], -1)
    c = np.zeros((len(sph), psi.shape[0]), dtype=np.complex128)
    for J, s in enumerate(sph):
        c[J] = grid.dv * (flat[:, s.idx] @ s.p)
    return c


def apply(grid: Grid, sph: List[Sphere], ekb: float, psi: np.ndarray) -> np.ndarray:
    """V_NL psi for psi of shape [n_orb, z, y, x]."""
    c = contract(grid, sph, psi)
    out = np.zeros((psi.shape[0], grid.N), dtype=np.complex128)
    for J, s in enumerate(sph):
        # np.add.at accumulates correctly where spheres overlap
        np.add.at(out, (slice(None), s.idx), ekb * np.outer(c[J], s.p))
    return out.reshape(psi.shape)


def force_columns(grid: Grid, sph: List[Sphere], sigma: float,
                  psi: np.ndarray) -> np.ndarray:
    """d[J, A, :] = h^3 sum_k (d_k / sigma^2) p_J(r_k) psi_A(r_k) = d c_JA / d R_J."""
    flat = psi.reshape(psi.shape[0], -1)
    out = np.zeros((len(sph), psi.shape[0], 3), dtype=np.complex128)
    for J, s in enumerate(sph):
        w = s.p[:, None] * s.d / (sigma * sigma)      # [K, 3]
        out[J] = grid.dv * (flat[:, s.idx] @ w)
    return out


def force_columns_gradient(grid: Grid, sph: List[Sphere], psi: np.ndarray) -> np.ndarray:
    """The wave-function-gradient form of d c_JA / d R_J (the footnote of
    sec. 5.1): d/dR_J of p_J(r - R_J) is -grad_r p_J, moved onto the orbital,
    d[J, A, :] = h^3 sum_k p_J(r_k) (grad psi_A)(r_k) with the 8th-order
    finite-difference gradient."""
    g = grid.gradient(psi).reshape(3, psi.shape[0], -1)     # [3, A, N]
    out = np.zeros((len(sph), psi.shape[0], 3), dtype=np.complex128)
    for J, s in enumerate(sph):
        for c in range(3):
            out[J, :, c] = grid.dv * (g[c][:, s.idx] @ s.p)
    return out


def energy(c: np.ndarray, ekb: float, occ: float) -> float:
    """E_NL = f E_KB sum_{J,A} |c_JA|^2."""
    return occ * ekb * float(np.sum(np.abs(c) ** 2))


def forces(c: np.ndarray, dc: np.ndarray, ekb: float, occ: float) -> np.ndarray:
    """F_J = -dE_NL/dR_J = -2 f E_KB sum_A Re[conj(c_JA) dc_JA/dR_J]."""
    return -2.0 * occ * ekb * np.real(np.einsum("ja,jac->jc", np.conj(c), dc))
