"""The finite-system geometry of the paper's calculations (sec. 5, Methods,
and the runs of sec. 6): the simulation box is the union of spheres of a
fixed radius around the atoms, orbitals vanish outside it, and the
potentials are those of an isolated system.  TEST INFRASTRUCTURE ONLY.

Readings (the paper uses Octopus with an interpolating-scaling-function
Poisson solver, which is out of scope):
* The grid is the same uniform cube; the box is the set of grid points
  within `radius` of an atom at the start of the run (the box does not follow
  the ions).  H acts as P H P with P the projector onto the box points: the
  orbitals stay zero outside (a zero boundary condition).  The cube must
  leave four empty planes around the box, so the periodic stencil never
  couples the two sides.
* Hartree: the free-space potential of the grid charge,
      v_H(r_i) = h^3 sum_j rho_j g(r_i - r_j),  g(r) = 1/|r|, g(0) = c0 / h,
  c0 = 3 ln(2 + sqrt 3) - pi/2, the average of 1/|r| over a grid cell (the
  potential of a uniform cube of charge at its centre).
* Local ionic potential: the Gaussian ions of the periodic model without
  periodic images, V_loc(r) = -sum_J Z_J erf(|r - R_J| / a) / |r - R_J|
  (-2 Z_J / (a sqrt pi) at r = R_J).
* Ion-ion energy: point charges, sum_{I<J} Z_I Z_J / |R_I - R_J|.
* No uniform external field (the finite runs are field free).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy.special import erf

from .model import Model
from . import kb, potentials

CELL_COULOMB = 3.0 * math.log(2.0 + math.sqrt(3.0)) - 0.5 * math.pi


def sphere_mask(grid, pos0: np.ndarray, radius: float) -> np.ndarray:
    """1.0 at grid points within `radius` of any atom (no periodic images)."""
    x, y, z = grid.coords()
    m = np.zeros(grid.shape, dtype=bool)
    for R in np.asarray(pos0, dtype=np.float64):
        d2 = (x - R[0]) ** 2 + (y - R[1]) ** 2 + (z - R[2]) ** 2
        m |= d2 <= radius * radius
    return m.astype(np.float64)


def coulomb_kernel(r: np.ndarray, h: float) -> np.ndarray:
    with np.errstate(divide="ignore"):
        g = 1.0 / r
    return np.where(r == 0.0, CELL_COULOMB / h, g)


def hartree_free(grid, rho: np.ndarray, points: Optional[np.ndarray] = None, chunk: int = 512) -> np.ndarray:
    """v_H at every grid point (or at the flat indices `points`) by the plain
    sum over the charged points."""
    x, y, z = (np.broadcast_to(c, grid.shape).ravel() for c in grid.coords())
    q = rho.ravel()
    nz = np.nonzero(q)[0]
    src = np.stack([x[nz], y[nz], z[nz]], axis=1)
    qs = q[nz]
    idx = np.arange(grid.N) if points is None else np.asarray(points)
    out = np.zeros(idx.size)
    for k0 in range(0, idx.size, chunk):
        sel = idx[k0:k0 + chunk]
        tgt = np.stack([x[sel], y[sel], z[sel]], axis=1)
        r = np.sqrt(((tgt[:, None, :] - src[None, :, :]) ** 2).sum(axis=2))
        out[k0:k0 + sel.size] = grid.dv * (coulomb_kernel(r, grid.h) @ qs)
    return out.reshape(grid.shape) if points is None else out


def vloc_free(grid, pos: np.ndarray, zval: np.ndarray, a: float) -> np.ndarray:
    x, y, z = grid.coords()
    v = np.zeros(grid.shape)
    for R, Z in zip(np.asarray(pos, dtype=np.float64), zval):
        d = np.sqrt((x - R[0]) ** 2 + (y - R[1]) ** 2 + (z - R[2]) ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = erf(d / a) / d
        v -= Z * np.where(d == 0.0, 2.0 / (a * math.sqrt(math.pi)), t)
    return v


def local_forces_free(grid, pos: np.ndarray, zval: np.ndarray, a: float, rho: np.ndarray) -> np.ndarray:
    """F_J = -d/dR_J h^3 sum_i rho_i V_loc(r_i): with v(d) = -Z erf(d/a)/d,
    dv/dd = Z [erf(d/a)/d^2 - 2 exp(-d^2/a^2) / (a sqrt(pi) d)], and
    dd/dR_J = (R_J - r_i)/d, so F_J = -h^3 sum_i rho_i v'(d) (R_J - r_i)/d."""
    x, y, z = grid.coords()
    f = np.zeros((len(pos), 3))
    for J, (R, Z) in enumerate(zip(np.asarray(pos, dtype=np.float64), zval)):
        dx, dy, dz = R[0] - x, R[1] - y, R[2] - z
        d = np.sqrt(dx * dx + dy * dy + dz * dz)
        with np.errstate(divide="ignore", invalid="ignore"):
            vp = Z * (erf(d / a) / d ** 2 - 2.0 * np.exp(-(d / a) ** 2) / (a * math.sqrt(math.pi) * d))
            w = np.where(d == 0.0, 0.0, rho * vp / d)
        for c, dc in enumerate((dx, dy, dz)):
            f[J, c] = -grid.dv * float(np.sum(w * dc))
    return f


def ion_coulomb(pos: np.ndarray, zval: np.ndarray):
    """(E, F) of point ions: E = sum_{I<J} Z_I Z_J / R_IJ, F = -dE/dR."""
    pos = np.asarray(pos, dtype=np.float64)
    e = 0.0
    f = np.zeros_like(pos)
    for I in range(len(pos)):
        for J in range(I + 1, len(pos)):
            d = pos[I] - pos[J]
            r = math.sqrt(float(d @ d))
            e += zval[I] * zval[J] / r
            g = zval[I] * zval[J] * d / r ** 3
            f[I] += g
            f[J] -= g
    return e, f


@dataclass
class FiniteModel(Model):
    """Model on the union-of-spheres box; `pos0` fixes the box."""
    pos0: np.ndarray = None
    radius: float = 7.6
    mask: np.ndarray = field(init=False, default=None)

    def __post_init__(self):
        super().__post_init__()
        self.mask = sphere_mask(self.grid, self.pos0, self.radius)

    def vloc(self, pos):
        v = vloc_free(self.grid, pos, self.zval, self.loc_a)
        if self.vstatic is not None:
            v = v + self.vstatic
        return v

    def v_hxc(self, rho):
        return hartree_free(self.grid, rho) + potentials.slater_potential(rho)

    def apply_H(self, psi, veff, sph):
        return self.mask[None] * super().apply_H(psi, veff, sph)

    def energy(self, pos, psi, rho=None, vloc=None) -> dict:
        g = self.grid
        if rho is None:
            rho = self.density(psi)
        if vloc is None:
            vloc = self.vloc(pos)
        ekin = self.occ * g.dv * float(np.sum(np.real(np.conj(psi) * g.kinetic(psi))))
        eloc = g.dv * float(np.sum(rho * vloc))
        eh = 0.5 * g.dv * float(np.sum(rho * hartree_free(g, rho)))
        ex = potentials.slater_energy(g, rho)
        c = kb.contract(g, self.spheres(pos), psi)
        enl = kb.energy(c, self.kb_energy, self.occ)
        eion, _ = ion_coulomb(pos, self.zval)
        parts = {"kinetic": ekin, "local": eloc, "hartree": eh, "xc": ex, "nonlocal": enl, "ion": eion}
        parts["ks"] = sum(parts.values())
        return parts

    def forces(self, pos, psi, rho, nl_form: str = "projector") -> dict:
        g = self.grid
        floc = local_forces_free(g, pos, self.zval, self.loc_a, rho)
        sph = self.spheres(pos)
        c = kb.contract(g, sph, psi)
        dc = kb.force_columns_gradient(g, sph, psi) if nl_form == "gradient" else \
            kb.force_columns(g, sph, self.kb_sigma, psi)
        fnl = kb.forces(c, dc, self.kb_energy, self.occ)
        _, fion = ion_coulomb(pos, self.zval)
        return {"local": floc, "nonlocal": fnl, "ion": fion, "total": floc + fnl + fion}

    def field_x(self):
        raise ValueError("the finite-box model runs without an external field")
