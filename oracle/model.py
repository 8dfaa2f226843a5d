"""The Kohn-Sham model: Hamiltonian, density, energy and ionic forces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Hamiltonian (eq. new_EoM(a)): H psi = -1/2 Lap psi + v_eff psi + V_NL psi,
  v_eff = V_loc(R) + V_H[rho] + v_x[rho] (+ an optional static potential and
  an optional uniform field eps * x).
* Density (eq. density): rho = f sum_A |psi_A|^2 with occupation f = 2.
* Energy (eq. E_KS, with the nonlocal term added and the ion-ion term in its
  periodic Ewald form):
  E_KS = f sum_A h^3 Re<psi_A|T psi_A> + h^3 sum rho V_loc + E_H + E_x + E_NL + E_ion.
* Forces (eq. new_EoM(b)): F_J = -dE_KS/dR_J at fixed orbitals; the
  orbitals and the ion positions are independent variables of the
  Lagrangian (secs. 2 and 4.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .grid import Grid
from . import kb, potentials


@dataclass
class Model:
    n: int
    h: float
    zval: np.ndarray
    mass: np.ndarray
    loc_a: float = 0.5
    kb_sigma: float = 0.4
    kb_rcut: float = 1.2
    kb_energy: float = 2.0
    occ: float = 2.0
    mu: float = 1.0
    dt: float = 0.02
    taylor_order: int = 4
    freeze_ions: bool = False
    vstatic: Optional[np.ndarray] = None   # extra static local potential
    grid: Grid = field(init=False)

    def __post_init__(self):
        self.grid = Grid(self.n, self.h)
        self.zval = np.asarray(self.zval, dtype=np.float64)
        self.mass = np.asarray(self.mass, dtype=np.float64)

    @classmethod
    def from_config(cls, cfg, **over):
        kw = dict(n=cfg.n, h=cfg.h, zval=np.full(cfg.n_ions, cfg.zval),
                  mass=np.full(cfg.n_ions, cfg.mass), loc_a=cfg.loc_a,
                  kb_sigma=cfg.kb_sigma, kb_rcut=cfg.kb_rcut,
                  kb_energy=cfg.kb_energy, occ=cfg.occ, mu=cfg.mu, dt=cfg.dt,
                  freeze_ions=cfg.freeze_ions)
        kw.update(over)
        return cls(**kw)

    # ------------------------------------------------------------ fields
    def field_x(self) -> np.ndarray:
        """Sawtooth dipole coordinate x_i = h*ix - L/2 on the (z, y, x) grid."""
        x, _, _ = self.grid.coords()
        return np.broadcast_to(x - 0.5 * self.grid.L, self.grid.shape).copy()

    def vloc(self, pos: np.ndarray) -> np.ndarray:
        v = potentials.vloc(self.grid, pos, self.zval, self.loc_a)
        if self.vstatic is not None:
            v = v + self.vstatic
        return v

    def spheres(self, pos: np.ndarray):
        return kb.spheres(self.grid, pos, self.kb_sigma, self.kb_rcut)

    def density(self, psi: np.ndarray) -> np.ndarray:
        """rho = f sum_A |psi_A|^2 (eq. density)."""
        return self.occ * np.sum(np.abs(psi) ** 2, axis=0)

    def v_hxc(self, rho: np.ndarray) -> np.ndarray:
        return potentials.v_hxc(self.grid, rho)

    # ------------------------------------------------------------ H
    def apply_H(self, psi: np.ndarray, veff: np.ndarray, sph) -> np.ndarray:
        """H psi for psi of shape [n_orb, z, y, x] (eq. new_EoM(a))."""
        out = self.grid.kinetic(psi) + veff[None] * psi
        if len(sph):
            out = out + kb.apply(self.grid, sph, self.kb_energy, psi)
        return out

    # ------------------------------------------------------------ norms
    def overlaps(self, psi: np.ndarray) -> np.ndarray:
        flat = psi.reshape(psi.shape[0], -1)
        return self.grid.dv * (flat.conj() @ flat.T)

    def norms(self, psi: np.ndarray) -> np.ndarray:
        return self.grid.dv * np.sum(np.abs(psi.reshape(psi.shape[0], -1)) ** 2, axis=1)

    # ------------------------------------------------------------ energy
    def kinetic_sum(self, psi: np.ndarray) -> float:
        """sum over the given orbitals and points of Re(conj(psi) T psi)."""
        return float(np.sum(np.real(np.conj(psi) * self.grid.kinetic(psi))))

    def energy(self, pos: np.ndarray, psi: np.ndarray, rho: Optional[np.ndarray] = None,
               vloc: Optional[np.ndarray] = None, kin_sum: Optional[float] = None) -> dict:
        """kin_sum: kinetic_sum(psi) when already known (e.g. summed over
        chunks of orbitals)."""
        g = self.grid
        if rho is None:
            rho = self.density(psi)
        if vloc is None:
            vloc = self.vloc(pos)
        if kin_sum is None:
            kin_sum = self.kinetic_sum(psi)
        ekin = self.occ * g.dv * kin_sum
        eloc = g.dv * float(np.sum(rho * vloc))
        vh = potentials.hartree(g, rho)
        eh = potentials.hartree_energy(g, rho, vh)
        ex = potentials.slater_energy(g, rho)
        sph = self.spheres(pos)
        c = kb.contract(g, sph, psi)
        enl = kb.energy(c, self.kb_energy, self.occ)
        eion, _ = potentials.ewald(g.L, pos, self.zval)
        parts = {"kinetic": ekin, "local": eloc, "hartree": eh, "xc": ex,
                 "nonlocal": enl, "ion": eion}
        parts["ks"] = sum(parts.values())
        return parts

    # ------------------------------------------------------------ forces
    def forces(self, pos: np.ndarray, psi: np.ndarray, rho: np.ndarray, nl_form: str = "projector",
               floc: Optional[np.ndarray] = None) -> dict:
        """Hellmann-Feynman forces; nl_form "gradient" takes the nonlocal part
        in the wave-function-gradient form (kb.force_columns_gradient).
        floc: the local-potential forces when already known."""
        g = self.grid
        if floc is None:
            floc = potentials.local_forces(g, pos, self.zval, self.loc_a, rho)
        sph = self.spheres(pos)
        c = kb.contract(g, sph, psi)
        if nl_form == "gradient":
            dc = kb.force_columns_gradient(g, sph, psi)
        else:
            dc = kb.force_columns(g, sph, self.kb_sigma, psi)
        fnl = kb.forces(c, dc, self.kb_energy, self.occ)
        _, fion = potentials.ewald(g.L, pos, self.zval)
        return {"local": floc, "nonlocal": fnl, "ion": fion,
                "total": floc + fnl + fion}

    # ------------------------------------------------------------ dense H
    def dense_H(self, veff: np.ndarray, sph) -> np.ndarray:
        """The full N x N matrix of H, column j = H applied to unit vector j.
        Only for tiny grids."""
        N = self.grid.N
        out = np.empty((N, N), dtype=np.complex128)
        chunk = 64
        for j0 in range(0, N, chunk):
            j1 = min(N, j0 + chunk)
            e = np.zeros((j1 - j0, N), dtype=np.complex128)
            e[np.arange(j1 - j0), np.arange(j0, j1)] = 1.0
            out[:, j0:j1] = self.apply_H(e.reshape((-1,) + self.grid.shape), veff,
                                         sph).reshape(j1 - j0, N).T
        return out
