"""Orbital-parallel driver of the oracle's AETRS step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Inside one AETRS step the orbitals are independent once v_eff(t), the
extrapolated v_Hxc(t+dt) and R(t+dt) are fixed: the paper distributes them
over processors on exactly this ground (sec. 5.2).  This driver keeps the
orbitals in one shared-memory array, propagates chunks of them in worker
processes (one BLAS/OpenMP thread each), and reduces the density, the forces
and the energy in the parent.  Every piece of arithmetic is the oracle's own
(``dynamics.step_hamiltonians``, ``dynamics.taylor``, ``Model.density``,
``Model.forces``, ``Model.energy``, ``potentials``, ``kb``); the driver only
splits the orbital axis, and the ion axis of the per-ion loops of the local
forces and the projector spheres, whose rows are independent.  A step
therefore equals ``dynamics.aetrs_step`` up to the order of the density and
energy sums over orbitals.  The ionic fields of a position set are computed
once and reused by the two steps that need them.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from multiprocessing import shared_memory
from typing import Callable, List, Optional

import numpy as np

from . import dynamics, kb, potentials
from .model import Model

# worker-side state, set in the parent before each fork
_G: dict = {}


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:          # pragma: no cover
        pass


def _task_propagate(span):
    a0, a1 = span
    g = _G
    psi = g["psi"]
    half = dynamics.taylor(g["model"], g["tau"], g["h0"][0], g["h0"][1], psi[a0:a1])
    psi[a0:a1] = dynamics.taylor(g["model"], g["tau"], g["h1"][0], g["h1"][1], half)
    return a0


def _task_kinetic(span):
    a0, a1 = span
    return a0, _G["model"].kinetic_sum(_G["psi"][a0:a1])


def _task_local_forces(span):
    j0, j1 = span
    m = _G["model"]
    return j0, potentials.local_forces(m.grid, _G["pos"][j0:j1], m.zval[j0:j1], m.loc_a, _G["rho"])


def _task_spheres(span):
    j0, j1 = span
    m = _G["model"]
    return j0, kb.spheres(m.grid, _G["pos"][j0:j1], m.kb_sigma, m.kb_rcut)


class _FieldCache:
    """Model proxy whose V_loc and projector spheres are computed once per
    position set (the spheres in the worker pool)."""

    def __init__(self, driver: "Driver"):
        self._d = driver
        self._m = driver.model
        self._vloc = {}
        self._sph = {}

    def __getattr__(self, name):
        return getattr(self._m, name)

    @staticmethod
    def _key(pos):
        return np.ascontiguousarray(pos, dtype=np.float64).tobytes()

    def _trim(self, cache, key):
        while len(cache) > 2:
            cache.pop(next(iter(cache)))

    def vloc(self, pos):
        k = self._key(pos)
        if k not in self._vloc:
            self._vloc[k] = self._m.vloc(pos)
            self._trim(self._vloc, k)
        return self._vloc[k]

    def spheres(self, pos):
        k = self._key(pos)
        if k not in self._sph:
            self._sph[k] = self._d.spheres(pos)
            self._trim(self._sph, k)
        return self._sph[k]


class Driver:
    """Orbitals of one system in shared memory plus a pool of `workers`
    processes (default: every core this process may run on)."""

    def __init__(self, model: Model, n_orb: int, workers: Optional[int] = None,
                 orbitals_per_task: int = 2):
        self.model = model
        self.n_orb = int(n_orb)
        self.workers = int(workers or len(os.sched_getaffinity(0)))
        self.per_task = max(1, int(orbitals_per_task))
        shape = (self.n_orb,) + model.grid.shape
        nbytes = int(np.prod(shape)) * 16
        self._shm = shared_memory.SharedMemory(create=True, size=max(nbytes, 16))
        self.psi = np.ndarray(shape, dtype=np.complex128, buffer=self._shm.buf)
        self.fields = _FieldCache(self)

    def close(self):
        self.psi = None
        self._shm.close()
        self._shm.unlink()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ pool
    def _map(self, fn: Callable, spans: List[tuple], **state):
        _G.clear()
        _G.update(model=self.model, psi=self.psi, **state)
        ctx = mp.get_context("fork")
        with ctx.Pool(min(self.workers, len(spans)), initializer=_init_worker) as pool:
            out = pool.map(fn, spans, chunksize=1)
        _G.clear()
        return out

    def _orbital_spans(self):
        return [(a, min(self.n_orb, a + self.per_task)) for a in range(0, self.n_orb, self.per_task)]

    @staticmethod
    def _ion_spans(n: int, parts: int):
        k = max(1, -(-n // max(1, parts)))
        return [(j, min(n, j + k)) for j in range(0, n, k)]

    # ------------------------------------------------------------ pieces
    def spheres(self, pos):
        if len(pos) == 0:
            return []
        res = dict(self._map(_task_spheres, self._ion_spans(len(pos), self.workers), pos=pos))
        out = []
        for j0 in sorted(res):
            out.extend(res[j0])
        return out

    def local_forces(self, pos, rho):
        f = np.zeros((len(pos), 3))
        if len(pos) == 0:
            return f
        for j0, rows in self._map(_task_local_forces, self._ion_spans(len(pos), self.workers),
                                  pos=pos, rho=rho):
            f[j0:j0 + len(rows)] = rows
        return f

    def density(self) -> np.ndarray:
        """f sum_A |psi_A|^2, summed chunk by chunk of orbitals in order."""
        rho = np.zeros(self.model.grid.shape)
        for a0, a1 in self._orbital_spans():
            rho += self.model.density(self.psi[a0:a1])
        return rho

    def kinetic_sum(self) -> float:
        parts = dict(self._map(_task_kinetic, self._orbital_spans()))
        return float(sum(parts[a] for a in sorted(parts)))

    def propagate(self, h0, h1):
        """psi <- T(tau, H1) T(tau, H0) psi in place, orbital chunks in the pool."""
        tau = self.model.dt / (2.0 * self.model.mu)
        self._map(_task_propagate, self._orbital_spans(), tau=tau, h0=h0, h1=h1)

    # ------------------------------------------------------------ steps
    def init_state(self, psi: np.ndarray, pos: np.ndarray,
                   vel: Optional[np.ndarray] = None) -> dynamics.State:
        """dynamics.init_state for orbitals copied into the shared array."""
        if psi is not self.psi:
            self.psi[...] = psi
        pos = np.asarray(pos, dtype=np.float64).copy()
        vel = np.zeros_like(pos) if vel is None else np.asarray(vel, np.float64).copy()
        rho = self.density()
        f = self.forces(pos, rho)
        return dynamics.State(psi=self.psi, pos=pos, vel=vel, force=f, rho=rho,
                              hist=[self.model.v_hxc(rho)])

    def forces(self, pos, rho) -> np.ndarray:
        floc = self.local_forces(pos, rho)
        return Model.forces(self.fields, pos, self.psi, rho, floc=floc)["total"]

    def aetrs_step(self, st: dynamics.State, eps: float = 0.0) -> dynamics.State:
        """dynamics.aetrs_step with the orbitals propagated in the pool (in place)."""
        m = self.model
        pos1, h0, h1 = dynamics.step_hamiltonians(self.fields, st, eps)
        self.propagate(h0, h1)
        rho1 = self.density()
        hist = (st.hist + [m.v_hxc(rho1)])[-3:]
        f1 = self.forces(pos1, rho1)
        if m.freeze_ions:
            vel1 = st.vel.copy()
        else:
            vel1 = st.vel + (st.force + f1) * m.dt / (2.0 * m.mass[:, None])
        return dynamics.State(psi=self.psi, pos=pos1, vel=vel1, force=f1, rho=rho1, hist=hist,
                              step=st.step + 1)

    def total_energy(self, st: dynamics.State) -> dict:
        """dynamics.total_energy with the kinetic sum taken in the pool."""
        parts = Model.energy(self.fields, st.pos, self.psi, st.rho,
                             vloc=self.fields.vloc(st.pos), kin_sum=self.kinetic_sum())
        parts["ion_kinetic"] = 0.5 * float(np.sum(self.model.mass[:, None] * st.vel ** 2))
        parts["total"] = parts["ks"] + parts["ion_kinetic"]
        return parts
