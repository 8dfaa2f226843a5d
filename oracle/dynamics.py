"""Taylor exponential, AETRS propagator and velocity Verlet.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One molecular-dynamics step follows the paper's sec. 5.1:

* the orbitals obey i mu dphi/dt = H phi (eq. new_EoM(a)); writing
  mu dphi/dt = dphi/dt_e (eq. transf) the electronic step is the standard
  Ehrenfest one over the electronic time Delta t / mu;
* the propagator is AETRS (eq. aetrs):
  U = exp(-i dt_e/2 H(t+dt)) exp(-i dt_e/2 H(t)), dt_e = dt/mu, with
  H(t+dt) taken from previous steps;
* each exponential is the fourth-order Taylor polynomial
  sum_{k<=4} (-i tau H)^k / k!, tau = dt/(2 mu);
* the ions follow velocity Verlet with F = -grad_R E_KS (eq. new_EoM(b)).

Readings where the paper is silent: the ions are moved first, so the ionic
part of H(t+dt) is evaluated exactly at R(t+dt); only the Hartree-exchange
potential, the part that depends on the not-yet-known orbitals, is
extrapolated from the stored history, quadratically
(3 v_n - 3 v_{n-1} + v_{n-2}), dropping to linear and constant
extrapolation on the first steps.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

from .model import Model


def taylor(model: Model, tau: float, veff: np.ndarray, sph, psi: np.ndarray,
           order: Optional[int] = None) -> np.ndarray:
    """sum_{k=0..order} (-i tau H)^k psi / k!, term by term: t_k = (-i tau / k) H t_{k-1}."""
    order = model.taylor_order if order is None else order
    term = psi
    out = psi.copy()
    for k in range(1, order + 1):
        term = (-1j * tau / k) * model.apply_H(term, veff, sph)
        out = out + term
    return out


def extrapolate(hist: List[np.ndarray]) -> np.ndarray:
    """v_Hxc(t+dt) from the newest-last history (quadratic/linear/constant)."""
    if len(hist) >= 3:
        return 3.0 * hist[-1] - 3.0 * hist[-2] + hist[-3]
    if len(hist) == 2:
        return 2.0 * hist[-1] - hist[-2]
    return hist[-1].copy()


@dataclass
class State:
    psi: np.ndarray             # [n_orb, z, y, x] complex128
    pos: np.ndarray             # [n_ions, 3]
    vel: np.ndarray             # [n_ions, 3]
    force: np.ndarray           # [n_ions, 3] total force at pos
    rho: np.ndarray
    hist: List[np.ndarray] = field(default_factory=list)
    step: int = 0


def init_state(model: Model, psi: np.ndarray, pos: np.ndarray,
               vel: Optional[np.ndarray] = None) -> State:
    pos = np.asarray(pos, dtype=np.float64).copy()
    vel = np.zeros_like(pos) if vel is None else np.asarray(vel, np.float64).copy()
    rho = model.density(psi)
    f = model.forces(pos, psi, rho)["total"]
    return State(psi=psi.copy(), pos=pos, vel=vel, force=f, rho=rho,
                 hist=[model.v_hxc(rho)])


def step_hamiltonians(model: Model, st: State, eps: float = 0.0):
    """New positions and the two (v_eff, spheres) pairs of one AETRS step."""
    dt = model.dt
    if model.freeze_ions:
        pos1 = st.pos.copy()
    else:
        pos1 = st.pos + st.vel * dt + st.force * (dt * dt) / (2.0 * model.mass[:, None])
    ext = eps * model.field_x() if eps != 0.0 else 0.0
    veff0 = model.vloc(st.pos) + st.hist[-1] + ext
    veff1 = model.vloc(pos1) + extrapolate(st.hist) + ext
    return pos1, (veff0, model.spheres(st.pos)), (veff1, model.spheres(pos1))


def propagate_orbitals(model: Model, psi: np.ndarray, h0, h1) -> np.ndarray:
    """psi(t+dt) = T4(tau, H(t+dt)) T4(tau, H(t)) psi(t), each orbital independent."""
    tau = model.dt / (2.0 * model.mu)
    half = taylor(model, tau, h0[0], h0[1], psi)
    return taylor(model, tau, h1[0], h1[1], half)


def aetrs_step(model: Model, st: State, eps: float = 0.0) -> State:
    pos1, h0, h1 = step_hamiltonians(model, st, eps)
    psi1 = propagate_orbitals(model, st.psi, h0, h1)
    rho1 = model.density(psi1)
    hist = (st.hist + [model.v_hxc(rho1)])[-3:]
    f1 = model.forces(pos1, psi1, rho1)["total"]
    if model.freeze_ions:
        vel1 = st.vel.copy()
    else:
        vel1 = st.vel + (st.force + f1) * model.dt / (2.0 * model.mass[:, None])
    return State(psi=psi1, pos=pos1, vel=vel1, force=f1, rho=rho1, hist=hist,
                 step=st.step + 1)


def etrs_step(model: Model, st: State, eps: float = 0.0, iterations: int = 2) -> State:
    """The enforced time-reversal-symmetry propagator that AETRS approximates
    (sec. 5.1): the second exponential uses H(t+dt) built from the density of
    the orbitals it produces.  Here: the AETRS result (extrapolated v_Hxc) is
    the prediction, then `iterations` corrections recompute the second
    exponential from the half-step orbitals with v_Hxc of the latest
    density.  iterations = 0 is AETRS."""
    pos1, h0, h1 = step_hamiltonians(model, st, eps)
    tau = model.dt / (2.0 * model.mu)
    half = taylor(model, tau, h0[0], h0[1], st.psi)
    psi1 = taylor(model, tau, h1[0], h1[1], half)
    ext = eps * model.field_x() if eps != 0.0 else 0.0
    for _ in range(iterations):
        veff1 = model.vloc(pos1) + model.v_hxc(model.density(psi1)) + ext
        psi1 = taylor(model, tau, veff1, h1[1], half)
    rho1 = model.density(psi1)
    hist = (st.hist + [model.v_hxc(rho1)])[-3:]
    f1 = model.forces(pos1, psi1, rho1)["total"]
    if model.freeze_ions:
        vel1 = st.vel.copy()
    else:
        vel1 = st.vel + (st.force + f1) * model.dt / (2.0 * model.mass[:, None])
    return State(psi=psi1, pos=pos1, vel=vel1, force=f1, rho=rho1, hist=hist,
                 step=st.step + 1)


def total_energy(model: Model, st: State) -> dict:
    parts = model.energy(st.pos, st.psi, st.rho)
    parts["ion_kinetic"] = 0.5 * float(np.sum(model.mass[:, None] * st.vel ** 2))
    parts["total"] = parts["ks"] + parts["ion_kinetic"]
    return parts


def run(model: Model, st: State, steps: int, ctrl: Optional[np.ndarray] = None,
        callback=None) -> State:
    for n in range(steps):
        eps = 0.0 if ctrl is None else float(ctrl[n])
        st = aetrs_step(model, st, eps)
        if callback is not None:
            callback(st)
    return st
