"""Car-Parrinello molecular dynamics on the same Hamiltonian -- the paper's
comparison scheme (sec. 3, eq. L_CP and eq. EoM_CP), whose electronic part
is integrated by RATTLE / velocity Verlet (sec. 5, the paragraph on the CP
implementation, citing Tuckerman and Parrinello 1994).  TEST INFRASTRUCTURE
ONLY, like the rest of this package.

Equations of motion, as read here (the printed signs are garbled):
    mu_cp psi_A'' = -H psi_A + sum_B psi_B Lambda_BA,   <psi_A|psi_B> = delta_AB,
    M_J R_J''    = -grad_J E_KS,
with Lambda Hermitian.  The conserved energy is
    E_CP = f mu_cp sum_A <psi_A'|psi_A'> + E_KS + sum_J M_J |R_J'|^2 / 2
(f the occupation; the factor f makes d/dt E_CP vanish for the orbital
equation without f, the same reading as the Ehrenfest step's).

One step (dt), orbitals as the columns of Psi:
 1. R(t+dt) = R + V dt + F dt^2 / 2M.
 2. Psi~ = Psi + dt Psi' - dt^2/(2 mu_cp) H Psi.
 3. Psi(t+dt) = Psi~ + Psi X with X Hermitian such that Psi(t+dt) is
    orthonormal: A + B^H X + X B + X^2 = I, A = <Psi~|Psi~>, B = <Psi|Psi~>,
    solved by the fixed-point iteration
        X <- ((I - A) + X (I - B) + (I - B^H) X - X^2) / 2,   X_0 = (I - A) / 2.
 4. Psi'(t+dt/2) = (Psi(t+dt) - Psi) / dt.
 5. rho, v_Hxc, H Psi and the forces at (Psi(t+dt), R(t+dt)) -- no
    extrapolation: the new orbitals are known before H is needed.
 6. Psi'' = Psi'(t+dt/2) - dt/(2 mu_cp) H Psi(t+dt); the velocity
    constraint <Psi'|Psi> + <Psi|Psi'> = 0 fixes
    Psi'(t+dt) = Psi'' + Psi(t+dt) Y,  Y = -(Q + Q^H)/2,  Q = <Psi(t+dt)|Psi''>.
 7. V(t+dt) = V + (F + F(t+dt)) dt / 2M.
The orthonormalisation costs O(N_W^2 N_C) per step (the matrices A, B, Q
and the two rotations), against O(N_W N_C) for the modified Ehrenfest step
(sec. 5, numerical properties).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .model import Model


@dataclass
class CPState:
    psi: np.ndarray      # [n_orb, z, y, x] complex128, orthonormal
    psidot: np.ndarray   # [n_orb, z, y, x] complex128
    pos: np.ndarray      # [n_ions, 3]
    vel: np.ndarray      # [n_ions, 3]
    force: np.ndarray    # [n_ions, 3] total force at (psi, pos)
    rho: np.ndarray
    hpsi: np.ndarray     # H psi at (psi, pos): v_eff = V_loc(R) + v_Hxc[rho]
    step: int = 0


def _h_psi(model: Model, psi: np.ndarray, pos: np.ndarray, rho: np.ndarray) -> np.ndarray:
    veff = model.vloc(pos) + model.v_hxc(rho)
    return model.apply_H(psi, veff, model.spheres(pos))


def _gram(model: Model, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """G[i, j] = <a_i|b_j> = h^3 sum conj(a_i) b_j."""
    fa = a.reshape(a.shape[0], -1)
    fb = b.reshape(b.shape[0], -1)
    return model.grid.dv * (fa.conj() @ fb.T)


def _combine(psi: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Columns of Psi M: out_j = sum_i psi_i M[i, j]."""
    flat = psi.reshape(psi.shape[0], -1)
    return (m.T @ flat).reshape(psi.shape)


def init_state(model: Model, psi: np.ndarray, pos: np.ndarray,
               vel: Optional[np.ndarray] = None, psidot: Optional[np.ndarray] = None) -> CPState:
    pos = np.asarray(pos, dtype=np.float64).copy()
    vel = np.zeros_like(pos) if vel is None else np.asarray(vel, np.float64).copy()
    psi = np.asarray(psi, dtype=np.complex128).copy()
    pd = np.zeros_like(psi) if psidot is None else np.asarray(psidot, np.complex128).copy()
    rho = model.density(psi)
    f = model.forces(pos, psi, rho)["total"]
    return CPState(psi=psi, psidot=pd, pos=pos, vel=vel, force=f, rho=rho,
                   hpsi=_h_psi(model, psi, pos, rho))


def solve_position_constraint(a: np.ndarray, b: np.ndarray, tol: float = 1e-14,
                              max_iter: int = 500):
    """Hermitian X with A + B^H X + X B + X^2 = I (step 3); returns (X, iterations,
    final residual max|A + B^H X + X B + X^2 - I|)."""
    n = a.shape[0]
    eye = np.eye(n)
    x = 0.5 * (eye - a)
    for it in range(1, max_iter + 1):
        x = 0.5 * ((eye - a) + x @ (eye - b) + (eye - b.conj().T) @ x - x @ x)
        res = np.abs(a + b.conj().T @ x + x @ b + x @ x - eye).max()
        if res < tol:
            return x, it, res
    return x, max_iter, res


def cp_step(model: Model, st: CPState, mu_cp: float, dt: float, tol: float = 1e-14) -> CPState:
    # 1. ions
    if model.freeze_ions:
        pos1 = st.pos.copy()
    else:
        pos1 = st.pos + st.vel * dt + st.force * (dt * dt) / (2.0 * model.mass[:, None])
    # 2-3. unconstrained orbital positions, then the constraint rotation
    psit = st.psi + dt * st.psidot - (dt * dt / (2.0 * mu_cp)) * st.hpsi
    a = _gram(model, psit, psit)
    b = _gram(model, st.psi, psit)
    x, _, res = solve_position_constraint(a, b, tol)
    if res >= tol:
        raise RuntimeError(f"position constraint did not converge (residual {res:.2e})")
    psi1 = psit + _combine(st.psi, x)
    # 4. half-step orbital velocities
    pd_half = (psi1 - st.psi) / dt
    # 5. fields, H psi and forces at the new configuration
    rho1 = model.density(psi1)
    hpsi1 = _h_psi(model, psi1, pos1, rho1)
    f1 = model.forces(pos1, psi1, rho1)["total"]
    # 6. velocity half kick and the velocity constraint
    pdd = pd_half - (dt / (2.0 * mu_cp)) * hpsi1
    q = _gram(model, psi1, pdd)
    y = -0.5 * (q + q.conj().T)
    pd1 = pdd + _combine(psi1, y)
    # 7. ion velocities
    if model.freeze_ions:
        vel1 = st.vel.copy()
    else:
        vel1 = st.vel + (st.force + f1) * dt / (2.0 * model.mass[:, None])
    return CPState(psi=psi1, psidot=pd1, pos=pos1, vel=vel1, force=f1, rho=rho1,
                   hpsi=hpsi1, step=st.step + 1)


def energy(model: Model, st: CPState, mu_cp: float) -> dict:
    parts = model.energy(st.pos, st.psi, st.rho)
    parts["fictitious"] = model.occ * mu_cp * float(np.sum(model.norms(st.psidot)))
    parts["ion_kinetic"] = 0.5 * float(np.sum(model.mass[:, None] * st.vel ** 2))
    parts["total"] = parts["ks"] + parts["fictitious"] + parts["ion_kinetic"]
    return parts


def run(model: Model, st: CPState, mu_cp: float, dt: float, steps: int) -> CPState:
    for _ in range(steps):
        st = cp_step(model, st, mu_cp, dt)
    return st
