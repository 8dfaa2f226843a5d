"""Reverse-mode derivative of an AETRS trajectory with frozen ions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward model is the step of ``dynamics`` with the ions held fixed and a
control entering the effective potential of both exponentials of step n as
eps_n * x (x the sawtooth dipole coordinate), plus a static perturbation dV
of the local potential obtained from a coarse periodic grid by trilinear
interpolation.  The objective is the final dipole J = h^3 sum_i x_i rho_i(T).
The paper gives no gradient method (it points at field-driven dynamics only
as an outlook, sec. 7); this module is the plain chain rule, written from the
definitions, and is itself checked against finite differences in the tests.

Complex adjoints follow  xbar = dJ/dRe(x) + i dJ/dIm(x),  so that
dJ = Re sum conj(xbar) dx.

For one exponential y = P(A) psi with A = -i tau H(w), P(A) = sum_k A^k/k!:
  psibar = P(A)^H ybar = P(A^H) ybar, A^H = +i tau H  (H Hermitian),
  wbar(r) = sum_k (1/k!) sum_{j<k} Re[ conj((A^H)^j ybar)(r) * (-i tau) * (A^(k-1-j) psi)(r) ],
summed over orbitals (the term-by-term derivative of the polynomial).
"""
from __future__ import annotations

from math import factorial
from typing import Optional

import numpy as np

from .model import Model
from . import dynamics, potentials


# ------------------------------------------------------------ coarse grid
def interp_matrix_1d(n: int, m: int) -> np.ndarray:
    """Periodic linear interpolation from m coarse to n fine points (n/m integer):
    fine point i sits at coarse coordinate i*m/n."""
    if n % m:
        raise ValueError("fine size must be a multiple of the coarse size")
    r = n // m
    M = np.zeros((n, m))
    for i in range(n):
        i0, t = divmod(i, r)
        t = t / r
        M[i, i0 % m] += 1.0 - t
        M[i, (i0 + 1) % m] += t
    return M


def coarse_to_fine(dv_coarse: np.ndarray, n: int) -> np.ndarray:
    m = dv_coarse.shape[0]
    M = interp_matrix_1d(n, m)
    return np.einsum("zc,yb,xa,cba->zyx", M, M, M, dv_coarse)


def fine_to_coarse_adjoint(g_fine: np.ndarray, m: int) -> np.ndarray:
    n = g_fine.shape[0]
    M = interp_matrix_1d(n, m)
    return np.einsum("zc,yb,xa,zyx->cba", M, M, M, g_fine)


# ------------------------------------------------------------ one exponential
def _taylor_terms(model: Model, tau: float, veff, sph, psi, order: int):
    """F_m = A^m psi, m = 0..order-1, with A = -i tau H."""
    out = [psi]
    for _ in range(order - 1):
        out.append(-1j * tau * model.apply_H(out[-1], veff, sph))
    return out


def exp_adjoint(model: Model, tau: float, veff, sph, psi, ybar, order: Optional[int] = None):
    """(psibar, wbar) of y = T_order(tau, H(w)) psi for the cotangent ybar."""
    order = model.taylor_order if order is None else order
    F = _taylor_terms(model, tau, veff, sph, psi, order)
    B = [ybar]                           # (A^H)^j ybar
    for _ in range(order - 1):
        B.append(1j * tau * model.apply_H(B[-1], veff, sph))
    wbar = np.zeros(model.grid.shape)
    for k in range(1, order + 1):
        ck = 1.0 / factorial(k)
        for j in range(k):
            wbar += ck * np.sum(np.real(np.conj(B[j]) * (-1j * tau) * F[k - 1 - j]), axis=0)
    # psibar = P(A^H) ybar, summed term by term
    psibar = ybar.copy()
    term = ybar
    for k in range(1, order + 1):
        term = (1j * tau / k) * model.apply_H(term, veff, sph)
        psibar = psibar + term
    return psibar, wbar


def _extrap_coeffs(nhist: int):
    if nhist >= 3:
        return (3.0, -3.0, 1.0)
    if nhist == 2:
        return (2.0, -1.0)
    return (1.0,)


def _vhxc_adjoint(model: Model, rho: np.ndarray, vbar: np.ndarray) -> np.ndarray:
    """rhobar contribution of v = V_H[rho] + v_x(rho) for cotangent vbar:
    K vbar (the Hartree kernel is symmetric) + vbar * dv_x/drho."""
    fx = -(1.0 / 3.0) * np.cbrt(3.0 / np.pi) * np.cbrt(rho) ** (-2)
    return potentials.hartree(model.grid, vbar) + vbar * fx


# ------------------------------------------------------------ trajectory
def forward(model: Model, psi0: np.ndarray, pos: np.ndarray, ctrl: np.ndarray,
            dv_coarse: Optional[np.ndarray] = None, keep: bool = False):
    """Frozen-ion trajectory; returns J (and the stored states when keep)."""
    m = _with_static(model, dv_coarse)
    st = dynamics.init_state(m, psi0, pos)
    states = [st] if keep else None
    for n in range(len(ctrl)):
        st = dynamics.aetrs_step(m, st, float(ctrl[n]))
        if keep:
            states.append(st)
    J = objective(m, st.rho)
    return (J, states, m) if keep else J


def objective(model: Model, rho: np.ndarray) -> float:
    return model.grid.dv * float(np.sum(model.field_x() * rho))


def _with_static(model: Model, dv_coarse):
    if dv_coarse is None:
        return model
    import copy
    m = copy.copy(model)
    m.vstatic = coarse_to_fine(dv_coarse, model.n)
    m.freeze_ions = True
    return m


def gradient(model: Model, psi0: np.ndarray, pos: np.ndarray, ctrl: np.ndarray,
             dv_coarse: Optional[np.ndarray] = None):
    """J, dJ/deps[n] and dJ/d(dV_coarse) (or dJ/d(dV_fine) when dv_coarse is None)."""
    if not model.freeze_ions:
        raise ValueError("the adjoint is defined for frozen ions")
    J, states, m = forward(model, psi0, pos, ctrl, dv_coarse, keep=True)
    N = len(ctrl)
    tau = m.dt / (2.0 * m.mu)
    x = m.field_x()
    sph = m.spheres(states[0].pos)
    vloc = m.vloc(states[0].pos)
    v = [m.v_hxc(s.rho) for s in states]          # v_n = v_Hxc(rho_n)
    vbar = [np.zeros(m.grid.shape) for _ in range(N + 1)]
    rhobar_final = m.grid.dv * x
    psibar = np.zeros_like(psi0)
    g_eps = np.zeros(N)
    g_fine = np.zeros(m.grid.shape)
    for n in range(N - 1, -1, -1):
        s1 = states[n + 1]
        rhobar = _vhxc_adjoint(m, s1.rho, vbar[n + 1])
        if n + 1 == N:
            rhobar = rhobar + rhobar_final
        psibar = psibar + 2.0 * m.occ * rhobar[None] * s1.psi
        # forward pieces of step n
        s0 = states[n]
        a = _extrap_coeffs(min(n + 1, 3))
        vt = sum(a[j] * v[n - j] for j in range(len(a)))
        w1 = vloc + v[n] + ctrl[n] * x
        w2 = vloc + vt + ctrl[n] * x
        half = dynamics.taylor(m, tau, w1, sph, s0.psi)
        psibar, wbar2 = exp_adjoint(m, tau, w2, sph, half, psibar)
        psibar, wbar1 = exp_adjoint(m, tau, w1, sph, s0.psi, psibar)
        g_eps[n] = float(np.sum(x * (wbar1 + wbar2)))
        g_fine += wbar1 + wbar2
        vbar[n] += wbar1
        for j in range(len(a)):
            vbar[n - j] += a[j] * wbar2
    if dv_coarse is None:
        return J, g_eps, g_fine
    return J, g_eps, fine_to_coarse_adjoint(g_fine, dv_coarse.shape[0])
