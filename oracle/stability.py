"""Time-step stability limits of the two propagators (sec. 5.1 and the
comparison with CP in sec. 6, Fig. spacing).  TEST INFRASTRUCTURE ONLY.

* The order-K Taylor approximation of exp(-i tau H) multiplies an eigen-
  component of energy E by R_K(-i theta), theta = tau E, R_K(z) = sum_{k<=K}
  z^k / k!.  It is stable while |R_K(-i theta)| <= 1 for every eigenvalue,
  i.e. for |theta| up to the first theta_K > 0 where |R_K(-i theta)| exceeds 1
  (2 sqrt 2 for K = 4).  Each exponential of the AETRS step has
  tau = dt / (2 mu), so dt_max = 2 mu theta_K / max|E|.
* CP's velocity Verlet integrates mu_cp psi'' = -(H - Lambda) psi; a mode of
  frequency omega = sqrt((E - e) / mu_cp) is stable while dt omega <= 2, so
  dt_max = 2 sqrt(mu_cp / (E_max - e_min)) with e_min the lowest occupied
  level (taken as E_min, a bound).
Both scale with E_max, which the finite-difference kinetic term makes
proportional to 1/h^2: dt_max is quadratic in h for the Taylor propagator and
linear for CP.
"""
from __future__ import annotations

import math

import numpy as np

from .model import Model


def taylor_amplification(order: int, theta: float) -> float:
    """|R_K(-i theta)| with R_K the order-K Taylor polynomial of exp."""
    z = -1j * theta
    term, s = 1.0 + 0j, 1.0 + 0j
    for k in range(1, order + 1):
        term = term * z / k
        s = s + term
    return abs(s)


def taylor_stability_limit(order: int) -> float:
    """The first theta > 0 where |R_K(-i theta)| exceeds 1, from the exact
    polynomial P(theta) = |R_K(-i theta)|^2 - 1 (real and imaginary parts of
    R_K as polynomials); 0 when P is positive right after 0 (K = 1, 2, 5, 6)."""
    re = np.zeros(order + 1)
    im = np.zeros(order + 1)
    for k in range(order + 1):
        c = 1.0 / math.factorial(k)
        if k % 2 == 0:
            re[k] = c * (-1) ** (k // 2)
        else:
            im[k] = -c * (-1) ** ((k - 1) // 2)       # (-i)^k, k odd
    P = np.polynomial.polynomial.polyadd(np.polynomial.polynomial.polymul(re, re),
                                         np.polynomial.polynomial.polymul(im, im))
    P[0] -= 1.0
    P[np.abs(P) < 1e-15] = 0.0
    nz = np.nonzero(P)[0]
    if len(nz) == 0:
        return math.inf
    if P[nz[0]] > 0:
        return 0.0
    roots = np.polynomial.polynomial.polyroots(P)
    pos = sorted(r.real for r in roots if abs(r.imag) < 1e-9 and r.real > 1e-9)
    return pos[0] if pos else math.inf


def fd_kinetic_max(h: float) -> float:
    """Largest eigenvalue of -1/2 times the 8th-order FD Laplacian in 3-D: the
    1-D symbol at k = pi, c0 + 2 sum_m c_m (-1)^m, three times, over 2 h^2."""
    c = [-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0]
    sym = c[0] + 2.0 * sum(c[m] * (-1) ** m for m in range(1, 5))
    return -1.5 * sym / (h * h)


def h_extreme_eigenvalues(model: Model, veff: np.ndarray, sph, iters: int = 300, seed: int = 0):
    """(E_min, E_max) of H (v_eff, projectors) by power iteration on H and on
    E_max - H, from a random start."""
    rng = np.random.default_rng(seed)
    shape = (1,) + model.grid.shape

    def rayleigh_top(apply):
        v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        v /= np.linalg.norm(v)
        lam = 0.0
        for _ in range(iters):
            w = apply(v)
            lam = float(np.real(np.vdot(v, w)))
            v = w / np.linalg.norm(w)
        return lam

    hop = lambda v: model.apply_H(v, veff, sph)
    # shift by a bound so the top of the spectrum has the largest magnitude
    shift = abs(float(np.min(veff))) + 1.0
    e_max = rayleigh_top(lambda v: hop(v) + shift * v) - shift
    e_min = e_max - rayleigh_top(lambda v: e_max * v - hop(v))
    return e_min, e_max


def ehrenfest_dt_max(mu: float, order: int, e_abs_max: float) -> float:
    return 2.0 * mu * taylor_stability_limit(order) / e_abs_max


def cp_dt_max(mu_cp: float, e_max: float, e_min: float) -> float:
    return 2.0 * math.sqrt(mu_cp / (e_max - e_min))
