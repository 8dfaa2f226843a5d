"""The two-band toy model of sec. 6 (eq. L_toy): two electronic angles
theta_1, theta_2, a bond length R and a gap coordinate G, propagated by the
modified-Ehrenfest Lagrangian, by its Car-Parrinello analogue and compared
with the ground-state Born-Oppenheimer (gsBO) motion, each integrated by the
classical fourth-order Runge-Kutta method.  TEST INFRASTRUCTURE ONLY.

Equations of motion, from the Euler-Lagrange equations of eq. L_toy (the
theta part of the kinetic term is linear in the velocities, so the angles
obey first-order equations):
    mu theta_1' =  (G/2) sin(theta_2 - R)
    mu theta_2' = -(G/2) sin(theta_1 - R)
    M_R R''     = -K_R (R - R_0) + (G/2) [sin(theta_1 - R) + sin(theta_2 - R)]
    M_G G''     = -K_G (G - G_0) + (1/2) [cos(theta_1 - R) + cos(theta_2 - R)]
CP replaces the theta kinetic term by (mu_CP/2)(theta_1'^2 + theta_2'^2):
    mu_CP theta_i'' = -(G/2) sin(theta_i - R).
gsBO sets mu = 0 and theta_1 = theta_2 = R (the minimum of the potential);
then R decouples, M_R R'' = -K_R (R - R_0), and with R(0) = 1.1 R_0,
R'(0) = 0 its motion is R_BO(t) = R_0 + 0.1 R_0 cos(omega_R t),
omega_R = sqrt(K_R / M_R) -- the closed form used as the reference.

Initial conditions (sec. 6): R and G 10 % above R_0 and G_0, at rest; the
angles at the gsBO minimum theta_i = R(0); CP angles at rest.

Distances (sec. 6, read on the samples of a run):
    d_R = 100 / Delta_R * sqrt(mean_j (R(t_j) - R_BO(t_j))^2)
over the samples t_j = j t_s, j = 1..n_s, Delta_R = 0.2 R_0 the full
variation of R_BO.  d_F compares the force on R averaged over consecutive
windows of length tau (between the electronic and the nuclear period: their
geometric mean, rounded to whole samples) with the gsBO force averaged over
the same windows, normalised by Delta_F = K_R Delta_R.  The force average of
a run is the trapezoid rule over its own steps.  Delta t_max (sec. 6): the
largest step whose trajectories of all the dynamical variables -- every
component of the integrated state, velocities included (six for the
first-order angles, eight for CP) -- stay within a distance of 0.1 (the
d-measure above, each variable normalised by its own variation in the
reference) of a run with a much smaller step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# physical constants for the N2 molecule (the paper names the molecule, not the values): bond length 1.09768 A,
# reduced mass of 14N2, harmonic wavenumber 2358.57 cm^-1; atomic units
_BOHR_A = 0.529177210903
_AMU_ME = 1822.888486
_HA_CM = 219474.6313632


@dataclass(frozen=True)
class ToyParams:
    R0: float = 1.09768 / _BOHR_A
    M_R: float = 0.5 * 14.003074 * _AMU_ME
    K_R: float = 0.5 * 14.003074 * _AMU_ME * (2358.57 / _HA_CM) ** 2
    G0: float = 0.30
    M_G: float = 0.5 * 14.003074 * _AMU_ME
    K_G: float = 20.0

    @property
    def omega_R(self) -> float:
        return math.sqrt(self.K_R / self.M_R)

    @property
    def period_R(self) -> float:
        return 2.0 * math.pi / self.omega_R


SCHEMES = ("ehrenfest", "cp")


def potential(p: ToyParams, th1, th2, R, G):
    """The potential energy of eq. L_toy (minus its non-kinetic part)."""
    return (0.5 * p.K_R * (R - p.R0) ** 2 + 0.5 * p.K_G * (G - p.G0) ** 2
            - 0.5 * G * (np.cos(th1 - R) + np.cos(th2 - R)))


def lagrangian(p: ToyParams, scheme: str, mu: float, q, qd):
    """eq. L_toy at coordinates q = (theta_1, theta_2, R, G) and velocities qd
    (the CP variant with its quadratic theta kinetic energy)."""
    th1, th2, R, G = q
    th1d, th2d, Rd, Gd = qd
    if scheme == "ehrenfest":
        kin_th = 0.5 * mu * (th1d * th2 - th2d * th1)
    else:
        kin_th = 0.5 * mu * (th1d ** 2 + th2d ** 2)
    return kin_th + 0.5 * p.M_R * Rd ** 2 + 0.5 * p.M_G * Gd ** 2 - potential(p, th1, th2, R, G)


def rhs(p: ToyParams, scheme: str, mu, y):
    """Time derivative of the state.  Ehrenfest: y = (theta_1, theta_2, R, R',
    G, G'); CP: y = (theta_1, theta_2, theta_1', theta_2', R, R', G, G').
    The last axis holds the state; mu broadcasts over the leading axes."""
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    if scheme == "ehrenfest":
        th1, th2, R, Rd, G, Gd = (y[..., k] for k in range(6))
        s1, s2 = np.sin(th1 - R), np.sin(th2 - R)
        out[..., 0] = 0.5 * G * s2 / mu
        out[..., 1] = -0.5 * G * s1 / mu
        out[..., 2] = Rd
        out[..., 3] = (-p.K_R * (R - p.R0) + 0.5 * G * (s1 + s2)) / p.M_R
        out[..., 4] = Gd
        out[..., 5] = (-p.K_G * (G - p.G0) + 0.5 * (np.cos(th1 - R) + np.cos(th2 - R))) / p.M_G
    else:
        th1, th2, th1d, th2d, R, Rd, G, Gd = (y[..., k] for k in range(8))
        s1, s2 = np.sin(th1 - R), np.sin(th2 - R)
        out[..., 0] = th1d
        out[..., 1] = th2d
        out[..., 2] = -0.5 * G * s1 / mu
        out[..., 3] = -0.5 * G * s2 / mu
        out[..., 4] = Rd
        out[..., 5] = (-p.K_R * (R - p.R0) + 0.5 * G * (s1 + s2)) / p.M_R
        out[..., 6] = Gd
        out[..., 7] = (-p.K_G * (G - p.G0) + 0.5 * (np.cos(th1 - R) + np.cos(th2 - R))) / p.M_G
    return out


def rk4_step(f, y, dt):
    """One step of the classical fourth-order Runge-Kutta method."""
    k1 = f(y)
    k2 = f(y + 0.5 * dt * k1)
    k3 = f(y + 0.5 * dt * k2)
    k4 = f(y + dt * k3)
    return y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def coords(scheme: str, y):
    """(theta_1, theta_2, R, G) of a state."""
    idx = (0, 1, 2, 4) if scheme == "ehrenfest" else (0, 1, 4, 6)
    return np.stack([y[..., k] for k in idx], axis=-1)


def initial_state(p: ToyParams, scheme: str, n: int = 1):
    R, G = 1.1 * p.R0, 1.1 * p.G0
    y = [R, R, R, 0.0, G, 0.0] if scheme == "ehrenfest" else [R, R, 0.0, 0.0, R, 0.0, G, 0.0]
    return np.tile(np.array(y, dtype=np.float64), (n, 1))


def force_R(p: ToyParams, scheme: str, y):
    th1, th2, R, G = (coords(scheme, y)[..., k] for k in range(4))
    return -p.K_R * (R - p.R0) + 0.5 * G * (np.sin(th1 - R) + np.sin(th2 - R))


def energy(p: ToyParams, scheme: str, mu, y):
    """The conserved energy: the theta term of the Ehrenfest Lagrangian is
    linear in the velocities and carries none; CP's carries mu_CP theta'^2/2."""
    th1, th2, R, G = (coords(scheme, y)[..., k] for k in range(4))
    if scheme == "ehrenfest":
        Rd, Gd, kin_th = y[..., 3], y[..., 5], 0.0
    else:
        Rd, Gd = y[..., 5], y[..., 7]
        kin_th = 0.5 * mu * (y[..., 2] ** 2 + y[..., 3] ** 2)
    return kin_th + 0.5 * p.M_R * Rd ** 2 + 0.5 * p.M_G * Gd ** 2 + potential(p, th1, th2, R, G)


def gsbo_R(p: ToyParams, t):
    return p.R0 + 0.1 * p.R0 * np.cos(p.omega_R * np.asarray(t, dtype=np.float64))


def gsbo_force_mean(p: ToyParams, t0, t1):
    """The gsBO force on R, -K_R (R_BO - R_0), averaged over [t0, t1]."""
    w = p.omega_R
    return -p.K_R * 0.1 * p.R0 * (np.sin(w * t1) - np.sin(w * t0)) / (w * (t1 - t0))


def electronic_period(p: ToyParams, scheme: str, mu: float) -> float:
    """Period of the small electronic oscillation about theta_i = R at G = G_0:
    frequency G_0 / (2 mu) for the first-order angles, sqrt(G_0 / (2 mu_CP))
    for CP."""
    if scheme == "ehrenfest":
        return 2.0 * math.pi * 2.0 * mu / p.G0
    return 2.0 * math.pi * math.sqrt(2.0 * mu / p.G0)


def averaging_window(p: ToyParams, scheme: str, mu: float, t_sample: float) -> int:
    """The force-averaging window in whole samples: the geometric mean of the
    electronic and the nuclear period, at least one sample."""
    tau = math.sqrt(electronic_period(p, scheme, mu) * p.period_R)
    return max(1, int(round(tau / t_sample)))


def run(p: ToyParams, scheme: str, mu, substeps: int, n_samples: int, t_total: float, window=None):
    """RK4 over [0, t_total] with dt = t_total / (n_samples * substeps) for a
    set of mu (one trajectory each).  Returns the state at every sample
    (shape [n_mu, n_samples + 1, 6 or 8], the layout of rhs()), d_R and d_F
    per trajectory; `window` (samples per force average) defaults to
    averaging_window per mu."""
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    n = mu.size
    t_s = t_total / n_samples
    dt = t_s / substeps
    if window is None:
        window = [averaging_window(p, scheme, float(m), t_s) for m in mu]
    window = np.broadcast_to(np.asarray(window, dtype=np.int64), (n,))
    y = initial_state(p, scheme, n)
    f = lambda v: rhs(p, scheme, mu, v)
    samples = np.empty((n, n_samples + 1, y.shape[1]))
    samples[:, 0] = y
    sq_R = np.zeros(n)
    sq_F = np.zeros(n)
    n_blocks = np.zeros(n, dtype=np.int64)
    facc = np.zeros(n)
    F = force_R(p, scheme, y)
    step = 0
    for j in range(1, n_samples + 1):
        for _ in range(substeps):
            y = rk4_step(f, y, dt)
            F1 = force_R(p, scheme, y)
            facc += 0.5 * dt * (F + F1)
            F = F1
            step += 1
        samples[:, j] = y
        t = j * t_s
        sq_R += (coords(scheme, y)[:, 2] - gsbo_R(p, t)) ** 2
        done = (j % window) == 0
        if done.any():
            tau = window * t_s
            fbar = facc / tau
            fbo = gsbo_force_mean(p, t - tau, t)
            sq_F = np.where(done, sq_F + (fbar - fbo) ** 2, sq_F)
            n_blocks = n_blocks + done
            facc = np.where(done, 0.0, facc)
    dR = 0.2 * p.R0
    d_R = 100.0 / dR * np.sqrt(sq_R / n_samples)
    d_F = 100.0 / (p.K_R * dR) * np.sqrt(sq_F / np.maximum(n_blocks, 1))
    return {"samples": samples, "d_R": d_R, "d_F": d_F, "dt": dt, "window": np.array(window)}


def trajectory_distance(samples, ref):
    """max over the variables (last axis) of 100 / Delta_x * rms(x - x_ref)
    over the samples, Delta_x the variable's variation (max - min) in the
    reference."""
    samples = np.asarray(samples)
    ref = np.asarray(ref)
    span = ref.max(axis=-2) - ref.min(axis=-2)
    rms = np.sqrt(np.mean((samples - ref) ** 2, axis=-2))
    return np.max(100.0 * rms / span, axis=-1)


def dt_max(p: ToyParams, scheme: str, mu: float, n_samples: int, t_total: float, substeps_list,
           ref_substeps: int, threshold: float = 0.1):
    """The largest step t_total / (n_samples * s), s from `substeps_list`,
    such that it and every smaller step in the list stay within `threshold`
    of the run with ref_substeps."""
    ref = run(p, scheme, mu, ref_substeps, n_samples, t_total)["samples"][0]
    best = None
    for s in sorted(substeps_list, reverse=True):          # smallest step first
        d = trajectory_distance(run(p, scheme, mu, s, n_samples, t_total)["samples"][0], ref)
        if d >= threshold:
            break
        best = t_total / (n_samples * s)
    return best
