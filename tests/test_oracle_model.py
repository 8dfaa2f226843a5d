"""Pins of the oracle's Hamiltonian (eq. new_EoM(a)), nonlocal projector,
energy (eq. E_KS) and forces (eq. new_EoM(b), -grad_R E_KS at fixed orbitals)."""
import numpy as np
import pytest

import workloads as W
from oracle import Model, kb, potentials
from oracle.grid import Grid


def tiny_model(n=8, h=0.35, pos=None, **kw):
    if pos is None:
        pos = np.array([[0.7, 1.1, 0.9], [2.0, 1.9, 2.3]])
    m = Model(n=n, h=h, zval=np.full(len(pos), 4.0), mass=np.full(len(pos), W.BE9_MASS), **kw)
    return m, pos


def random_orbitals(shape, k, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((k,) + shape) + 1j * rng.standard_normal((k,) + shape)


def test_dense_H_is_hermitian_and_nl_has_rank_n_ions():
    m, pos = tiny_model()
    rng = np.random.default_rng(5)
    veff = rng.standard_normal(m.grid.shape)
    sph = m.spheres(pos)
    H = m.dense_H(veff, sph)
    assert np.abs(H - H.conj().T).max() < 1e-13 * np.abs(H).max()
    H0 = m.dense_H(veff, [])
    ev = np.linalg.eigvalsh(H - H0)
    # E_KB > 0: V_NL is positive semidefinite with exactly n_ions nonzero eigenvalues
    assert ev.min() > -1e-12
    assert int(np.sum(ev > 1e-8)) == len(pos)


def test_nl_is_sum_of_projector_outer_products():
    m, pos = tiny_model()
    sph = m.spheres(pos)
    N = m.grid.N
    P = np.zeros((len(sph), N))
    for J, s in enumerate(sph):
        P[J, s.idx] = s.p
    dense = m.kb_energy * m.grid.dv * P.T @ P
    H = m.dense_H(np.zeros(m.grid.shape), sph) - m.dense_H(np.zeros(m.grid.shape), [])
    assert np.abs(H - dense).max() < 1e-12


def test_overlapping_spheres_add():
    m, _ = tiny_model()
    one = np.array([[1.0, 1.2, 1.4]])
    two = np.array([[1.0, 1.2, 1.4], [1.0, 1.2, 1.4]])
    psi = random_orbitals(m.grid.shape, 2)
    a = kb.apply(m.grid, m.spheres(one), 2.0, psi)
    b = kb.apply(m.grid, m.spheres(two), 2.0, psi)
    assert np.abs(b - 2 * a).max() < 1e-12 * np.abs(a).max()


def test_projector_normalisation_converges():
    # h^3 sum p^2 -> 1 - (weight beyond the cutoff) as h -> 0; the Gaussian
    # p^2 has per-axis variance sigma^2/2, so the tail is a chi(3) tail at 3*sqrt(2)
    from scipy.stats import chi
    tail = chi.sf(3.0 * np.sqrt(2.0), 3)
    g = Grid(40, 0.08)
    s = kb.spheres(g, np.array([[1.6, 1.6, 1.6]]), 0.4, 1.2)[0]
    assert abs(g.dv * np.sum(s.p ** 2) - (1 - tail)) < 2e-3


def test_plane_waves_are_eigenvectors_of_H_without_projectors():
    m, _ = tiny_model(n=10, h=0.3)
    g = m.grid
    x, y, z = g.coords()
    k = 2 * np.pi * np.array([2, -1, 3]) / g.L
    f = (np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) * np.ones(g.shape))[None]
    v0 = -0.37
    Hf = m.apply_H(f, np.full(g.shape, v0), [])
    lam = -0.5 * sum(float(g.fd_symbol(np.array(kk))) for kk in k) + v0
    assert np.abs(Hf - lam * f).max() < 1e-12


def _clear_of_cutoffs(grid, pos, rcut, margin):
    x, y, z = grid.coords()
    X = np.broadcast_to(x, grid.shape).ravel()
    Y = np.broadcast_to(y, grid.shape).ravel()
    Z = np.broadcast_to(z, grid.shape).ravel()
    for p in pos:
        d = np.sqrt(grid.min_image(X - p[0]) ** 2 + grid.min_image(Y - p[1]) ** 2
                    + grid.min_image(Z - p[2]) ** 2)
        if np.min(np.abs(d - rcut)) < margin:
            return False
    return True


def test_total_forces_are_minus_energy_gradient_at_fixed_orbitals():
    cfg = W.C1
    inp = W.make_inputs(cfg)
    m = Model.from_config(cfg)
    pos = inp["pos"].copy()
    rng = np.random.default_rng(11)
    while not _clear_of_cutoffs(m.grid, pos, m.kb_rcut, 5e-4):
        pos = pos + rng.uniform(-0.01, 0.01, size=pos.shape)
    psi = inp["psi"]
    rho = m.density(psi)
    f = m.forces(pos, psi, rho)["total"]
    d = 1e-4
    for J in range(len(pos)):
        for c in range(3):
            pp = pos.copy(); pp[J, c] += d
            pm = pos.copy(); pm[J, c] -= d
            fd = -(m.energy(pp, psi, rho)["ks"] - m.energy(pm, psi, rho)["ks"]) / (2 * d)
            assert abs(fd - f[J, c]) < 2e-6 * max(1.0, abs(f[J, c])), (J, c, fd, f[J, c])


def test_energy_is_quadratic_form_of_H_for_frozen_potential():
    # with the local potential fixed, E_kin + E_loc + E_NL = f h^3 sum_A <psi_A|H|psi_A>
    m, pos = tiny_model(n=12, h=0.3)
    psi = random_orbitals(m.grid.shape, 3, seed=9) * 0.05
    rho = m.density(psi)
    vl = m.vloc(pos)
    e = m.energy(pos, psi, rho, vl)
    Hpsi = m.apply_H(psi, vl, m.spheres(pos))
    q = m.occ * m.grid.dv * float(np.sum(np.real(np.conj(psi) * Hpsi)))
    assert abs(q - (e["kinetic"] + e["local"] + e["nonlocal"])) < 1e-10 * abs(q)


def test_density_integrates_to_electron_count():
    cfg = W.C1
    inp = W.make_inputs(cfg)
    m = Model.from_config(cfg)
    rho = m.density(inp["psi"])
    assert abs(m.grid.dv * rho.sum() - cfg.occ * cfg.n_orb) < 1e-10
    S = m.overlaps(inp["psi"])
    assert np.abs(S - np.eye(cfg.n_orb)).max() < 1e-12
