"""Pins of the stability limits used by the time-step scans: the Taylor-4
limit 2 sqrt 2 in closed form, the orders without a stable interval, the FD
kinetic spectrum edge against a dense matrix, the power iteration against
the dense spectrum, and the limits against actual propagation."""
import math

import numpy as np

from oracle import Model, dynamics, stability


def test_taylor4_limit_is_two_sqrt_two():
    # |R_4(-i theta)|^2 = 1 - theta^6 / 72 + theta^8 / 576
    assert abs(stability.taylor_stability_limit(4) - 2.0 * math.sqrt(2.0)) < 1e-10
    for t in (0.5, 1.7, 2.8):
        r2 = 1 - t ** 6 / 72 + t ** 8 / 576
        assert abs(stability.taylor_amplification(4, t) ** 2 - r2) < 1e-12


def test_orders_without_a_stable_interval():
    # K = 1, 2 (and 5, 6) grow for every small theta; K = 3 is stable up to sqrt 3
    for k in (1, 2, 5, 6):
        assert stability.taylor_stability_limit(k) == 0.0
    assert abs(stability.taylor_stability_limit(3) - math.sqrt(3.0)) < 1e-10
    assert stability.taylor_stability_limit(8) > stability.taylor_stability_limit(4)


def test_fd_kinetic_edge_against_dense_matrix():
    m = Model(n=8, h=0.37, zval=np.zeros(0), mass=np.zeros(0))
    H = m.dense_H(np.zeros(m.grid.shape), [])
    top = np.linalg.eigvalsh(H).max()
    assert abs(top - stability.fd_kinetic_max(0.37)) < 1e-10 * top


def test_power_iteration_finds_the_spectrum_edges():
    pos = np.array([[0.7, 1.1, 0.9], [2.0, 1.9, 2.3]])
    m = Model(n=8, h=0.35, zval=np.full(2, 4.0), mass=np.full(2, 16000.0))
    rng = np.random.default_rng(4)
    veff = m.vloc(pos) + 0.3 * rng.standard_normal(m.grid.shape)
    sph = m.spheres(pos)
    ev = np.linalg.eigvalsh(m.dense_H(veff, sph))
    e_min, e_max = stability.h_extreme_eigenvalues(m, veff, sph, iters=1500)
    assert abs(e_max - ev.max()) < 1e-3 * abs(ev.max())
    assert abs(e_min - ev.min()) < 2e-2 * (ev.max() - ev.min())


def test_limit_separates_stable_from_growing_propagation():
    # the oracle's own Taylor-4 exponential on a tiny system: just below the
    # limit the norm is kept within the Taylor truncation; just above, the top
    # eigencomponent grows step after step
    m = Model(n=8, h=0.35, zval=np.zeros(0), mass=np.zeros(0))
    veff = np.zeros(m.grid.shape)
    e_max = stability.fd_kinetic_max(0.35)
    tau_lim = stability.taylor_stability_limit(4) / e_max
    x, y, z = m.grid.coords()
    top = np.exp(1j * np.pi / m.h * (x + y + z)).reshape((1,) + m.grid.shape)   # the k = pi mode
    top = top / np.sqrt(m.norms(top)[0])
    for f, grows in ((0.98, False), (1.02, True)):
        psi = top.copy()
        for _ in range(400):
            psi = dynamics.taylor(m, f * tau_lim, veff, [], psi)
        assert (m.norms(psi)[0] > 1.0 + 1e-6) == grows, f
