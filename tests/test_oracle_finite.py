"""Pins of the finite-box model: the cell-averaged Coulomb constant against
numerical quadrature, the free-space Hartree sum against the analytic
potential of a Gaussian charge (converging with h), the isolated local
potential against Poisson's equation and its far field, forces against
finite differences of the energies, and the box projector (H Hermitian on
the box, orbitals kept zero outside, norms conserved)."""
import math

import numpy as np
import pytest
from scipy.integrate import tplquad
from scipy.special import erf

import workloads as W
from oracle import dynamics, finite
from oracle.grid import Grid


def test_cell_coulomb_constant():
    val = tplquad(lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z + 1e-300),
                  0, 0.5, 0, 0.5, 0, 0.5, epsabs=1e-10, epsrel=1e-10)[0] * 8
    assert abs(val - finite.CELL_COULOMB) < 1e-6


def _gauss(grid, c, sigma, q=1.0):
    x, y, z = grid.coords()
    r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    return q * (2 * np.pi * sigma ** 2) ** -1.5 * np.exp(-r2 / (2 * sigma ** 2))


def test_hartree_free_converges_to_the_gaussian_potential():
    errs = []
    for n, h in ((24, 0.4), (48, 0.2)):
        g = Grid(n, h)
        c = np.full(3, 0.5 * n * h + 0.013)
        rho = _gauss(g, c, 0.9)
        rho[rho < 1e-13 * rho.max()] = 0.0
        rng = np.random.default_rng(1)
        pts = rng.choice(g.N, 24, replace=False)
        v = finite.hartree_free(g, rho, points=pts)
        x, y, z = (np.broadcast_to(a, g.shape).ravel()[pts] for a in g.coords())
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        want = erf(r / (math.sqrt(2) * 0.9)) / r
        errs.append(np.abs(v - want).max())
    assert errs[0] < 2e-3 and errs[1] < errs[0] / 3.0, errs


def test_hartree_of_a_point_charge_and_reciprocity():
    g = Grid(10, 0.5)
    rho = np.zeros(g.shape)
    rho[3, 4, 5] = 2.0
    v = finite.hartree_free(g, rho)
    x, y, z = g.coords()
    r = np.sqrt((x - 5 * 0.5) ** 2 + (y - 4 * 0.5) ** 2 + (z - 3 * 0.5) ** 2)
    want = g.dv * 2.0 * np.where(r == 0, finite.CELL_COULOMB / 0.5, 1.0 / np.where(r == 0, 1, r))
    assert np.abs(v - want).max() < 1e-14 * np.abs(want).max()
    rng = np.random.default_rng(2)
    a, b = rng.random(g.shape), rng.random(g.shape)
    assert abs(np.sum(a * finite.hartree_free(g, b)) - np.sum(b * finite.hartree_free(g, a))) < 1e-10


def test_isolated_local_potential():
    # -Lap V_loc = 4 pi (charge of the Gaussian ions, -Z (pi a^2)^-3/2 exp(-r^2/a^2));
    # far field -Z / r; smooth through r = 0
    n, h, a = 40, 0.2, 0.8
    g = Grid(n, h)
    R = np.array([[4.0, 4.1, 3.9]])
    Z = np.array([3.0])
    v = finite.vloc_free(g, R, Z, a)
    x, y, z = g.coords()
    r2 = (x - R[0, 0]) ** 2 + (y - R[0, 1]) ** 2 + (z - R[0, 2]) ** 2
    charge = -Z[0] * (np.pi * a * a) ** -1.5 * np.exp(-r2 / (a * a))
    lap = -2.0 * g.kinetic(v[None].astype(np.complex128))[0].real
    inner = (slice(6, -6),) * 3
    assert np.abs(-lap[inner] - 4 * np.pi * charge[inner]).max() < 1e-3 * np.abs(4 * np.pi * charge).max()
    far = finite.vloc_free(g, np.array([[0.0, 0.0, 0.0]]), Z, a)
    assert abs(far[n - 1, n - 1, n - 1] + Z[0] / (math.sqrt(3) * (n - 1) * h)) < 1e-12
    at = finite.vloc_free(g, np.array([[2.0, 2.0, 2.0]]), Z, a)[10, 10, 10]
    near = finite.vloc_free(g, np.array([[2.0 + 1e-6, 2.0, 2.0]]), Z, a)[10, 10, 10]
    assert abs(at - near) < 1e-9


def test_local_and_ion_forces_are_energy_derivatives():
    g = Grid(20, 0.4)
    rng = np.random.default_rng(3)
    pos = np.array([[3.1, 4.0, 3.7], [4.9, 3.6, 4.4]])
    Z = np.array([4.0, 2.0])
    rho = _gauss(g, np.array([4.0, 3.9, 4.1]), 1.1, 6.0) * (1 + 0.1 * rng.random(g.shape))
    f = finite.local_forces_free(g, pos, Z, 0.5, rho)
    fi = finite.ion_coulomb(pos, Z)[1]
    eps = 1e-5
    for J in range(2):
        for c in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[J, c] += eps
            p2[J, c] -= eps
            dE = g.dv * np.sum(rho * (finite.vloc_free(g, p1, Z, 0.5) - finite.vloc_free(g, p2, Z, 0.5))) / (2 * eps)
            assert abs(f[J, c] + dE) < 1e-6 * max(1.0, abs(dE)), (J, c, f[J, c], -dE)
            dI = (finite.ion_coulomb(p1, Z)[0] - finite.ion_coulomb(p2, Z)[0]) / (2 * eps)
            assert abs(fi[J, c] + dI) < 1e-7 * max(1.0, abs(dI))


@pytest.fixture(scope="module")
def f0():
    c = W.F0
    inp = W.make_inputs(c)
    m = finite.FiniteModel.from_config(c, pos0=inp["pos"], radius=c.finite_radius)
    return c, inp, m


def test_box_mask_and_hermitian_h(f0):
    c, inp, m = f0
    assert np.array_equal(m.mask.astype(bool), W.box_mask(c, inp["pos"]))
    g = Grid(8, 0.6)
    mm = finite.FiniteModel(n=8, h=0.6, zval=np.array([1.0]), mass=np.array([1.0]),
                            pos0=np.array([[2.4, 2.4, 2.4]]), radius=1.3)
    veff = mm.vloc(mm.pos0) + 0.1
    H = mm.dense_H(veff, mm.spheres(mm.pos0))
    inside = mm.mask.astype(bool).ravel()
    assert 0 < inside.sum() < g.N
    Hb = H[np.ix_(inside, inside)]                  # P H P on the box
    assert np.abs(Hb - Hb.conj().T).max() < 1e-12 * np.abs(Hb).max()
    assert np.abs(H[~inside]).max() == 0.0          # nothing leaves the box


def test_forces_are_the_energy_gradient_and_steps_keep_the_box(f0):
    c, inp, m = f0
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    eps = 1e-4
    for J, k in ((0, 0), (1, 2)):
        p1, p2 = st.pos.copy(), st.pos.copy()
        p1[J, k] += eps
        p2[J, k] -= eps
        dE = (m.energy(p1, st.psi)["ks"] - m.energy(p2, st.psi)["ks"]) / (2 * eps)
        assert abs(st.force[J, k] + dE) < 1e-5 * max(1.0, abs(dE)), (J, k, st.force[J, k], -dE)
    for _ in range(2):
        st = dynamics.aetrs_step(m, st)
    out = ~m.mask.astype(bool)
    assert np.abs(st.psi[:, out]).max() == 0.0
    assert np.abs(m.norms(st.psi) - 1.0).max() < 1e-8
