"""Periodic real-space grid and the finite-difference kinetic operator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper represents orbitals on a real-space grid and takes derivatives by
finite differences (sec. 5, "Methods").  The order of the stencil is not
given there; this oracle uses the standard 8th-order central second
difference (nine points per axis, 25 points in 3-D).  Its coefficients are
derived here from the Taylor conditions rather than typed in, so the tests
can check them independently (polynomial exactness, plane-wave symbol).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def central_second_difference_coeffs(order: int = 8):
    """Exact rational coefficients c_0..c_{order/2} of the central second
    difference  f''(0) ~ (1/h^2) [c_0 f(0) + sum_m c_m (f(m h) + f(-m h))].

    Solves the moment conditions sum_m c_m * 2 m^(2k) = (2k)! delta_{k,1} for
    k = 1..order/2 together with c_0 + 2 sum c_m = 0, in exact arithmetic."""
    p = order // 2
    # unknowns c_1..c_p ; rows k = 1..p : sum_m 2 m^(2k) c_m = 2 if k == 1 else 0
    a = [[Fraction(2 * m ** (2 * k)) for m in range(1, p + 1)] for k in range(1, p + 1)]
    b = [Fraction(2) if k == 1 else Fraction(0) for k in range(1, p + 1)]
    # Gaussian elimination in exact rationals
    n = p
    for i in range(n):
        piv = next(r for r in range(i, n) if a[r][i] != 0)
        a[i], a[piv] = a[piv], a[i]
        b[i], b[piv] = b[piv], b[i]
        for r in range(n):
            if r != i and a[r][i] != 0:
                f = a[r][i] / a[i][i]
                a[r] = [x - f * y for x, y in zip(a[r], a[i])]
                b[r] = b[r] - f * b[i]
    c = [b[i] / a[i][i] for i in range(n)]
    c0 = -2 * sum(c)
    return [c0] + c


FD8 = tuple(float(x) for x in central_second_difference_coeffs(8))


def central_first_difference_coeffs(order: int = 8):
    """Exact rational a_1..a_{order/2} of f'(0) ~ (1/h) sum_m a_m (f(m h) - f(-m h)):
    the moment conditions sum_m 2 m^(2k-1) a_m = delta_{k,1}, k = 1..order/2."""
    p = order // 2
    a = [[Fraction(2 * m ** (2 * k - 1)) for m in range(1, p + 1)] for k in range(1, p + 1)]
    b = [Fraction(1) if k == 1 else Fraction(0) for k in range(1, p + 1)]
    n = p
    for i in range(n):
        piv = next(r for r in range(i, n) if a[r][i] != 0)
        a[i], a[piv] = a[piv], a[i]
        b[i], b[piv] = b[piv], b[i]
        for r in range(n):
            if r != i and a[r][i] != 0:
                f = a[r][i] / a[i][i]
                a[r] = [x - f * y for x, y in zip(a[r], a[i])]
                b[r] = b[r] - f * b[i]
    return [b[i] / a[i][i] for i in range(n)]


FD8_FIRST = tuple(float(x) for x in central_first_difference_coeffs(8))


class Grid:
    """Periodic cube of n^3 points with spacing h (origin at a corner)."""

    def __init__(self, n: int, h: float):
        self.n = int(n)
        self.h = float(h)
        self.L = self.n * self.h
        self.omega = self.L ** 3
        self.dv = self.h ** 3
        self.N = self.n ** 3

    @property
    def shape(self):
        return (self.n, self.n, self.n)

    def coords(self):
        """x, y, z coordinate arrays broadcastable to (z, y, x)."""
        r = self.h * np.arange(self.n)
        return r[None, None, :], r[:, None][None], r[:, None, None]

    def gvectors(self):
        """Gx, Gy, Gz broadcastable to the (z, y, x) FFT layout and |G|^2.
        Integer wave numbers follow numpy's fftfreq (the most negative one at
        the Nyquist index)."""
        m = np.fft.fftfreq(self.n) * self.n
        g = 2.0 * np.pi * m / self.L
        gx = g[None, None, :]
        gy = g[None, :, None]
        gz = g[:, None, None]
        g2 = gx ** 2 + gy ** 2 + gz ** 2
        return gx, gy, gz, g2

    # ---------------------------------------------------------------- kinetic
    def laplacian(self, f: np.ndarray) -> np.ndarray:
        """8th-order finite-difference Laplacian with periodic wrap, applied to
        the last three axes (z, y, x)."""
        c = FD8
        out = 3.0 * c[0] * f
        for ax in (-1, -2, -3):
            for m in range(1, 5):
                out = out + c[m] * (np.roll(f, m, axis=ax) + np.roll(f, -m, axis=ax))
        return out / (self.h * self.h)

    def gradient(self, f: np.ndarray) -> np.ndarray:
        """8th-order central first differences of f [..., z, y, x] along x, y, z;
        returns [3, ...]."""
        a = FD8_FIRST
        out = []
        for ax in (-1, -2, -3):
            g = np.zeros_like(f)
            for m in range(1, 5):
                g = g + a[m - 1] * (np.roll(f, -m, axis=ax) - np.roll(f, m, axis=ax))
            out.append(g / self.h)
        return np.array(out)

    def kinetic(self, f: np.ndarray) -> np.ndarray:
        """T f = -1/2 Laplacian f (eq. new_EoM(a))."""
        return -0.5 * self.laplacian(f)

    def fd_symbol(self, k: np.ndarray) -> np.ndarray:
        """Eigenvalue of the 1-D FD second difference on exp(i k x)."""
        c = FD8
        s = c[0] + sum(2.0 * c[m] * np.cos(m * k * self.h) for m in range(1, 5))
        return s / (self.h * self.h)

    def inner(self, a: np.ndarray, b: np.ndarray) -> complex:
        return self.dv * complex(np.vdot(a, b))

    def min_image(self, d: np.ndarray) -> np.ndarray:
        return d - self.L * np.round(d / self.L)
