"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module holds the configurations (grid, ions, orbitals, propagation
parameters) and the seeded generators of their inputs: ion positions, initial
orbitals and control amplitudes.  It contains none of the method's arithmetic
(no Hamiltonian, no propagator, no density, no forces); both the FP64 CPU
oracle and the GPU library receive the arrays produced here as plain inputs.

Recipe of the inputs (all seeded; see ``rngs``):

* Ion positions.  ``pair``: two ions at L*(1/4,1/2,1/2) and L*(3/4,1/2,1/2)
  plus N(0, 0.1 bohr) jitter per coordinate.  ``uniform``: uniform in the
  periodic cube with rejection of any candidate closer than ``min_sep``
  (minimum image) to an accepted ion.  ``lattice``: simple cubic lattice of
  ceil(N^(1/3)) sites per side, the first N sites in a seeded random order,
  each jittered by U(-jitter, +jitter) per coordinate.
* Orbitals.  Per orbital a complex field with independent N(0,1) real and
  imaginary parts at every grid point, multiplied in Fourier space by
  exp(-(|G| h)^2), normalised to h^3 sum |psi|^2 = 1, then one Loewdin step
  Psi <- Psi S^(-1/2) with S = h^3 Psi^H Psi, so the set is orthonormal under
  the grid quadrature.
* Controls.  Per-step field amplitudes eps_n ~ N(0, sigma), sigma = 0.01 au.

The ion mass is that of beryllium-9 (the element with Z=4), in electron
masses; initial ion velocities are zero.
"""
from __future__ import annotations

import dataclasses
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

AMU_IN_ME = 1822.888486
BE9_MASS = 9.0121831 * AMU_IN_ME

PRECISIONS = ("f64", "f32", "f32_bf16x3")


@dataclass(frozen=True)
class Config:
    """One system: grid, ions, orbitals and propagation parameters (atomic units)."""
    name: str
    n: int                      # grid points per axis (periodic cube)
    h: float                    # grid spacing, bohr
    n_ions: int
    n_orb: int
    mu: float                   # the electronic time-scale parameter
    dt: float                   # ionic time step, au
    steps: int
    placement: str = "uniform"  # pair | uniform | lattice
    min_sep: float = 2.5
    jitter: float = 0.0
    zval: float = 4.0
    mass: float = BE9_MASS
    loc_a: float = 0.5          # V_loc = -Z erf(r/a)/r
    kb_sigma: float = 0.4
    kb_rcut_sigmas: float = 3.0
    kb_energy: float = 2.0
    occ: float = 2.0            # closed shell: two electrons per orbital
    freeze_ions: bool = False
    precision: str = "f64"
    seed: int = 812
    control_sigma: float = 0.0  # > 0: per-step control amplitudes are drawn
    coarse_n: int = 0           # > 0: coarse static-potential perturbation grid
    finite_radius: float = 0.0  # > 0: finite box, the union of spheres of this radius around the ions
    ring_radius: float = 2.64   # placement "ring": atoms on a circle in the xy-plane through the centre

    @property
    def L(self) -> float:
        return self.n * self.h

    @property
    def n_points(self) -> int:
        return self.n ** 3

    @property
    def kb_rcut(self) -> float:
        return self.kb_rcut_sigmas * self.kb_sigma

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


# The five workloads.  Where the workload description leaves a value open the
# chosen value is noted: c2 dt; c3 h/mu/dt; c4 h/mu/dt; c5 h/mu/dt.
C1 = Config("c1_fp64_16", n=16, h=0.3, n_ions=2, n_orb=4, mu=1.0, dt=0.02,
            steps=10, placement="pair", seed=812 + 1)
C2 = Config("c2_single_96", n=96, h=0.25, n_ions=64, n_orb=128, mu=4.0,
            dt=0.08, steps=100, placement="uniform", min_sep=2.5,
            seed=812 + 2, precision="f32")
C4 = Config("c4_precision_128", n=128, h=0.25, n_ions=216, n_orb=432, mu=4.0,
            dt=0.08, steps=20, placement="lattice", jitter=0.25,
            seed=812 + 4, precision="f32_bf16x3")
C5 = Config("c5_adjoint_64", n=64, h=0.25, n_ions=32, n_orb=64, mu=1.0,
            dt=0.02, steps=50, placement="uniform", min_sep=2.5,
            freeze_ions=True, seed=812 + 5, precision="f32",
            control_sigma=0.01, coarse_n=16)

# Finite boxes (the union of 7.6-bohr spheres around the atoms of the
# paper's molecular runs, at its converged spacing 0.35 bohr): a six-atom
# ring of the benzene carbon radius, twelve orbitals; F0 is a small case
# for the oracle (two atoms, 3.5-bohr spheres, 28^3 points).
F3 = Config("f3_ring_finite_72", n=72, h=0.35, n_ions=6, n_orb=12, mu=4.0, dt=0.08, steps=20,
            placement="ring", jitter=0.05, finite_radius=7.6, seed=812 + 33, precision="f32")
F0 = Config("f0_pair_finite_28", n=28, h=0.6, n_ions=2, n_orb=4, mu=1.0, dt=0.02, steps=4,
            placement="ring", ring_radius=0.8, jitter=0.05, finite_radius=3.5, seed=812 + 30)

CONFIGS = {"c1": C1, "c2": C2, "c4": C4, "c5": C5, "f3": F3}

# Two-band toy model (eq. L_toy) with the N2 constants in atomic units: bond
# length 1.09768 A, reduced mass of 14N2, harmonic wavenumber 2358.57 cm^-1;
# the gap G0 = 0.30 Ha and the gap coordinate's mass and force constant
# (M_G = M_R, K_G = 20 Ha) are not given by the paper.
_M_N2 = 0.5 * 14.003074 * AMU_IN_ME
TOY_N2 = dict(R0=1.09768 / 0.529177210903, M_R=_M_N2, K_R=_M_N2 * (2358.57 / 219474.6313632) ** 2,
              G0=0.30, M_G=_M_N2, K_G=20.0)
# the sweep of Fig. 1 (c, d): four gsBO periods sampled 200 times; 2048
# log-spaced masses per scheme; RK4 substeps per sample on a 2^(1/3) ladder
# from 128 down to 1 (the largest stable steps of these masses need 2 to 40),
# below a reference of 512
TOY_SWEEP = dict(periods=4.0, n_samples=200, n_mu=2048, mu_ehrenfest=(0.02, 20.0), mu_cp=(2.0, 2000.0),
                 ladder_steps=28, finest=512, ratio=2 ** (1 / 3))


def batch_configs(n_systems: int = 16, seed: int = 812 + 3,
                  steps: int = 50) -> List[Config]:
    """The batched uneven workload: grids in {32,48,64,80,96}^3, 4-64 ions on
    a jittered lattice, 8-256 orbitals (multiples of 8), complex FP32."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    out = []
    for s in range(n_systems):
        n = int(rng.choice([32, 48, 64, 80, 96]))
        n_ions = int(rng.integers(4, 65))
        n_orb = 8 * int(rng.integers(1, 33))
        out.append(Config(f"c3_sys{s:02d}_{n}", n=n, h=0.25, n_ions=n_ions,
                          n_orb=n_orb, mu=4.0, dt=0.08, steps=steps,
                          placement="lattice", seed=seed * 100 + s,
                          precision="f32"))
    # the lattice jitter is a tenth of the lattice constant
    return [c.replace(jitter=0.1 * c.L / math.ceil(c.n_ions ** (1.0 / 3.0) - 1e-9))
            for c in out]


def rngs(cfg: Config) -> Tuple[np.random.Generator, np.random.Generator,
                               np.random.Generator]:
    """Independent streams for positions, orbitals and controls."""
    ss = np.random.SeedSequence(cfg.seed)
    a, b, c = ss.spawn(3)
    return (np.random.default_rng(a), np.random.default_rng(b),
            np.random.default_rng(c))


def _min_image_dist(a: np.ndarray, b: np.ndarray, L: float) -> np.ndarray:
    d = a[None, :] - b
    d -= L * np.round(d / L)
    return np.sqrt((d * d).sum(-1))


def ion_positions(cfg: Config, rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """[n_ions, 3] float64 positions in [0, L)^3."""
    if rng is None:
        rng = rngs(cfg)[0]
    L = cfg.L
    if cfg.n_ions == 0:
        return np.zeros((0, 3))
    if cfg.placement == "pair":
        base = np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]]) * L
        base = base[: cfg.n_ions]
        pos = base + rng.normal(0.0, 0.1, size=base.shape)
    elif cfg.placement == "uniform":
        acc = []
        tries = 0
        while len(acc) < cfg.n_ions:
            tries += 1
            if tries > 2_000_000:
                raise RuntimeError("could not place ions with the requested separation")
            cand = rng.uniform(0.0, L, size=3)
            if acc and _min_image_dist(cand, np.array(acc), L).min() < cfg.min_sep:
                continue
            acc.append(cand)
        pos = np.array(acc)
    elif cfg.placement == "ring":
        ang = 2.0 * math.pi * np.arange(cfg.n_ions) / cfg.n_ions
        pos = np.stack([cfg.ring_radius * np.cos(ang), cfg.ring_radius * np.sin(ang), np.zeros(cfg.n_ions)], axis=1)
        pos = pos + 0.5 * L + rng.uniform(-cfg.jitter, cfg.jitter, size=pos.shape)
    elif cfg.placement == "lattice":
        side = math.ceil(cfg.n_ions ** (1.0 / 3.0) - 1e-9)
        a = L / side
        sites = np.array([(i, j, k) for i in range(side) for j in range(side)
                          for k in range(side)], dtype=np.float64)
        order = rng.permutation(len(sites))[: cfg.n_ions]
        pos = (sites[order] + 0.5) * a
        pos = pos + rng.uniform(-cfg.jitter, cfg.jitter, size=pos.shape)
    else:
        raise ValueError(cfg.placement)
    return np.mod(pos, L)


def _gsq_smoothing(n: int, h: float) -> np.ndarray:
    m = np.fft.fftfreq(n) * n
    g = 2.0 * np.pi * m / (n * h)
    g2 = g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2
    return np.exp(-g2 * h * h)


def box_mask(cfg: Config, pos: np.ndarray) -> np.ndarray:
    """Finite box: 1 at grid points within cfg.finite_radius of an ion."""
    n, h = cfg.n, cfg.h
    ax = np.arange(n) * h
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    m = np.zeros((n, n, n), dtype=bool)
    for R in pos:
        m |= (x - R[0]) ** 2 + (y - R[1]) ** 2 + (z - R[2]) ** 2 <= cfg.finite_radius ** 2
    return m


def _finite_orbitals(cfg: Config, rng: np.random.Generator, no: int) -> np.ndarray:
    """Finite box: random combinations of atom-centred Gaussians times
    (1, x, y, z) (width 1.2 bohr), zero outside the box, Loewdin-orthonormal."""
    pos = ion_positions(cfg, rngs(cfg)[0])
    n, h = cfg.n, cfg.h
    if no > 4 * len(pos):
        raise ValueError("a finite box holds at most 4 orbitals per ion here")
    ax = np.arange(n) * h
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    basis = []
    for R in pos:
        dx, dy, dz = x - R[0], y - R[1], z - R[2]
        g = np.exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * 1.2 ** 2))
        basis += [g, dx * g, dy * g, dz * g]
    basis = np.stack(basis).reshape(len(basis), -1) * box_mask(cfg, pos).ravel()
    c = rng.standard_normal((no, basis.shape[0])) + 1j * rng.standard_normal((no, basis.shape[0]))
    flat = c @ basis
    h3 = h ** 3
    s = h3 * (flat.conj() @ flat.T)
    s = 0.5 * (s + s.conj().T)
    w, v = np.linalg.eigh(s)
    xm = (v * (1.0 / np.sqrt(w))) @ v.conj().T
    return (xm.T @ flat).reshape(no, n, n, n)


def initial_orbitals(cfg: Config, rng: Optional[np.random.Generator] = None,
                     n_orb: Optional[int] = None) -> np.ndarray:
    """[n_orb, n, n, n] complex128, orthonormal under h^3 sum conj(a) b.

    Axis order is (z, y, x): x is the fastest-varying index in memory."""
    import scipy.fft as sfft
    if rng is None:
        rng = rngs(cfg)[1]
    if cfg.finite_radius > 0:
        return _finite_orbitals(cfg, rng, cfg.n_orb if n_orb is None else n_orb)
    n, h = cfg.n, cfg.h
    no = cfg.n_orb if n_orb is None else n_orb
    filt = _gsq_smoothing(n, h)
    psi = np.empty((no, n, n, n), dtype=np.complex128)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    h3 = h ** 3
    for a in range(no):
        f = rng.standard_normal((2, n, n, n))
        z = f[0] + 1j * f[1]
        z = sfft.ifftn(sfft.fftn(z, workers=workers) * filt, workers=workers)
        z /= math.sqrt(h3 * float(np.vdot(z, z).real))
        psi[a] = z
    flat = psi.reshape(no, -1)
    s = h3 * (flat.conj() @ flat.T)
    s = 0.5 * (s + s.conj().T)
    w, v = np.linalg.eigh(s)
    x = (v * (1.0 / np.sqrt(w))) @ v.conj().T   # S^(-1/2), Hermitian
    xt = np.ascontiguousarray(x.T)
    chunk = 1 << 18
    for i0 in range(0, flat.shape[1], chunk):
        flat[:, i0:i0 + chunk] = xt @ flat[:, i0:i0 + chunk]
    return psi


def initial_orbitals_device(cfg: Config, device="cuda:0", chunk: int = 16):
    """The same recipe as initial_orbitals (complex Gaussian fields, G-space
    smoothing exp(-(|G| h)^2), normalisation, Loewdin orthonormalisation),
    drawn and processed with torch on `device` in FP64: for large benchmark
    batches, where the host recipe takes minutes.  The random fields come
    from torch's generator seeded with cfg.seed, so the values differ from
    initial_orbitals'; the distribution is the same.  Returns a
    [n_orb, n^3] complex128 tensor on `device`."""
    import torch
    n, h, no = cfg.n, cfg.h, cfg.n_orb
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(cfg.seed))
    filt = torch.from_numpy(_gsq_smoothing(n, h)).to(dev)
    h3 = h ** 3
    psi = torch.empty((no, n, n, n), dtype=torch.complex128, device=dev)
    for a0 in range(0, no, chunk):
        a1 = min(no, a0 + chunk)
        f = torch.randn((a1 - a0, 2, n, n, n), generator=gen, dtype=torch.float64, device=dev)
        z = torch.complex(f[:, 0], f[:, 1])
        del f
        z = torch.fft.ifftn(torch.fft.fftn(z, dim=(1, 2, 3)) * filt, dim=(1, 2, 3))
        nrm = (z.abs() ** 2).sum(dim=(1, 2, 3)) * h3
        psi[a0:a1] = z / nrm.sqrt()[:, None, None, None]
        del z
    flat = psi.reshape(no, -1)
    s = h3 * (flat.conj() @ flat.T)
    s = 0.5 * (s + s.conj().T)
    w, v = torch.linalg.eigh(s)
    x = (v * (1.0 / w.sqrt())) @ v.conj().T
    return x.T.contiguous() @ flat


# ---------------------------------------------------------------- per-orbital streams
# The same recipe as initial_orbitals, but each orbital draws its fields from
# a stream of its own (child a of SeedSequence([seed, 4321])), so that any
# machine can draw any subset of the orbitals, in parallel, bit for bit.
# Used where the orbital set is too large for one sequential stream (the
# 128^3 x 432 precision workload, whose FP64 oracle reference is computed on
# one machine and compared on another).

def _orbital_seeds(cfg: Config):
    return np.random.SeedSequence([cfg.seed, 4321]).spawn(cfg.n_orb)


def orbital_fields(cfg: Config, a0: int, a1: int, threads: int = 16) -> np.ndarray:
    """The raw N(0,1) fields of orbitals a0..a1-1: float64 [a1-a0, 2, n, n, n]
    (real and imaginary parts), each orbital from its own stream."""
    import concurrent.futures as cf
    n = cfg.n
    seeds = _orbital_seeds(cfg)[a0:a1]
    out = np.empty((a1 - a0, 2, n, n, n))

    def draw(i):
        np.random.default_rng(seeds[i]).standard_normal(out=out[i])

    with cf.ThreadPoolExecutor(max(1, min(threads, a1 - a0))) as ex:
        list(ex.map(draw, range(a1 - a0)))
    return out


def loewdin_matrix(s: np.ndarray) -> np.ndarray:
    """S^(-1/2) of a Hermitian positive overlap matrix (FP64)."""
    s = 0.5 * (s + s.conj().T)
    w, v = np.linalg.eigh(s)
    return (v * (1.0 / np.sqrt(w))) @ v.conj().T


def initial_orbitals_streamed(cfg: Config, out: Optional[np.ndarray] = None,
                              chunk: int = 8) -> np.ndarray:
    """[n_orb, n, n, n] complex128 (into `out` when given): per-orbital
    streams, smoothing exp(-(|G| h)^2), normalisation, one Loewdin step."""
    import scipy.fft as sfft
    n, h, no = cfg.n, cfg.h, cfg.n_orb
    psi = np.empty((no, n, n, n), dtype=np.complex128) if out is None else out
    filt = _gsq_smoothing(n, h)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    h3 = h ** 3
    for a0 in range(0, no, chunk):
        a1 = min(no, a0 + chunk)
        f = orbital_fields(cfg, a0, a1)
        for i in range(a1 - a0):
            z = f[i, 0] + 1j * f[i, 1]
            z = sfft.ifftn(sfft.fftn(z, workers=workers) * filt, workers=workers)
            z /= math.sqrt(h3 * float(np.vdot(z, z).real))
            psi[a0 + i] = z
    flat = psi.reshape(no, -1)
    s = np.zeros((no, no), dtype=np.complex128)
    step = 1 << 16
    for i0 in range(0, flat.shape[1], step):
        blk = flat[:, i0:i0 + step]
        s += blk.conj() @ blk.T
    xt = np.ascontiguousarray(loewdin_matrix(h3 * s).T)
    for i0 in range(0, flat.shape[1], step):
        flat[:, i0:i0 + step] = xt @ flat[:, i0:i0 + step]
    return psi


def initial_orbitals_streamed_device(cfg: Config, device="cuda:0", chunk: int = 16):
    """initial_orbitals_streamed with the fields drawn on the host (the same
    bits) and the smoothing, normalisation and Loewdin step done by torch on
    `device` in FP64.  Returns [n_orb, n^3] complex128 on `device`."""
    import torch
    n, h, no = cfg.n, cfg.h, cfg.n_orb
    dev = torch.device(device)
    filt = torch.from_numpy(_gsq_smoothing(n, h)).to(dev)
    h3 = h ** 3
    psi = torch.empty((no, n, n, n), dtype=torch.complex128, device=dev)
    for a0 in range(0, no, chunk):
        a1 = min(no, a0 + chunk)
        f = torch.from_numpy(orbital_fields(cfg, a0, a1)).to(dev)
        z = torch.complex(f[:, 0], f[:, 1])
        del f
        z = torch.fft.ifftn(torch.fft.fftn(z, dim=(1, 2, 3)) * filt, dim=(1, 2, 3))
        nrm = (z.abs() ** 2).sum(dim=(1, 2, 3)) * h3
        psi[a0:a1] = z / nrm.sqrt()[:, None, None, None]
        del z
    flat = psi.reshape(no, -1)
    s = h3 * (flat.conj() @ flat.T)
    x = torch.from_numpy(loewdin_matrix(s.cpu().numpy())).to(dev)
    return x.T.contiguous() @ flat


def controls(cfg: Config, rng: Optional[np.random.Generator] = None,
             steps: Optional[int] = None) -> np.ndarray:
    """Per-step control amplitudes eps_n, float64 [steps]."""
    if rng is None:
        rng = rngs(cfg)[2]
    k = cfg.steps if steps is None else steps
    return rng.normal(0.0, cfg.control_sigma, size=k)


def coarse_perturbation(cfg: Config, scale: float, seed_offset: int = 0) -> np.ndarray:
    """A seeded smooth coarse-grid static potential perturbation [m,m,m] float64."""
    rng = np.random.default_rng(np.random.SeedSequence([cfg.seed, 77, seed_offset]))
    m = cfg.coarse_n
    return scale * rng.standard_normal((m, m, m))


def make_inputs(cfg: Config, n_orb: Optional[int] = None) -> dict:
    """Everything a run needs, as plain arrays."""
    rp, ro, rc = rngs(cfg)
    out = {"pos": ion_positions(cfg, rp),
           "psi": initial_orbitals(cfg, ro, n_orb),
           "vel": np.zeros((cfg.n_ions, 3)),
           "zval": np.full(cfg.n_ions, cfg.zval),
           "mass": np.full(cfg.n_ions, cfg.mass)}
    if cfg.control_sigma > 0:
        out["ctrl"] = controls(cfg, rc)
    return out
