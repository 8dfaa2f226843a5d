"""Seeded input generators: determinism, orthonormality and edge cases."""
import numpy as np

import workloads as W


def test_inputs_are_deterministic_and_orthonormal():
    a = W.make_inputs(W.C1)
    b = W.make_inputs(W.C1)
    assert np.array_equal(a["psi"], b["psi"]) and np.array_equal(a["pos"], b["pos"])
    flat = a["psi"].reshape(W.C1.n_orb, -1)
    S = W.C1.h ** 3 * (flat.conj() @ flat.T)
    assert np.abs(S - np.eye(W.C1.n_orb)).max() < 1e-12


def test_placements_respect_their_rules():
    cfg = W.C2.replace(n=32, n_orb=1)
    pos = W.ion_positions(cfg.replace(n_ions=20, min_sep=2.5))
    L = cfg.L
    d = pos[:, None] - pos[None]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(20) * 1e9
    assert r.min() >= 2.5
    lat = W.ion_positions(cfg.replace(n_ions=27, placement="lattice", jitter=0.25))
    assert lat.shape == (27, 3) and np.all((lat >= 0) & (lat < L))
    assert W.ion_positions(cfg.replace(n_ions=0)).shape == (0, 3)


def test_batch_configs_cover_the_stated_ranges():
    cs = W.batch_configs()
    assert len(cs) == 16
    for c in cs:
        assert c.n in (32, 48, 64, 80, 96)
        assert 4 <= c.n_ions <= 64
        assert c.n_orb % 8 == 0 and 8 <= c.n_orb <= 256


def test_device_orbital_recipe_on_cpu():
    """The torch form of the orbital recipe (used for large benchmark batches)
    gives an orthonormal, smooth, reproducible set."""
    import torch
    cfg = W.C1.replace(n=16, n_orb=6, seed=77)
    a = W.initial_orbitals_device(cfg, "cpu")
    b = W.initial_orbitals_device(cfg, "cpu")
    assert a.shape == (6, 16 ** 3) and a.dtype == torch.complex128
    assert torch.equal(a, b)
    S = cfg.h ** 3 * (a.conj() @ a.T)
    assert (S - torch.eye(6, dtype=S.dtype)).abs().max() < 1e-12
    # the smoothing exp(-(|G| h)^2) leaves almost no weight at the highest |G|
    spec = torch.fft.fftn(a.reshape(6, 16, 16, 16), dim=(1, 2, 3)).abs() ** 2
    assert spec[:, 8, 8, 8].max() < 1e-12 * spec.sum(dim=(1, 2, 3)).max()
