"""Largest stable time step on the GPU against the oracle's stability
limits (Fig. spacing): the Taylor-4 AETRS step at 2 mu theta_4 / max|E| and
CP's Verlet step at 2 sqrt(mu_cp / (E_max - E_min)), with the extreme
eigenvalues of H from the oracle's power iteration at the same state."""
import numpy as np
import pytest

from gpu_common import note

pytestmark = pytest.mark.gpu


def test_dt_max_matches_the_predicted_limits():
    import workloads as W
    from oracle import Model, stability
    from paper_0812_2801_amd import scan
    cfg = scan.spacing_config(40)
    psi0 = scan.noisy_orbitals(cfg)
    m = Model.from_config(cfg)
    pos = W.ion_positions(cfg)
    psi = psi0.cpu().numpy().reshape((cfg.n_orb,) + m.grid.shape)
    veff = m.vloc(pos) + m.v_hxc(m.density(psi))
    e_min, e_max = stability.h_extreme_eigenvalues(m, veff, m.spheres(pos), iters=400)
    mu, mu_cp = 4.0, 200.0
    want_t4 = stability.ehrenfest_dt_max(mu, 4, max(abs(e_min), abs(e_max)))
    want_cp = stability.cp_dt_max(mu_cp, e_max, e_min)
    got_t4 = scan.dt_max(cfg, psi0, "ehrenfest", mu, mu_cp, 0.05, 4, rel_tol=0.02)
    got_cp = scan.dt_max(cfg, psi0, "cp", mu, mu_cp, 0.5, 4, rel_tol=0.02)
    note(f"E in [{e_min:.2f}, {e_max:.2f}]; Taylor-4 dt_max {got_t4:.4f} (limit {want_t4:.4f}); "
         f"CP dt_max {got_cp:.4f} (limit {want_cp:.4f})")
    assert 0.85 * want_t4 < got_t4 < 1.15 * want_t4
    assert 0.85 * want_cp < got_cp < 1.1 * want_cp
