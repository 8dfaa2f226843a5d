"""The two-band toy model (eq. L_toy) on the GPU through the C ABI against
the oracle's RK4: samples, d_R and d_F of uneven (mass, step) sets for both
schemes; the distance kernel; invalid entries; and, at the full sweep of
Fig. 1 (c, d), sampled trajectories against the oracle plus the trends the
model fixes (d_R -> 0 and smaller Delta t_max as the mass goes to zero)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note

pytestmark = pytest.mark.gpu


def _oracle_params():
    from oracle import toy as T
    return T, T.ToyParams(**W.TOY_N2)


@pytest.mark.parametrize("scheme,mus", [("ehrenfest", [2.0, 0.5, 0.1, 0.03]), ("cp", [600.0, 120.0, 25.0, 5.0])])
def test_toy_runs_match_oracle(scheme, mus):
    import torch
    from paper_0812_2801_amd import binding as B, toy
    T, P = _oracle_params()
    p = toy.params()
    n_s, t_total = 80, P.period_R
    mu = np.array(mus * 2)
    sub = np.array([4, 6, 12, 40, 8, 12, 24, 80], np.int32)
    win = np.array([3, 1, 4, 2, 7, 5, 1, 2], np.int32)
    note(f"toy {scheme}: {mu.size} trajectories")
    out = B.toy_run(p, scheme, mu, sub, win, n_s, t_total)
    S = out["samples"].cpu().numpy()
    d_R, d_F = out["d_R"].cpu().numpy(), out["d_F"].cpu().numpy()
    for i in range(mu.size):
        r = T.run(P, scheme, [mu[i]], int(sub[i]), n_s, t_total, window=[int(win[i])])
        ds = np.abs(S[:, :, i] - r["samples"][0]).max()
        note(f"  mu {mu[i]} sub {sub[i]}: max|d samples| {ds:.2e}; d_R {d_R[i]:.6g} ({r['d_R'][0]:.6g}), "
             f"d_F {d_F[i]:.6g} ({r['d_F'][0]:.6g})")
        assert ds < 1e-9
        assert abs(d_R[i] - r["d_R"][0]) < 1e-8 * max(1.0, r["d_R"][0])
        assert abs(d_F[i] - r["d_F"][0]) < 1e-8 * max(1.0, r["d_F"][0])
    ref = torch.tensor([4, 5, 6, 7, 4, 5, 6, 7], dtype=torch.int32)
    dist = B.toy_distance(out["samples"], ref).cpu().numpy()
    Sm = np.moveaxis(S, 2, 0)
    want = np.array([T.trajectory_distance(Sm[i], Sm[ref[i]]) for i in range(mu.size)])
    assert np.abs(dist - want).max() < 1e-10 * max(1.0, np.abs(want).max())
    assert np.all(dist[4:] == 0.0)


def test_toy_invalid_entries_and_arguments():
    from paper_0812_2801_amd import binding as B, toy
    p = toy.params()
    out = B.toy_run(p, "ehrenfest", [1.0, -1.0, 1.0, 1.0], [2, 2, 0, 9], [1, 1, 1, 1], 10, 100.0, max_substeps=8)
    d_R = out["d_R"].cpu().numpy()
    assert np.isfinite(d_R[0]) and np.isnan(d_R[1:]).all()
    assert np.isnan(out["samples"][:, :, 1:].cpu().numpy()).all()
    empty = B.toy_run(p, "cp", [], [], [], 10, 100.0, max_substeps=1)      # no trajectories: nothing to do
    assert empty["d_R"].numel() == 0 and tuple(empty["samples"].shape) == (11, 8, 0)
    with pytest.raises(B.ModehrError):
        B.toy_run(p, "ehrenfest", [1.0], [1], [1], 1 << 12, 100.0, max_substeps=1 << 13)
    with pytest.raises(B.ModehrError):
        B.toy_run(toy.params(M_R=-1.0), "cp", [1.0], [1], [1], 10, 100.0)


@pytest.mark.parametrize("scheme", ["ehrenfest", "cp"])
def test_toy_full_sweep(scheme):
    from paper_0812_2801_amd import toy
    T, P = _oracle_params()
    S = W.TOY_SWEEP
    mus = np.geomspace(*S["mu_" + scheme], S["n_mu"])
    ladder = toy.substep_ladder(S["ladder_steps"], S["finest"], S["ratio"])
    r = toy.sweep(scheme, mus, ladder, S["n_samples"], S["periods"])
    note(f"toy sweep {scheme}: {r['n_traj']} trajectories, {r['rk4_steps']:.3e} RK4 steps")
    # one (mass, step) entry launched alone reproduces the sweep's distance table
    m, s = S["n_mu"] // 2, 16
    got = toy.sweep(scheme, mus[m:m + 1], [s, ladder[-1]], S["n_samples"], S["periods"])
    k = ladder.index(s)
    assert abs(got["dist"][0, 0] - r["dist"][k, m]) <= 1e-12 * max(1.0, r["dist"][k, m])
    # sampled trajectories of the sweep's shape against the oracle
    from paper_0812_2801_amd import binding as B
    pick = mus[S["n_mu"] // 4::S["n_mu"] // 4]   # masses whose RK4 at this step is stable (omega dt < 1)
    t_s = r["t_total"] / S["n_samples"]
    win = [toy.window(toy.params(), scheme, float(x), t_s) for x in pick]
    o = T.run(P, scheme, pick, s, S["n_samples"], r["t_total"], window=win)
    g = B.toy_run(toy.params(), scheme, pick, [s] * len(pick), win, S["n_samples"], r["t_total"])
    ds = np.abs(np.moveaxis(g["samples"].cpu().numpy(), 2, 0) - o["samples"]).max()
    note(f"  {len(pick)} sampled trajectories at {s} substeps: max|d samples| {ds:.2e}")
    assert ds < 1e-9
    assert np.allclose(g["d_R"].cpu().numpy(), o["d_R"], rtol=1e-8, atol=1e-10)
    assert np.allclose(g["d_F"].cpu().numpy(), o["d_F"], rtol=1e-8, atol=1e-10)
    # the trends of Fig. 1: d_R vanishes with the mass, and so does Delta t_max
    d_R, dt_max = r["d_R"], r["dt_max"]
    note(f"  d_R {d_R[0]:.3g} .. {d_R[-1]:.3g}; dt_max {np.nanmin(dt_max):.3g} .. {np.nanmax(dt_max):.3g}")
    assert d_R[0] < 0.05 * d_R[-1]
    assert np.all(np.isfinite(dt_max[: S["n_mu"] // 2]))
    assert dt_max[0] < dt_max[S["n_mu"] // 2]


@pytest.mark.parametrize("scheme,mu", [("ehrenfest", 0.3), ("cp", 5.0)])
def test_dt_max_matches_oracle(scheme, mu):
    # the Delta t_max selection on a short run that the oracle can afford
    from paper_0812_2801_amd import toy
    T, P = _oracle_params()
    ladder = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 128]
    n_s, periods = 60, 1.0
    r = toy.sweep(scheme, [mu], ladder, n_s, periods)
    want = T.dt_max(P, scheme, mu, n_s, periods * P.period_R, ladder[:-1], ladder[-1])
    note(f"toy {scheme} mu {mu}: dt_max {r['dt_max'][0]} (oracle {want}); distances {r['dist'][:, 0].round(4)}")
    assert want is not None and abs(r["dt_max"][0] - want) <= 1e-12 * want
