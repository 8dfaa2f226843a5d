"""Batched systems on the GPU: the persistent multi-system stencil, the
6-step hipGraph replay and the autotuner must reproduce what each system
gives when it runs alone (same kernels per point, so the orbitals agree to
rounding), and the FP64 batch follows the oracle."""
import json
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu

# uneven: different grids (x rows 16..40), orbital counts, ion counts (one
# system without ions), a ragged last y-tile and z-slab with small blocks
UNEVEN = [
    W.C1.replace(name="b0", seed=1001),
    W.C1.replace(name="b1", n=24, n_orb=6, n_ions=5, placement="lattice", jitter=0.2, seed=1002),
    W.C1.replace(name="b2", n=20, n_orb=3, n_ions=0, seed=1003),
    W.C1.replace(name="b3", n=40, h=0.25, n_orb=2, n_ions=3, placement="lattice", jitter=0.2, seed=1004),
]


def _params(cfgs, prec, **over):
    from paper_0812_2801_amd import binding as B
    ps, keep, inps = [], [], []
    for c in cfgs:
        inp = W.make_inputs(c)
        p, k = B.params_from_config(c, inp["pos"], precision=prec, **over)
        ps.append(p)
        keep.append(k)
        inps.append(inp)
    return ps, keep, inps


def _batch(cfgs, prec, **over):
    import torch
    from paper_0812_2801_amd import binding as B
    ps, keep, inps = _params(cfgs, prec, **over)
    b = B.Batch(ps, keep)
    for s, c, inp in zip(b.systems, cfgs, inps):
        s.set_state(torch.from_numpy(inp["psi"].reshape(c.n_orb, -1)))
    return b


def _alone(cfg, prec, steps, **over):
    import torch
    from paper_0812_2801_amd import binding as B
    ps, keep, inps = _params([cfg], prec, **over)
    s = B.System(ps[0], keep)
    s.set_state(torch.from_numpy(inps[0]["psi"].reshape(cfg.n_orb, -1)))
    for _ in range(steps):
        s.step()
    out = (to_np(s.get_state()), s.ions()[0], s.forces())
    s.close()
    return out


def _state(s):
    return to_np(s.get_state()), s.ions()[0], s.forces()


TOL = {"f64": 1e-12, "f32": 2e-6, "f32_bf16x3": 2e-6}


def _maxabs(a):
    return float(np.abs(a).max()) if np.size(a) else 0.0


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_bf16x3"])
def test_batch_graph_matches_systems_alone(prec):
    steps = 14                       # 2 eager warm-up steps + 2 graph replays of 6
    note(f"batch vs alone {prec}, {steps} steps")
    b = _batch(UNEVEN, prec)
    b.propagate(steps, use_graph=True)
    for c, s in zip(UNEVEN, b.systems):
        psi, pos, frc = _state(s)
        psi0, pos0, frc0 = _alone(c, prec, steps)
        d = _maxabs(psi - psi0)
        note(f"  {c.name}: max|dpsi| {d:.2e} dpos {_maxabs(pos - pos0):.2e} "
             f"dF {_maxabs(frc - frc0):.2e}")
        assert d <= TOL[prec]
        assert _maxabs(pos - pos0) <= 1e-12
        assert _maxabs(frc - frc0) <= (1e-10 if prec == "f64" else 1e-5)
        assert s.report()["step"] == steps
    b.close()


def test_graph_replays_match_eager_batch():
    """Every replay of the captured graph against eager steps of a second,
    identical batch, with eager work and synchronisation between replays."""
    import torch
    note("graph replays vs eager batch f32")
    g = _batch(UNEVEN, "f32")
    e = _batch(UNEVEN, "f32")
    g.propagate(2, use_graph=True)            # warm-up: history ring filled
    e.propagate(2, use_graph=False)
    for r in range(3):
        g.propagate(6, use_graph=True)
        e.propagate(6, use_graph=False)
        torch.cuda.synchronize()
        for c, sg, se in zip(UNEVEN, g.systems, e.systems):
            a, b_ = to_np(sg.get_state()), to_np(se.get_state())
            d = np.abs(a - b_).max()
            note(f"  replay {r} {c.name}: max|dpsi| {d:.2e}")
            assert d == 0.0
            assert np.array_equal(sg.forces(), se.forces())
    # a remainder shorter than the graph period runs eagerly, and the next
    # call recaptures at the new phase
    g.propagate(9, use_graph=True)
    e.propagate(9, use_graph=False)
    for sg, se in zip(g.systems, e.systems):
        assert np.abs(to_np(sg.get_state()) - to_np(se.get_state())).max() == 0.0
    g.close()
    e.close()


def test_batch_f64_follows_the_oracle():
    from oracle import Model, dynamics
    note("batch f64 vs oracle")
    cfgs = UNEVEN[:3]
    b = _batch(cfgs, "f64")
    steps = 8
    b.propagate(steps, use_graph=True)
    for c, s in zip(cfgs, b.systems):
        inp = W.make_inputs(c)
        m = Model.from_config(c)
        st = dynamics.init_state(m, inp["psi"], inp["pos"])
        for _ in range(steps):
            st = dynamics.aetrs_step(m, st)
        psi = to_np(s.get_state()).reshape(st.psi.shape)
        d = np.abs(psi - st.psi).max()
        note(f"  {c.name}: max|dpsi| {d:.2e}")
        assert d < 1e-10
        assert _maxabs(s.forces() - st.force) < 1e-9
    b.close()


@pytest.mark.parametrize("block,wpc,zdiv", [(256, 1, 4), (512, 2, 2), (1024, 1, 1), (768, 0, 1), (512, 0, 2)])
def test_batch_launch_shapes(block, wpc, zdiv):
    """Small blocks force two halo runs per thread (8 n_x > block) and ragged
    y-tiles; zdiv > 1 gives short last z-slabs."""
    note(f"batch shape block={block} wpc={wpc} zdiv={zdiv}")
    b = _batch(UNEVEN, "f32")
    b.set_tuning(block, wpc, zdiv)
    assert b.tuning()["block"] == block
    b.propagate(3, use_graph=False)
    for c, s in zip(UNEVEN, b.systems):
        psi0, _, _ = _alone(c, "f32", 3)
        d = np.abs(to_np(s.get_state()) - psi0).max()
        note(f"  {c.name}: max|dpsi| {d:.2e}")
        assert d <= TOL["f32"]
    b.close()


def test_autotuner_cache(tmp_path):
    from paper_0812_2801_amd import binding as B
    note("autotuner + cache")
    path = str(tmp_path / "tune.json")
    b = _batch(UNEVEN, "f32")
    t1 = b.autotune(path)
    note(f"  tuned {t1}")
    assert t1["stage_ms"] > 0
    data = json.load(open(path))
    assert len(data) == 1
    (key, val), = data.items()
    assert key.startswith("f32/K4/") and val["block"] == t1["block"]
    b.propagate(2, use_graph=False)
    b.close()
    b2 = _batch(UNEVEN, "f32")
    t2 = b2.autotune(path)                    # from the cache: same choice
    assert (t2["block"], t2["wg_per_cu"], t2["zdiv"]) == (t1["block"], t1["wg_per_cu"], t1["zdiv"])
    with pytest.raises(B.ModehrError):
        b2.set_tuning(128, 1, 1)              # 8 * 40 > 2 * 128: does not fit
    with pytest.raises(B.ModehrError):
        b2.set_tuning(512, 1, 3)              # zdiv must be 1, 2 or 4
    b2.close()


def test_batch_needs_state():
    import torch
    from paper_0812_2801_amd import binding as B
    ps, keep, inps = _params(UNEVEN[:2], "f32")
    b = B.Batch(ps, keep)
    with pytest.raises(B.ModehrError) as e:
        b.propagate(1)
    assert e.value.status == B.ME_ESTATE
    b.close()
