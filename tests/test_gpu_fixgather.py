"""The fused projector pass (a Horner stage's nonlocal fix-up and the next
stage's gather of c_JA in one pass over the projector points) against the
two separate passes (MODEHR_FIXGATHER=0), for every contraction: plain FP64,
plain FP32 and split-bf16 MFMA.  The fixed values come from the same
arithmetic in either case and the contraction reads the same values, so the
orbitals, forces and energies must agree bit for bit.  The workload packs 10
ions closely enough that 85 grid points lie in two or three projector
spheres (the points the fused pass leaves to its second kernel), and 19
orbitals leave a ragged group of the 16-orbital MFMA tile."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import note, to_np

pytestmark = pytest.mark.gpu

CFG = W.C1.replace(n=24, h=0.3, n_orb=19, n_ions=10, placement="uniform", min_sep=0.9, seed=73)


def _with_env(fused, fn):
    old = os.environ.get("MODEHR_FIXGATHER")
    os.environ["MODEHR_FIXGATHER"] = "1" if fused else "0"
    try:
        return fn()
    finally:
        if old is None:
            os.environ.pop("MODEHR_FIXGATHER", None)
        else:
            os.environ["MODEHR_FIXGATHER"] = old


def _run(prec, fused, steps):
    import torch
    from paper_0812_2801_amd import binding as B

    def go():
        inp = W.make_inputs(CFG)
        p, keep = B.params_from_config(CFG, inp["pos"], precision=prec)
        s = B.System(p, keep)
        s.set_state(torch.from_numpy(inp["psi"].reshape(CFG.n_orb, -1)))
        reps = [s.step(report=True) for _ in range(steps)]
        out = (to_np(s.get_state()), s.forces().copy(), [r["e_total"] for r in reps])
        s.close()
        return out, inp
    return _with_env(fused, go)


def test_workload_has_shared_points():
    from collections import Counter
    from oracle import Model
    inp = W.make_inputs(CFG)
    c = Counter()
    for s in Model.from_config(CFG).spheres(inp["pos"]):
        idx = s[0] if isinstance(s, tuple) else s.idx
        c.update(np.asarray(idx).ravel().tolist())
    assert sum(1 for v in c.values() if v > 1) > 50 and max(c.values()) == 3


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_bf16x3"])
def test_fused_pass_is_bit_identical(prec):
    from oracle import Model, dynamics
    (psi_a, f_a, e_a), inp = _run(prec, True, 3)
    (psi_b, f_b, e_b), _ = _run(prec, False, 3)
    note(f"{prec}: fused vs separate passes: max|dpsi| {np.abs(psi_a - psi_b).max():.1e}, "
         f"max|dF| {np.abs(f_a - f_b).max():.1e}")
    assert np.array_equal(psi_a, psi_b)
    assert np.array_equal(f_a, f_b)
    assert e_a == e_b
    m = Model.from_config(CFG)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    for _ in range(3):
        st = dynamics.aetrs_step(m, st)
    d = np.abs(psi_a - st.psi.reshape(CFG.n_orb, -1)).max()
    df = np.abs(f_a - st.force).max()
    note(f"  vs oracle after 3 steps: max|dpsi| {d:.1e}, max|dF| {df:.1e}")
    tol = {"f64": (1e-10, 1e-9), "f32": (1e-4, 1e-4), "f32_bf16x3": (1e-4, 1e-4)}[prec]
    assert d <= tol[0] and df <= tol[1]


@pytest.mark.parametrize("prec", ["f32", "f32_bf16x3"])
def test_fused_pass_in_a_batch_is_bit_identical(prec):
    import torch
    from paper_0812_2801_amd import binding as B
    cfgs = [CFG, CFG.replace(n=20, n_orb=7, n_ions=4, placement="pair", seed=2412)]

    def go():
        ps, keep, inps = [], [], []
        for c in cfgs:
            inp = W.make_inputs(c)
            p, k = B.params_from_config(c, inp["pos"], precision=prec)
            ps.append(p)
            keep.append(k)
            inps.append(inp)
        b = B.Batch(ps, keep)
        for s, c, inp in zip(b.systems, cfgs, inps):
            s.set_state(torch.from_numpy(inp["psi"].reshape(c.n_orb, -1)))
        b.propagate(2, use_graph=False)
        out = [(to_np(s.get_state()), s.forces().copy()) for s in b.systems]
        b.close()
        return out
    a = _with_env(True, go)
    b = _with_env(False, go)
    for (pa, fa), (pb, fb) in zip(a, b):
        note(f"{prec} batch: max|dpsi| {np.abs(pa - pb).max():.1e}, max|dF| {np.abs(fa - fb).max():.1e}")
        assert np.array_equal(pa, pb)
        assert np.array_equal(fa, fb)
