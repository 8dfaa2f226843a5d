"""GPU adjoint: the library's reverse sweep (through the C ABI and the
torch.autograd.Function) against the FP64 oracle's gradient and against
central finite differences of the GPU forward trajectory."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note

pytestmark = pytest.mark.gpu


def _system(cfg, prec):
    from paper_0812_2801_amd import binding as B
    inp = W.make_inputs(cfg)
    p, keep = B.params_from_config(cfg, inp["pos"], precision=prec, enable_adjoint=True)
    return B.System(p, keep), inp


def _run(cfg, prec, ctrl, dv, every):
    import torch
    from paper_0812_2801_amd.autograd import DipoleObjective
    s, inp = _system(cfg, prec)
    psi0 = torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1))
    c = torch.tensor(ctrl, dtype=torch.float64, requires_grad=True)
    d = torch.tensor(dv, dtype=torch.float64, requires_grad=True)
    J = DipoleObjective.apply(c, d, s, psi0, every)
    J.backward()
    out = (float(J), c.grad.numpy().copy(), d.grad.numpy().copy())
    s.close()
    return out


@pytest.mark.parametrize("every", [2, 10])
def test_adjoint_matches_oracle_gradient_fp64(every):
    from oracle import Model, adjoint
    note(f"adjoint vs oracle, checkpoint every {every}")
    cfg = W.C1.replace(freeze_ions=True, coarse_n=4, control_sigma=0.01, steps=5, seed=901)
    inp = W.make_inputs(cfg)
    dv = 0.01 * np.random.default_rng(0).standard_normal((4, 4, 4))
    m = Model.from_config(cfg)
    J0, ge0, gv0 = adjoint.gradient(m, inp["psi"], inp["pos"], inp["ctrl"], dv)
    J, ge, gv = _run(cfg, "f64", inp["ctrl"], dv, every)
    note(f"  J {J:.12e} oracle {J0:.12e}; |dge| {np.abs(ge - ge0).max():.2e} |dgv| {np.abs(gv - gv0).max():.2e}")
    assert abs(J - J0) < 1e-11 * max(1, abs(J0))
    assert np.abs(ge - ge0).max() < 1e-9 * max(1e-3, np.abs(ge0).max())
    assert np.abs(gv - gv0).max() < 1e-9 * max(1e-3, np.abs(gv0).max())


def test_adjoint_fp32_reduced_c5_vs_oracle():
    from oracle import Model, adjoint
    note("adjoint fp32 reduced c5 vs oracle")
    cfg = W.C5.replace(n=32, n_ions=6, n_orb=8, steps=6, coarse_n=8, seed=905)
    inp = W.make_inputs(cfg)
    dv = 0.01 * np.random.default_rng(1).standard_normal((8, 8, 8))
    m = Model.from_config(cfg)
    J0, ge0, gv0 = adjoint.gradient(m, inp["psi"], inp["pos"], inp["ctrl"], dv)
    J, ge, gv = _run(cfg, "f32", inp["ctrl"], dv, 3)
    rel_e = np.abs(ge - ge0).max() / np.abs(ge0).max()
    rel_v = np.abs(gv - gv0).max() / np.abs(gv0).max()
    note(f"  rel err eps-grad {rel_e:.2e}, dV-grad {rel_v:.2e}")
    assert abs(J - J0) < 1e-5 * max(1, abs(J0))
    assert rel_e < 1e-3 and rel_v < 1e-3


def test_adjoint_c5_shape_vs_finite_differences():
    """Full c5 shape (64^3, 32 ions, 64 orbitals, 50 steps, checkpoints every 10):
    the FP32 adjoint gradient against central differences (h = 1e-4) of the FP64
    GPU forward along a random direction."""
    import torch
    note("adjoint c5 shape vs FD")
    cfg = W.C5
    inp = W.make_inputs(cfg)
    dv = np.zeros((16, 16, 16))
    J, ge, gv = _run(cfg, "f32", inp["ctrl"], dv, 10)
    rng = np.random.default_rng(7)
    de = rng.standard_normal(cfg.steps)
    dd = 0.1 * rng.standard_normal((16, 16, 16))
    from paper_0812_2801_amd.autograd import DipoleObjective

    def fwd(c, d):
        s, _ = _system(cfg, "f64")
        psi0 = torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1))
        with torch.no_grad():
            j = float(DipoleObjective.apply(torch.tensor(c), torch.tensor(d), s, psi0, 1000))
        s.close()
        return j

    h = 1e-4
    fd = (fwd(inp["ctrl"] + h * de, dv + h * dd) - fwd(inp["ctrl"] - h * de, dv - h * dd)) / (2 * h)
    an = float(np.dot(ge, de) + np.sum(gv * dd))
    note(f"  FD {fd:.8e} adjoint {an:.8e}")
    assert abs(fd - an) < 2e-3 * max(1e-6, abs(fd))
