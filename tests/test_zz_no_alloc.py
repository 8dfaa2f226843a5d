"""me_dipole_noalloc (the dipole with its partial sums in the library's fixed
device array, for callers that cannot allocate) against me_dipole, the entry
point it is a variant of: two calls in a row, the second on a smaller grid,
each on a system's own density.  Both run the same kernels in the same fixed
summation order, so the bits must agree; the oracle's objective checks the
value itself."""
import numpy as np
import pytest

import workloads as W
from gpu_common import note

pytestmark = pytest.mark.gpu


def _system(cfg):
    import torch
    from paper_0812_2801_amd import binding as B
    inp = W.make_inputs(cfg)
    p, keep = B.params_from_config(cfg, inp["pos"], precision="f64")
    s = B.System(p, keep)
    s.set_state(torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1)))
    return s


def test_dipole_noalloc_matches_me_dipole_twice():
    import torch
    from oracle import Model, adjoint
    from paper_0812_2801_amd import binding as B
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
    for cfg in (W.C1.replace(n=24, n_orb=3, seed=1301), W.C1.replace(n=16, n_orb=2, seed=1302)):
        note(f"dipole_noalloc {cfg.n}^3")
        s = _system(cfg)
        s.step()
        rho = s.density()
        want = s.dipole()
        B.dipole_noalloc(rho, (cfg.n,) * 3, cfg.h, out)
        torch.cuda.synchronize()
        got = float(out.item())
        note(f"  noalloc {got!r}  me_dipole {want!r}")
        assert got == want
        m = Model(n=cfg.n, h=cfg.h, zval=np.zeros(0), mass=np.zeros(0))
        ref = adjoint.objective(m, rho.cpu().numpy().reshape((cfg.n,) * 3))
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref))
        s.close()


def test_dipole_noalloc_refuses_oversize_grids():
    import torch
    from paper_0812_2801_amd import binding as B
    rho = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(B.ModehrError, match="too large"):
        B.dipole_noalloc(rho, (1024, 1024, 1024), 0.3, out)
