"""The x-tiled stencil (tiles of TX points of TY rows with an x-halo in LDS,
the default for FP32 rows wider than 96 points) against the FP64 oracle.
Small grids force it with MODEHR_TX / MODEHR_TY (read when a system is
created): 16 x 8 tiles on 20^3 and 40^3 leave ragged tiles along x and y;
the 48 x 16 and 32 x 24 shapes run on 96^3 with a few orbitals, and the
default 64 x 12 on 128^3 (ragged along y).  H psi (all stencil modes but the
adjoint's scaled one, which the emulation covers) and one AETRS step."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import make_pair, note, to_np

pytestmark = pytest.mark.gpu

CASES = [
    ("n20_16x8", W.C1.replace(n=20, h=0.3, n_orb=3, n_ions=3, placement="lattice", jitter=0.2, seed=2001), 16, 8),
    ("n40_16x8", W.C1.replace(n=40, h=0.25, n_orb=2, n_ions=4, placement="lattice", jitter=0.2, seed=4001), 16, 8),
    ("n96_48x16", W.C1.replace(n=96, h=0.25, n_orb=2, n_ions=8, placement="lattice", jitter=0.3, seed=9601), 48, 16),
    ("n96_32x24", W.C1.replace(n=96, h=0.25, n_orb=2, n_ions=8, placement="lattice", jitter=0.3, seed=9602), 32, 24),
    ("n128_64x12", W.C1.replace(n=128, h=0.25, n_orb=2, n_ions=8, placement="lattice", jitter=0.3, seed=12801),
     None, None),
]


@pytest.fixture
def tiles(request):
    tx, ty = request.param
    old = {k: os.environ.get(k) for k in ("MODEHR_TX", "MODEHR_TY")}
    if tx is not None:
        os.environ["MODEHR_TX"] = str(tx)
        os.environ["MODEHR_TY"] = str(ty)
    yield tx, ty
    for k, v in old.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


@pytest.mark.parametrize("name,cfg,tiles", [(n, c, (tx, ty)) for n, c, tx, ty in CASES],
                         indirect=["tiles"], ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_xtiled_stencil_matches_oracle(name, cfg, tiles, prec):
    from oracle import dynamics
    if prec == "f64" and tiles[0] is None:
        pytest.skip("FP64 keeps whole rows unless a tile is forced")
    note(f"x-tiles {name} {prec}")
    sysm, m, st, inp, cfg = make_pair(cfg, precision=prec)
    rng = np.random.default_rng(11)
    shape = (2,) + m.grid.shape
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * 0.05
    got = to_np(sysm.apply_H(x.reshape(2, -1))).reshape(shape)
    want = m.apply_H(x, m.vloc(st.pos) + st.hist[-1], m.spheres(st.pos))
    err = float(np.abs(got - want).max() / np.abs(want).max())
    rep0 = sysm.report()
    e0 = dynamics.total_energy(m, st)["total"]
    sysm.step()
    st1 = dynamics.aetrs_step(m, st)
    dpsi = float(np.abs(to_np(sysm.get_state()).reshape(st1.psi.shape) - st1.psi).max())
    note(f"  H psi rel err {err:.2e}, one step max|dpsi| {dpsi:.2e}, dE0 {rep0['e_total'] - e0:+.2e}")
    tol_h, tol_psi = (1e-11, 1e-10) if prec == "f64" else (3e-6, 1e-4)
    assert err < tol_h and dpsi < tol_psi
    assert abs(rep0["e_total"] - e0) < (1e-9 if prec == "f64" else 1e-5) * max(1.0, abs(e0))
    sysm.close()
