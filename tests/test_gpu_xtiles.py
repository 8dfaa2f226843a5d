"""The stencil's other tile shapes against the FP64 oracle: x-tiles (TX
points of TY rows with an x-halo in LDS; the default for FP32 rows wider than
256 points) and whole rows with two rows per thread (the default for FP32
rows of 97-256 points).  Environment variables read when a system is created
force them on small grids: 16 x 8 x-tiles on 20^3 and 40^3 leave ragged
tiles along x and y; the 48 x 16 and 32 x 24 shapes run on 96^3 and 64 x 12
on 128^3 (ragged along y) with a few orbitals; two rows per thread run by
default on 128^3 and forced on 32^3 (8 and 16 rows per tile, FP32 and
FP64).  H psi (all stencil modes but the adjoint's scaled one, which the
emulation covers), the energy report and one AETRS step."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_common import make_pair, note, to_np

pytestmark = pytest.mark.gpu

CASES = [
    ("n20_16x8", W.C1.replace(n=20, h=0.3, n_orb=3, n_ions=3, placement="lattice", jitter=0.2, seed=2001),
     {"MODEHR_TX": "16", "MODEHR_TY": "8"}),
    ("n40_16x8", W.C1.replace(n=40, h=0.25, n_orb=2, n_ions=4, placement="lattice", jitter=0.2, seed=4001),
     {"MODEHR_TX": "16", "MODEHR_TY": "8"}),
    ("n96_48x16", W.C1.replace(n=96, h=0.25, n_orb=2, n_ions=8, placement="lattice", jitter=0.3, seed=9601),
     {"MODEHR_TX": "48", "MODEHR_TY": "16"}),
    ("n96_32x24", W.C1.replace(n=96, h=0.25, n_orb=2, n_ions=8, placement="lattice", jitter=0.3, seed=9602),
     {"MODEHR_TX": "32", "MODEHR_TY": "24"}),
    ("n128_64x12", W.C1.replace(n=128, h=0.25, n_orb=2, n_ions=8, placement="lattice", jitter=0.3, seed=12801),
     {"MODEHR_TX": "64", "MODEHR_TY": "12"}),
    ("n128_default", W.C1.replace(n=128, h=0.25, n_orb=2, n_ions=8, placement="lattice", jitter=0.3, seed=12802),
     {}),
    ("n32_py8", W.C1.replace(n=32, h=0.25, n_orb=3, n_ions=4, placement="lattice", jitter=0.3, seed=3202),
     {"MODEHR_PY": "2", "MODEHR_PY_TY": "8"}),
    ("n32_py16", W.C1.replace(n=32, h=0.25, n_orb=3, n_ions=4, placement="lattice", jitter=0.3, seed=3203),
     {"MODEHR_PY": "2", "MODEHR_PY_TY": "16"}),
]
ENV_KEYS = ("MODEHR_TX", "MODEHR_TY", "MODEHR_PY", "MODEHR_PY_TY")


@pytest.fixture
def tiles(request):
    old = {k: os.environ.get(k) for k in ENV_KEYS}
    for k in ENV_KEYS:
        os.environ.pop(k, None)
    os.environ.update(request.param)
    yield request.param
    for k, v in old.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


@pytest.mark.parametrize("name,cfg,tiles", CASES, indirect=["tiles"], ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_xtiled_stencil_matches_oracle(name, cfg, tiles, prec):
    from oracle import dynamics
    if prec == "f64" and not tiles:
        pytest.skip("FP64 keeps whole rows of one per thread unless a shape is forced")
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
