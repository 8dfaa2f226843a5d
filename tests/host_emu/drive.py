"""Runs the library built for CPU emulation (tests/host_emu) through its C ABI
and compares with the FP64 oracle: drive.py LIB SCENARIO [PRECISION] [TMPDIR].
"Device" buffers are numpy arrays.  Prints OK on success; any misuse the
emulator or AddressSanitizer detects aborts the process."""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import workloads as W                                      # noqa: E402
from oracle import Model, adjoint, cp, dynamics, finite, toy  # noqa: E402
from paper_0812_2801_amd import binding as B               # noqa: E402

lib = B.load(sys.argv[1])
lib.mock_new_stream.restype = ctypes.c_void_p
lib.mock_live_handles.restype = ctypes.c_long
lib.mock_memsets_in_capture.restype = ctypes.c_long
scenario = sys.argv[2]
prec = sys.argv[3] if len(sys.argv) > 3 else "f64"
tmp = sys.argv[4] if len(sys.argv) > 4 else "."
stream = lib.mock_new_stream()
held = []
base_handles = lib.mock_live_handles()
CDT = np.complex128 if prec == "f64" else np.complex64
# one-step-scale tolerances: FP64 agrees with the oracle to rounding; FP32
# (and the split-bf16 contraction) to single precision over a few steps
TOL_PSI = {"f64": 1e-12, "f32": 2e-6, "f32_bf16x3": 2e-6}[prec]
TOL_F = {"f64": 1e-10, "f32": 1e-4, "f32_bf16x3": 1e-4}[prec]


def buf(nbytes):
    a = np.zeros(nbytes + 256, np.uint8)
    held.append(a)
    return (a.ctypes.data + 255) // 256 * 256


def ok(st, h=None, batch=False):
    if st != B.ME_OK:
        err = (lib.me_batch_last_error if batch else lib.me_last_error)(h)
        raise SystemExit(f"status {st}: {err.decode()}")


def orbitals(c, inp):
    return np.ascontiguousarray(inp["psi"].reshape(c.n_orb, -1).astype(CDT))


def state(h, c):
    out = np.zeros((c.n_orb, c.n_points), CDT)
    ok(lib.me_get_state(h, out.ctypes.data, c.n_points), h)
    f = np.zeros(3 * c.n_ions)
    ok(lib.me_forces(h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), h)
    return out, f


def oracle_run(c, inp, steps, ctrl=None):
    m = Model.from_config(c)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    for n in range(steps):
        st = dynamics.aetrs_step(m, st, 0.0 if ctrl is None else float(ctrl[n]))
    return st


def compare(name, c, psi, f, st):
    dpsi = np.abs(psi.reshape(st.psi.shape) - st.psi).max()
    df = np.abs(f - st.force.ravel()).max() if c.n_ions else 0.0
    print(f"{name}: max|dpsi| {dpsi:.2e} max|dF| {df:.2e}", flush=True)
    assert dpsi <= TOL_PSI, (name, dpsi)
    assert df <= TOL_F, (name, df)


def new_system(c, inp, **over):
    p, keep = B.params_from_config(c, inp["pos"], precision=prec, **over)
    held.append(keep)
    size = ctypes.c_size_t(0)
    ok(lib.me_workspace_size(ctypes.byref(p), ctypes.byref(size)))
    h = ctypes.c_void_p()
    ok(lib.me_init_system(ctypes.byref(p), buf(size.value), size.value, stream, ctypes.byref(h)))
    return h


UNEVEN = [
    W.C1.replace(name="b0", seed=1001),
    W.C1.replace(name="b1", n=24, n_orb=6, n_ions=5, placement="lattice", jitter=0.2, seed=1002),
    W.C1.replace(name="b2", n=20, n_orb=3, n_ions=0, seed=1003),
    W.C1.replace(name="b3", n=40, h=0.25, n_orb=2, n_ions=3, placement="lattice", jitter=0.2, seed=1004),
]

if scenario in ("system", "system_xt", "system_py"):
    # system_py runs with MODEHR_PY=2 MODEHR_PY_TY=8: the 16^3 case in tiles of
    # 8 whole rows, two rows per thread
    # system_xt runs with MODEHR_TX=16 MODEHR_TY=8: the 20^3 case in x-tiles,
    # ragged along x (16 + 4) and y (8 + 8 + 4)
    # 20^3 with 5 orbitals and 5 ions: a tile height of 4 rows, an odd
    # orbital count for the 8-orbital contraction blocks
    for c in (W.C1, W.C1.replace(name="odd", n=20, n_orb=5, n_ions=5, placement="lattice", jitter=0.2, seed=77)):
        inp = W.make_inputs(c)
        h = new_system(c, inp)
        psi = orbitals(c, inp)
        ok(lib.me_set_state(h, psi.ctypes.data, c.n_points), h)
        rep = B.StepReport()
        ok(lib.me_timing_enable(h, 1), h)
        for _ in range(3):
            ok(lib.me_propagate_step(h, None, ctypes.byref(rep)), h)
        n_, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        ok(lib.me_timing_read(h, ctypes.byref(n_), ctypes.byref(ms), ctypes.byref(by)), h)
        assert n_.value == 3 * 2 * 4, n_.value
        st = oracle_run(c, inp, 3)
        psi_out, f = state(h, c)
        compare(f"{c.name} 3 steps", c, psi_out, f, st)
        e = dynamics.total_energy(Model.from_config(c), st)
        de = abs(rep.e_total - e["total"])
        print(f"{c.name}: |dE_total| {de:.2e}", flush=True)
        assert de < (1e-9 if prec == "f64" else 1e-3) * max(1.0, abs(e["total"]))
        # H applied to the state, against the oracle's H at the same state
        hpsi = np.zeros_like(psi_out)
        ok(lib.me_apply_H(h, psi_out.ctypes.data, hpsi.ctypes.data, c.n_orb, c.n_points), h)
        m = Model.from_config(c)
        veff = m.vloc(st.pos) + m.v_hxc(st.rho)
        ref = m.apply_H(psi_out.reshape(st.psi.shape).astype(np.complex128), veff, m.spheres(st.pos))
        dh = np.abs(hpsi.reshape(ref.shape) - ref).max()
        print(f"{c.name}: max|d(H psi)| {dh:.2e}", flush=True)
        assert dh <= (1e-10 if prec == "f64" else 1e-3) * max(1.0, np.abs(ref).max())
        ok(lib.me_destroy(h))
        # the wave-function-gradient form of the nonlocal force, at the initial state
        h = new_system(c, inp, nl_force_form=1)
        ok(lib.me_set_state(h, psi.ctypes.data, c.n_points), h)
        _, f = state(h, c)
        m = Model.from_config(c)
        st0 = dynamics.init_state(m, inp["psi"], inp["pos"])
        want = m.forces(st0.pos, st0.psi, st0.rho, nl_form="gradient")["total"]
        dfg = np.abs(f - want.ravel()).max()
        print(f"{c.name}: gradient-form forces max|dF| {dfg:.2e}", flush=True)
        assert dfg <= TOL_F
        ok(lib.me_destroy(h))
elif scenario in ("batch", "batch_xt"):
    # batch_xt runs with MODEHR_BATCH_TX=16: every system wider than 16 points
    # in 16-point x-tiles (ragged for 20, 24 and 40)
    arr = (B.Params * len(UNEVEN))()
    keep, inps = [], []
    for i, c in enumerate(UNEVEN):
        inp = W.make_inputs(c)
        p, k = B.params_from_config(c, inp["pos"], precision=prec)
        arr[i] = p
        keep.append(k)
        inps.append(inp)
    size = ctypes.c_size_t(0)
    ok(lib.me_batch_workspace_size(arr, len(UNEVEN), ctypes.byref(size)))
    h = ctypes.c_void_p()
    ok(lib.me_init_batch(arr, len(UNEVEN), buf(size.value), size.value, stream, ctypes.byref(h)))
    sys_h = []
    for i, c in enumerate(UNEVEN):
        s = ctypes.c_void_p()
        ok(lib.me_batch_system(h, i, ctypes.byref(s)), h, True)
        psi = orbitals(c, inps[i])
        ok(lib.me_set_state(s, psi.ctypes.data, c.n_points), s)
        sys_h.append(s)
    # warm-up, capture, one replay; then shapes with two halo runs per
    # thread (block 256 < 8 n_x) and ragged z-slabs, eagerly
    ok(lib.me_propagate_batch(h, 8, 1), h, True)
    t = B.BatchTuning(block=256, wg_per_cu=1, zdiv=4, stage_ms=0.0)
    ok(lib.me_batch_set_tuning(h, ctypes.byref(t)), h, True)
    ok(lib.me_propagate_batch(h, 2, 0), h, True)
    t = B.BatchTuning(block=1024, wg_per_cu=1, zdiv=2, stage_ms=0.0)
    ok(lib.me_batch_set_tuning(h, ctypes.byref(t)), h, True)
    ok(lib.me_propagate_batch(h, 7, 1), h, True)        # a new phase: recapture, one replay, one eager
    total = 17
    for i, c in enumerate(UNEVEN):
        psi_out, f = state(sys_h[i], c)
        compare(f"batch {c.name} {total} steps", c, psi_out, f, oracle_run(c, inps[i], total))
    if prec == "f32":
        tt = B.BatchTuning()
        ok(lib.me_batch_autotune(h, os.path.join(tmp, "tune.json").encode(), ctypes.byref(tt)), h, True)
    ok(lib.me_batch_destroy(h))
elif scenario in ("adjoint", "adjoint_xt"):
    # adjoint_xt: a 20^3 grid, so that the forced 16 x 8 x-tiles are ragged
    c = W.C1.replace(freeze_ions=True, coarse_n=4, control_sigma=0.01, steps=4, seed=901,
                     n=20 if scenario == "adjoint_xt" else 16)
    inp = W.make_inputs(c)
    dv = 0.01 * np.random.default_rng(0).standard_normal((4, 4, 4))
    J0, ge0, gv0 = adjoint.gradient(Model.from_config(c), inp["psi"], inp["pos"], inp["ctrl"], dv)
    h = new_system(c, inp, enable_adjoint=True)
    dvb = np.ascontiguousarray(dv)
    ok(lib.me_set_static_potential_coarse(h, dvb.ctypes.data, 4), h)
    psi = orbitals(c, inp)
    ok(lib.me_set_state(h, psi.ctypes.data, c.n_points), h)
    cp = ctypes.c_size_t(0)
    ok(lib.me_checkpoint_size(h, ctypes.byref(cp)), h)
    ck = [buf(cp.value) for _ in range(c.steps)]
    for n in range(c.steps):
        ok(lib.me_save_checkpoint(h, ck[n]), h)
        e = ctypes.c_double(float(inp["ctrl"][n]))
        ok(lib.me_propagate_step(h, ctypes.byref(e), None), h)
    J = ctypes.c_double()
    ok(lib.me_dipole(h, ctypes.byref(J)), h)
    ok(lib.me_adjoint_begin(h, None), h)
    ge = np.zeros(c.steps)
    for n in reversed(range(c.steps)):
        ok(lib.me_load_checkpoint(h, ck[n]), h)
        g = ctypes.c_double()
        ok(lib.me_adjoint_step(h, float(inp["ctrl"][n]), ctypes.byref(g)), h)
        ge[n] = g.value
    gv = np.zeros((4, 4, 4))
    ok(lib.me_adjoint_grad_v(h, None, gv.ctypes.data, 4), h)
    dj = abs(J.value - J0)
    dge = np.abs(ge - ge0).max() / max(1e-3, np.abs(ge0).max())
    dgv = np.abs(gv - gv0).max() / max(1e-3, np.abs(gv0).max())
    print(f"adjoint: |dJ| {dj:.2e} rel|dge| {dge:.2e} rel|dgv| {dgv:.2e}", flush=True)
    tol = 1e-9 if prec == "f64" else 2e-3
    assert dj < tol * max(1.0, abs(J0)) and dge < tol and dgv < tol
    ok(lib.me_destroy(h))
elif scenario == "cp":
    # Car-Parrinello steps against the oracle's RATTLE / velocity Verlet
    mu_cp, dt = 50.0, 0.25
    for c in (W.C1, W.C1.replace(name="odd", n=20, n_orb=5, n_ions=5, placement="lattice", jitter=0.2, seed=77)):
        inp = W.make_inputs(c)
        h = new_system(c, inp)
        psi = orbitals(c, inp)
        ok(lib.me_set_state(h, psi.ctypes.data, c.n_points), h)
        ok(lib.me_cp_begin(h, mu_cp, dt), h)
        rep = B.StepReport()
        m = Model.from_config(c)
        st = cp.init_state(m, inp["psi"], inp["pos"])
        for k in range(4):
            ok(lib.me_cp_step(h, ctypes.byref(rep)), h)
            st = cp.cp_step(m, st, mu_cp, dt)
        psi_out, f = state(h, c)
        compare(f"cp {c.name} 4 steps", c, psi_out, f, st)
        e = cp.energy(m, st, mu_cp)
        de, dfict = abs(rep.e_total - e["total"]), abs(rep.e_fictitious - e["fictitious"])
        print(f"cp {c.name}: |dE_total| {de:.2e} |dE_fict| {dfict:.2e} (E_fict {e['fictitious']:.3e}) "
              f"constraint residual {rep.cp_constraint_residual:.1e}", flush=True)
        assert de < (1e-9 if prec == "f64" else 1e-3) * max(1.0, abs(e["total"]))
        assert dfict < (1e-9 if prec == "f64" else 1e-3) * max(1e-3, e["fictitious"])
        assert 0.0 <= rep.cp_constraint_residual < 1e-11
        s_ = m.overlaps(psi_out.reshape(st.psi.shape).astype(np.complex128))
        assert np.abs(s_ - np.eye(c.n_orb)).max() < (1e-12 if prec == "f64" else 2e-5)
        # any other step ends the CP run
        ok(lib.me_propagate_step(h, None, None), h)
        assert lib.me_cp_step(h, None) == B.ME_ESTATE
        ok(lib.me_destroy(h))
elif scenario == "etrs":
    # ETRS (two corrections of the second exponential) under a field, against
    # the oracle; batches and the adjoint refuse it
    for c in (W.C1, W.C1.replace(name="odd", n=20, n_orb=5, n_ions=5, placement="lattice", jitter=0.2, seed=77)):
        inp = W.make_inputs(c)
        h = new_system(c, inp, etrs_iterations=2)
        psi = orbitals(c, inp)
        ok(lib.me_set_state(h, psi.ctypes.data, c.n_points), h)
        m = Model.from_config(c)
        st = dynamics.init_state(m, inp["psi"], inp["pos"])
        rep = B.StepReport()
        for n in range(3):
            e = ctypes.c_double(0.01 * (n + 1))
            ok(lib.me_propagate_step(h, ctypes.byref(e), ctypes.byref(rep)), h)
            st = dynamics.etrs_step(m, st, e.value, iterations=2)
        psi_out, f = state(h, c)
        compare(f"etrs {c.name} 3 steps", c, psi_out, f, st)
        ok(lib.me_destroy(h))
    c = W.C1
    inp = W.make_inputs(c)
    p, keep = B.params_from_config(c, inp["pos"], precision=prec, etrs_iterations=1, enable_adjoint=True)
    size = ctypes.c_size_t(0)
    assert lib.me_workspace_size(ctypes.byref(p), ctypes.byref(size)) == B.ME_EUNSUPPORTED
    p, keep = B.params_from_config(c, inp["pos"], precision=prec, etrs_iterations=9)
    assert lib.me_workspace_size(ctypes.byref(p), ctypes.byref(size)) == B.ME_EINVAL
    arr = (B.Params * 1)()
    arr[0], keep = B.params_from_config(c, inp["pos"], precision=prec, etrs_iterations=1)
    ok(lib.me_batch_workspace_size(arr, 1, ctypes.byref(size)))
    hb = ctypes.c_void_p()
    assert lib.me_init_batch(arr, 1, buf(size.value), size.value, stream, ctypes.byref(hb)) == B.ME_EUNSUPPORTED
elif scenario == "finite":
    # the finite box: masked H, free-space Hartree by the doubled-grid FFTs,
    # isolated ions; three steps against the oracle's plain sums
    c = W.F0
    inp = W.make_inputs(c)
    m = finite.FiniteModel.from_config(c, pos0=inp["pos"], radius=c.finite_radius)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    h = new_system(c, inp)
    psi = orbitals(c, inp)
    ok(lib.me_set_state(h, psi.ctypes.data, c.n_points), h)
    vh = np.zeros(c.n_points)
    ok(lib.me_get_potential(h, 1, vh.ctypes.data), h)
    dv = np.abs(vh.reshape(m.grid.shape) - st.hist[-1]).max()
    print(f"finite: max|d v_Hxc| {dv:.2e}", flush=True)
    assert dv <= (1e-11 if prec == "f64" else 2e-6) * np.abs(st.hist[-1]).max()   # FP32: the orbitals are rounded on input
    rep = B.StepReport()
    for _ in range(3):
        ok(lib.me_propagate_step(h, None, ctypes.byref(rep)), h)
        st = dynamics.aetrs_step(m, st)
    psi_out, f = state(h, c)
    compare("finite 3 steps", c, psi_out, f, st)
    out = ~m.mask.astype(bool).ravel()
    assert np.abs(psi_out[:, out]).max() == 0.0
    e = dynamics.total_energy(m, st)
    de = abs(rep.e_total - e["total"])
    print(f"finite: |dE_total| {de:.2e} (E {e['total']:.6f})", flush=True)
    assert de < (1e-9 if prec == "f64" else 1e-4) * max(1.0, abs(e["total"]))
    e1 = ctypes.c_double(0.01)
    assert lib.me_propagate_step(h, ctypes.byref(e1), None) == B.ME_EUNSUPPORTED
    ok(lib.me_destroy(h))
    p, keep = B.params_from_config(c, inp["pos"], precision=prec, finite_radius=6.0)
    size = ctypes.c_size_t(0)
    assert lib.me_workspace_size(ctypes.byref(p), ctypes.byref(size)) == B.ME_EINVAL     # box touches the faces
    # more ions than one pass of the local-force kernel takes (groups of 8)
    c10 = c.replace(name="f10", n_ions=10, ring_radius=1.6, finite_radius=2.6, seed=1010)
    inp10 = W.make_inputs(c10)
    m10 = finite.FiniteModel.from_config(c10, pos0=inp10["pos"], radius=c10.finite_radius)
    h10 = new_system(c10, inp10)
    psi10 = orbitals(c10, inp10)                     # held: the copy is asynchronous
    ok(lib.me_set_state(h10, psi10.ctypes.data, c10.n_points), h10)
    _, f10 = state(h10, c10)
    want10 = m10.forces(inp10["pos"], inp10["psi"], m10.density(inp10["psi"]))["total"]
    d10 = np.abs(f10 - want10.ravel()).max()
    print(f"finite 10 ions: forces max|dF| {d10:.2e}", flush=True)
    assert d10 <= TOL_F * max(1.0, np.abs(want10).max())
    ok(lib.me_destroy(h10))
    # ETRS on the box: the corrections' v_Hxc comes from the free-space solve
    h = new_system(c, inp, etrs_iterations=1)
    ok(lib.me_set_state(h, psi.ctypes.data, c.n_points), h)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    for _ in range(2):
        ok(lib.me_propagate_step(h, None, None), h)
        st = dynamics.etrs_step(m, st, 0.0, iterations=1)
    psi_out, f = state(h, c)
    compare("finite ETRS 2 steps", c, psi_out, f, st)
    ok(lib.me_destroy(h))
elif scenario == "toy":
    # the toy-model sweep against the oracle: both schemes, uneven substeps
    # and windows, a trajectory with an invalid entry (NaN outputs), and the
    # distance kernel
    P = toy.ToyParams()
    tp = B.ToyParams(P.R0, P.M_R, P.K_R, P.G0, P.M_G, P.K_G)
    T, ns = 0.6 * P.period_R, 30
    dp = lambda a: ctypes.c_void_p(a.ctypes.data)
    for scheme, mus in (("ehrenfest", [1.5, 0.4, 0.1]), ("cp", [300.0, 60.0, 15.0])):
        mu = np.array(mus + [mus[0], -1.0])
        sub = np.array([3, 4, 20, 24, 3], np.int32)    # omega dt < 1 everywhere
        win = np.array([2, 1, 3, 5, 2], np.int32)
        n = mu.size
        S = np.zeros((ns + 1, 8 if scheme == "cp" else 6, n))
        dR, dF = np.zeros(n), np.zeros(n)
        ok(lib.me_toy_run(ctypes.byref(tp), B.TOY_SCHEMES[scheme], n, ns, T, 24, dp(mu), dp(sub), dp(win), dp(S),
                          dp(dR), dp(dF), stream))
        for i in range(n - 1):
            r = toy.run(P, scheme, [mu[i]], int(sub[i]), ns, T, window=[int(win[i])])
            ds = np.abs(S[:, :, i] - r["samples"][0]).max()
            print(f"toy {scheme} mu={mu[i]} sub={sub[i]}: max|d samples| {ds:.2e} d_R {dR[i]:.6f} "
                  f"({r['d_R'][0]:.6f}) d_F {dF[i]:.6f} ({r['d_F'][0]:.6f})", flush=True)
            assert ds < 1e-12
            assert abs(dR[i] - r["d_R"][0]) < 1e-10 * max(1.0, r["d_R"][0])
            assert abs(dF[i] - r["d_F"][0]) < 1e-10 * max(1.0, r["d_F"][0])
        assert np.isnan(dR[-1]) and np.isnan(dF[-1]) and np.isnan(S[:, :, -1]).all()
        ref = np.array([3, 3, 3, 3, 7], np.int32)
        dist = np.zeros(n)
        ok(lib.me_toy_distance(n, ns, S.shape[1], dp(S), dp(ref), dp(dist), stream))
        want = toy.trajectory_distance(np.moveaxis(S, 2, 0)[:4], np.moveaxis(S, 2, 0)[3])
        assert np.abs(dist[:4] - want).max() < 1e-12 * max(1.0, np.abs(want).max()), (dist, want)
        assert dist[3] == 0.0 and np.isnan(dist[4])
    bad = B.ToyParams(P.R0, 0.0, P.K_R, P.G0, P.M_G, P.K_G)
    z = np.zeros(1)
    assert lib.me_toy_run(ctypes.byref(bad), 0, 1, ns, T, 1, dp(z), dp(z), dp(z), None, dp(z), dp(z), stream) == B.ME_EINVAL
    assert lib.me_toy_run(ctypes.byref(tp), 0, 1, 1 << 12, T, 1 << 13, dp(z), dp(z), dp(z), None, dp(z), dp(z),
                          stream) == B.ME_EINVAL
elif scenario == "c2_sequence":
    # the benchmark's call sequence on the 96^3 workload (its grid, its 64
    # ions and projector tables, 2 of its 128 orbitals): state, one step
    # (sampled against the oracle), 3 warm-up steps, timing on, 6 steps (every
    # phase of the table / buffer / history rotation), timing read, timing
    # off, report, destroy, then the workspace released while the runtime
    # stays live
    c = W.C2.replace(n_orb=2)
    inp = W.make_inputs(c)
    h = new_system(c, inp)
    ws_holder = len(held) - 1                # new_system's last buffer is the workspace
    psi0 = orbitals(c, inp)
    held.append(psi0)
    ok(lib.me_set_state(h, psi0.ctypes.data, c.n_points), h)
    ok(lib.me_propagate_step(h, None, None), h)
    got, _ = state(h, c)
    m = Model.from_config(c)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    pos1, h0, h1 = dynamics.step_hamiltonians(m, st)
    ref = dynamics.propagate_orbitals(m, inp["psi"], h0, h1).reshape(c.n_orb, -1)
    d1 = float(np.abs(got - ref).max())
    print(f"c2_sequence: one step max|dpsi| {d1:.2e}", flush=True)
    assert d1 <= TOL_PSI * 10
    for _ in range(3):
        ok(lib.me_propagate_step(h, None, None), h)
    ok(lib.me_timing_enable(h, 1), h)
    for _ in range(6):
        ok(lib.me_propagate_step(h, None, None), h)
    n_, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    ok(lib.me_timing_read(h, ctypes.byref(n_), ctypes.byref(ms), ctypes.byref(by)), h)
    assert n_.value == 6 * 2 * 4, n_.value
    ok(lib.me_timing_enable(h, 0), h)
    rep = B.StepReport()
    ok(lib.me_report(h, ctypes.byref(rep)), h)
    print(f"c2_sequence: 10 steps, max norm deviation {rep.max_norm_dev:.2e}", flush=True)
    assert rep.max_norm_dev < 1e-5
    ok(lib.me_destroy(h))
    # the workspace goes back to the allocator (ASan poisons it): any access
    # that outlived the handle would now be reported
    del held[ws_holder]
    import gc
    gc.collect()
    ok(lib.me_dipole_noalloc(ctypes.c_void_p(np.zeros(8).ctypes.data), (ctypes.c_int32 * 3)(2, 2, 2), 0.3,
                             ctypes.c_void_p(np.zeros(1).ctypes.data), stream))
elif scenario == "noalloc":
    # the dipole with its partials in the library's fixed array: the same
    # bits as me_dipole on a system's density, then a smaller, non-cubic
    # density against the oracle's objective, then the refusals
    c = W.C1.replace(n=20, n_orb=3, seed=1201)
    inp = W.make_inputs(c)
    h = new_system(c, inp)
    psi0 = orbitals(c, inp)
    held.append(psi0)                        # the copy runs when the stream does
    ok(lib.me_set_state(h, psi0.ctypes.data, c.n_points), h)
    rho = np.zeros(c.n_points)
    ok(lib.me_density(h, rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), h)
    ok(lib.me_sync(h), h)
    d_sys = ctypes.c_double(0.0)
    ok(lib.me_dipole(h, ctypes.byref(d_sys)), h)
    d_dev = np.full(1, np.nan)
    n3 = (ctypes.c_int32 * 3)(c.n, c.n, c.n)
    ok(lib.me_dipole_noalloc(ctypes.c_void_p(rho.ctypes.data), n3, c.h, ctypes.c_void_p(d_dev.ctypes.data), stream))
    ok(lib.me_sync(h), h)
    print(f"noalloc {c.n}^3: {d_dev[0]!r} me_dipole {d_sys.value!r}", flush=True)
    assert d_dev[0] == d_sys.value
    ok(lib.me_destroy(h))
    m = Model(n=c.n, h=c.h, zval=np.zeros(0), mass=np.zeros(0))
    assert abs(d_dev[0] - adjoint.objective(m, rho.reshape(c.n, c.n, c.n))) < 1e-12 * abs(d_dev[0])
    rng = np.random.default_rng(5)
    small = rng.random((7, 10, 12))          # (z, y, x): n = (12, 10, 7)
    n3s = (ctypes.c_int32 * 3)(12, 10, 7)
    ok(lib.me_dipole_noalloc(ctypes.c_void_p(small.ctypes.data), n3s, 0.3, ctypes.c_void_p(d_dev.ctypes.data), stream))
    want = 0.3 ** 3 * float(np.sum((0.3 * np.arange(12) - 0.5 * 12 * 0.3)[None, None, :] * small))
    print(f"noalloc 12x10x7: {d_dev[0]!r} want {want!r}", flush=True)
    assert abs(d_dev[0] - want) < 1e-13 * max(1.0, abs(want))
    big = (ctypes.c_int32 * 3)(1024, 1024, 1024)
    assert lib.me_dipole_noalloc(ctypes.c_void_p(small.ctypes.data), big, 0.3, ctypes.c_void_p(d_dev.ctypes.data),
                                 stream) == B.ME_EINVAL
    assert b"too large" in lib.me_last_error(None)
    assert lib.me_dipole_noalloc(None, n3s, 0.3, ctypes.c_void_p(d_dev.ctypes.data), stream) == B.ME_EINVAL
else:
    raise SystemExit(f"unknown scenario {scenario}")

leaked = lib.mock_live_handles() - base_handles
assert leaked == 0, f"{leaked} runtime handles not released"
assert lib.mock_memsets_in_capture() == 0, "hipMemsetAsync recorded in a captured graph"
print("OK", scenario, prec, flush=True)
