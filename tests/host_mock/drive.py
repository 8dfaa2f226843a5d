"""Drives the library's host code, built against the CPU stand-in runtime
(mock_rt.cpp), through the C ABI: usage drive.py LIB SCENARIO [PRECISION].
Exits non-zero (the stand-in aborts) on any misuse it detects; prints OK."""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import workloads as W                                      # noqa: E402
from paper_0812_2801_amd import binding as B               # noqa: E402

lib = B.load(sys.argv[1])
lib.mock_new_stream.restype = ctypes.c_void_p
lib.mock_live_handles.restype = ctypes.c_long
lib.mock_memsets_in_capture.restype = ctypes.c_long
scenario = sys.argv[2]
prec = sys.argv[3] if len(sys.argv) > 3 else "f64"
stream = lib.mock_new_stream()
held = []                                                  # host "device" buffers


def buf(nbytes):
    a = np.zeros(nbytes + 256, np.uint8)
    held.append(a)
    return (a.ctypes.data + 255) // 256 * 256


def ok(st, h=None, batch=False):
    if st != B.ME_OK:
        err = (lib.me_batch_last_error if batch else lib.me_last_error)(h)
        raise SystemExit(f"status {st}: {err.decode()}")


def orbitals(c):
    return np.zeros((c.n_orb, c.n ** 3), np.complex128 if prec == "f64" else np.complex64)


UNEVEN = [
    W.C1.replace(name="b0", seed=1001),
    W.C1.replace(name="b1", n=24, n_orb=6, n_ions=5, placement="lattice", jitter=0.2, seed=1002),
    W.C1.replace(name="b2", n=20, n_orb=3, n_ions=0, seed=1003),
    W.C1.replace(name="b3", n=40, h=0.25, n_orb=2, n_ions=3, placement="lattice", jitter=0.2, seed=1004),
]
base_handles = lib.mock_live_handles()

if scenario == "batch":
    arr = (B.Params * len(UNEVEN))()
    keep = []
    for i, c in enumerate(UNEVEN):
        p, k = B.params_from_config(c, W.ion_positions(c), precision=prec)
        arr[i] = p
        keep.append(k)
    size = ctypes.c_size_t(0)
    ok(lib.me_batch_workspace_size(arr, len(UNEVEN), ctypes.byref(size)))
    h = ctypes.c_void_p()
    ok(lib.me_init_batch(arr, len(UNEVEN), buf(size.value), size.value, stream, ctypes.byref(h)))
    for i, c in enumerate(UNEVEN):
        s = ctypes.c_void_p()
        ok(lib.me_batch_system(h, i, ctypes.byref(s)), h, True)
        psi = orbitals(c)
        held.append(psi)
        ok(lib.me_set_state(s, psi.ctypes.data, c.n ** 3), s)
    ok(lib.me_propagate_batch(h, 14, 1), h, True)          # warm-up, capture, two replays
    ok(lib.me_propagate_batch(h, 9, 1), h, True)           # one replay and three eager steps
    ok(lib.me_propagate_batch(h, 7, 1), h, True)           # another phase: recapture
    ok(lib.me_propagate_batch(h, 2, 0), h, True)
    t = B.BatchTuning()
    ok(lib.me_batch_autotune(h, os.path.join(sys.argv[4], "tune.json").encode(), ctypes.byref(t)), h, True)
    ok(lib.me_batch_timing_enable(h, 1), h, True)
    ok(lib.me_propagate_batch(h, 2, 0), h, True)
    n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    ok(lib.me_batch_timing_read(h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)), h, True)
    assert n.value == 2 * 2 * 4, n.value                   # 2 steps x 2 exponentials x 4 stages
    ok(lib.me_batch_timing_enable(h, 0), h, True)
    ok(lib.me_propagate_batch(h, 6, 1), h, True)
    ok(lib.me_batch_destroy(h))
elif scenario in ("system", "adjoint"):
    adj = scenario == "adjoint"
    c = W.C1.replace(freeze_ions=True) if adj else W.C1.replace(n=24, n_ions=5, placement="lattice", jitter=0.2)
    p, keep = B.params_from_config(c, W.ion_positions(c), precision=prec, enable_adjoint=adj)
    size = ctypes.c_size_t(0)
    ok(lib.me_workspace_size(ctypes.byref(p), ctypes.byref(size)))
    h = ctypes.c_void_p()
    ok(lib.me_init_system(ctypes.byref(p), buf(size.value), size.value, stream, ctypes.byref(h)))
    psi = orbitals(c)
    ok(lib.me_set_state(h, psi.ctypes.data, c.n ** 3), h)
    rep = B.StepReport()
    cp = ctypes.c_size_t(0)
    ok(lib.me_checkpoint_size(h, ctypes.byref(cp)), h)
    ckpt = [buf(cp.value) for _ in range(4)]
    ok(lib.me_timing_enable(h, 1), h)
    for n in range(4):
        ok(lib.me_save_checkpoint(h, ckpt[n]), h)
        e = ctypes.c_double(0.01 * n)
        ok(lib.me_propagate_step(h, ctypes.byref(e), ctypes.byref(rep)), h)
    n_, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    ok(lib.me_timing_read(h, ctypes.byref(n_), ctypes.byref(ms), ctypes.byref(by)), h)
    assert n_.value == 4 * 2 * 4, n_.value
    ok(lib.me_timing_enable(h, 0), h)
    out = orbitals(c)
    ok(lib.me_apply_H(h, psi.ctypes.data, out.ctypes.data, c.n_orb, c.n ** 3), h)
    rho = np.zeros(c.n ** 3)
    ok(lib.me_density(h, rho.ctypes.data), h)
    f = np.zeros(3 * c.n_ions)
    ok(lib.me_forces(h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), h)
    if adj:
        ok(lib.me_adjoint_begin(h, None), h)
        g = ctypes.c_double()
        for n in reversed(range(4)):
            ok(lib.me_load_checkpoint(h, ckpt[n]), h)
            ok(lib.me_adjoint_step(h, 0.01 * n, ctypes.byref(g)), h)
        gv = np.zeros(c.n ** 3)
        ok(lib.me_adjoint_grad_v(h, gv.ctypes.data, None, 0), h)
    ok(lib.me_destroy(h))
else:
    raise SystemExit(f"unknown scenario {scenario}")

leaked = lib.mock_live_handles() - base_handles
assert leaked == 0, f"{leaked} runtime handles not released"
assert lib.mock_memsets_in_capture() == 0, "hipMemsetAsync recorded in a captured graph"
print("OK", scenario, prec, flush=True)
