"""The C ABI on the CPU: the built library loads, exports every function
declared in include/*.h, and validates parameters on the host (no device
work is launched by these calls)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(me_status|const\s+char\s*\*)\s*(me_\w+)\s*\(", text):
            names.add(m.group(2))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_0812_2801_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        from paper_0812_2801_amd.build import build
        build()
    return B.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_0812_2801_amd import binding as B
    assert set(B.SYMBOLS) <= set(names)


def test_workspace_size_is_pure_host_and_scales(lib):
    from paper_0812_2801_amd import binding as B
    pos = W.ion_positions(W.C1)
    p64, k1 = B.params_from_config(W.C1, pos, precision="f64")
    p32, k2 = B.params_from_config(W.C1, pos, precision="f32")
    s64 = B.workspace_size(p64)
    s32 = B.workspace_size(p32)
    N = W.C1.n ** 3
    # three orbital buffers dominate: complex128 vs complex64
    assert s64 > 3 * W.C1.n_orb * N * 16
    assert s32 > 3 * W.C1.n_orb * N * 8
    assert s64 > s32


@pytest.mark.parametrize("field,value,status", [
    ("n_orb", 0, 1), ("h", -0.3, 1), ("mu", 0.0, 1), ("dt", 0.0, 1),
    ("taylor_order", 0, 1), ("taylor_order", 9, 1), ("precision", 7, 1),
    ("kb_rcut", 2.5, 1), ("enable_adjoint", 1, 6),
])
def test_invalid_parameters_are_rejected(lib, field, value, status):
    from paper_0812_2801_amd import binding as B
    p, keep = B.params_from_config(W.C1, W.ion_positions(W.C1))
    setattr(p, field, value)
    out = ctypes.c_size_t(0)
    st = lib.me_workspace_size(ctypes.byref(p), ctypes.byref(out))
    assert st == status
    assert lib.me_last_error(None).decode() != ""


def test_grid_bounds_and_null_checks(lib):
    from paper_0812_2801_amd import binding as B
    p, keep = B.params_from_config(W.C1, W.ion_positions(W.C1))
    p.n[0] = 4
    out = ctypes.c_size_t(0)
    assert lib.me_workspace_size(ctypes.byref(p), ctypes.byref(out)) == B.ME_EINVAL
    assert lib.me_workspace_size(None, ctypes.byref(out)) == B.ME_EINVAL
    p2, k2 = B.params_from_config(W.C1, W.ion_positions(W.C1))
    assert lib.me_workspace_size(ctypes.byref(p2), None) == B.ME_EINVAL
    h = ctypes.c_void_p()
    # no workspace: rejected before any device call
    assert lib.me_init_system(ctypes.byref(p2), None, 0, None, ctypes.byref(h)) == B.ME_EINVAL
    assert lib.me_destroy(None) == B.ME_OK
    assert lib.me_strerror(B.ME_EUNSTABLE).decode() == "propagation unstable"


def _batch_params(B, cfgs, **over):
    ps, keep = [], []
    for c in cfgs:
        p, k = B.params_from_config(c, W.ion_positions(c), **over)
        ps.append(p)
        keep.append(k)
    return (B.Params * len(ps))(*ps), keep


def test_batch_workspace_is_the_sum_of_the_systems(lib):
    from paper_0812_2801_amd import binding as B
    cfgs = [W.C1, W.C1.replace(n=24, n_orb=8, seed=3), W.C1.replace(n=20, n_ions=0)]
    arr, keep = _batch_params(B, cfgs)
    total = ctypes.c_size_t(0)
    assert lib.me_batch_workspace_size(arr, len(cfgs), ctypes.byref(total)) == B.ME_OK
    singles = sum(-(-B.workspace_size(arr[i]) // 256) * 256 for i in range(len(cfgs)))
    assert singles < total.value <= singles + 4096


def test_batch_validation_happens_on_the_host(lib):
    from paper_0812_2801_amd import binding as B
    total = ctypes.c_size_t(0)
    arr, keep = _batch_params(B, [W.C1])
    assert lib.me_batch_workspace_size(arr, 0, ctypes.byref(total)) == B.ME_EINVAL
    assert lib.me_batch_workspace_size(arr, 33, ctypes.byref(total)) == B.ME_EINVAL
    assert lib.me_batch_last_error(None).decode() != ""
    # mixed precision / Taylor order and oversize rows are refused before the
    # workspace (a fake, aligned, never dereferenced address) is touched
    a, k1 = B.params_from_config(W.C1, W.ion_positions(W.C1), precision="f32")
    b, k2 = B.params_from_config(W.C1, W.ion_positions(W.C1), precision="f64")
    mixed = (B.Params * 2)(a, b)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.me_init_batch(mixed, 2, fake, 1 << 40, None, ctypes.byref(h)) == B.ME_EINVAL
    c, k3 = B.params_from_config(W.C1, W.ion_positions(W.C1), precision="f32", taylor_order=3)
    mixed = (B.Params * 2)(a, c)
    assert lib.me_init_batch(mixed, 2, fake, 1 << 40, None, ctypes.byref(h)) == B.ME_EINVAL
    # rows wider than one workgroup are taken in x-tiles: a 200-point row
    # passes validation and is stopped only by the too-small workspace
    big, k4 = B.params_from_config(W.C1.replace(n=200, h=0.3), W.ion_positions(W.C1), precision="f32")
    one = (B.Params * 1)(big)
    assert lib.me_init_batch(one, 1, fake, 16, None, ctypes.byref(h)) == B.ME_ENOMEM
    adj, k5 = B.params_from_config(W.C1, W.ion_positions(W.C1), precision="f32", enable_adjoint=True,
                                   freeze_ions=True)
    one = (B.Params * 1)(adj)
    assert lib.me_init_batch(one, 1, fake, 1 << 40, None, ctypes.byref(h)) == B.ME_EUNSUPPORTED
    assert lib.me_init_batch(arr, 1, fake, 16, None, ctypes.byref(h)) == B.ME_ENOMEM
    assert lib.me_propagate_batch(None, 1, 1) == B.ME_EINVAL
    assert lib.me_batch_destroy(None) == B.ME_OK


def test_one_hip_runtime_in_the_process():
    # the library binds to the HIP runtime torch brought (same soname), so
    # device memory and streams from torch are the library's own
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_0812_2801_amd import binding as B\n"
            "B.load()\n"
            "maps = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(maps))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1", out.stdout
