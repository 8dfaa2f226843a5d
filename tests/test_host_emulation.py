"""The library's kernels and host code executed on the CPU: the HIP sources
are rewritten for the emulator in tests/host_emu (work-items as cooperative
coroutines, wave operations, graph capture replayed, rocFFT by direct DFTs),
built with clang++ and AddressSanitizer/UBSan, with a poisoned redzone after
every workspace buffer, and driven through the C ABI.  Each scenario checks
the results against the FP64 oracle (FP64 to rounding, FP32 and split-bf16
to single precision) and fails on any access out of bounds, misuse of
streams, events or captures, or leaked handle.  Sizes are small (16^3-40^3)
but take the ragged tiles, z-slabs, two halo runs per thread, odd orbital
counts, systems without ions, graph capture and replay, and the adjoint."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "host_emu")
CSRC = os.path.join(ROOT, "paper_0812_2801_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
ASAN_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

SCENARIOS = [("system", "f64"), ("system", "f32"), ("system", "f32_bf16x3"), ("batch", "f64"),
             ("batch", "f32"), ("adjoint", "f64"), ("adjoint", "f32"), ("cp", "f64"), ("cp", "f32"),
             ("etrs", "f64"), ("toy", "f64"), ("finite", "f64"), ("finite", "f32"), ("noalloc", "f64"), ("system_xt", "f64"), ("system_xt", "f32"),
             ("adjoint_xt", "f64"), ("c2_sequence", "f32"), ("c2_sequence", "f32_bf16x3"), ("batch_xt", "f64"),
             ("batch_xt", "f32"), ("system_py", "f64"), ("system_py", "f32")]

pytestmark = pytest.mark.skipif(not (os.path.exists(CLANG) and ASAN_RT), reason="needs ROCm clang++ and its ASan runtime")


def _build(d):
    src = os.path.join(d, "src")
    r = subprocess.run([sys.executable, os.path.join(EMU, "transform.py"), CSRC, src, os.path.join(ROOT, "include")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    flags = ["-std=c++17", "-g", "-O2", "-fPIC", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-mllvm", "-asan-stack=0", "-fsanitize-address-use-after-return=never",
             f"-I{EMU}", f"-I{src}", f"-I{os.path.join(ROOT, 'include')}", "-Wno-unknown-pragmas", "-Wno-unused-value"]
    files = sorted(glob.glob(os.path.join(src, "*.cpp"))) + [os.path.join(EMU, "emu.cpp")]
    procs = []
    for f in files:
        obj = os.path.join(d, os.path.basename(f)[:-4] + ".o")
        procs.append((f, obj, subprocess.Popen([CLANG, *flags, "-c", f, "-o", obj], stderr=subprocess.PIPE, text=True)))
    for f, obj, p in procs:
        err = p.communicate()[1]
        assert p.returncode == 0, f"{f}:\n{err[-3000:]}"
    lib = os.path.join(d, "libmodehr_emu.so")
    r = subprocess.run([CLANG, "-shared", "-shared-libsan", "-fsanitize=address,undefined", "-o", lib,
                        *[o for _, o, _ in procs]], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return lib


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("host_emu"))
    lib = _build(d)
    env = dict(os.environ, LD_PRELOAD=ASAN_RT[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
    procs = {}
    for sc, prec in SCENARIOS:
        wd = os.path.join(d, f"{sc}_{prec}")
        os.makedirs(wd, exist_ok=True)
        # the _xt scenarios force the x-tiled stencil (16 x 8 tiles) on their grids
        env_sc = dict(env, MODEHR_TX="16", MODEHR_TY="8", MODEHR_BATCH_TX="16") if sc.endswith("_xt") else env
        # the _py scenarios force whole-row tiles of 8 rows with two rows per thread
        env_sc = dict(env_sc, MODEHR_PY="2", MODEHR_PY_TY="8") if sc.endswith("_py") else env_sc
        procs[(sc, prec)] = subprocess.Popen([sys.executable, "-u", os.path.join(EMU, "drive.py"), lib, sc, prec, wd],
                                             stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env_sc)
    out = {}
    for k, p in procs.items():
        try:
            so, se = p.communicate(timeout=600)
        except subprocess.TimeoutExpired:
            p.kill()
            so, se = p.communicate()
        out[k] = (p.returncode, so, se)
    return out


@pytest.mark.parametrize("scenario,prec", SCENARIOS)
def test_kernels_on_cpu_emulation(results, scenario, prec):
    rc, so, se = results[(scenario, prec)]
    se = "\n".join(l for l in se.splitlines() if "doesn't fully support makecontext" not in l)
    assert rc == 0 and f"OK {scenario} {prec}" in so, (so[-3000:], se[-6000:])
