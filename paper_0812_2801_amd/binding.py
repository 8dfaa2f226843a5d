"""Python binding of libmodehr.so (the C ABI in include/modehr.h).

Argument marshalling only: every step of the propagation runs in the HIP
library.  PyTorch provides device memory (the workspace and orbital
tensors) and the stream.  If the library is missing or cannot be loaded the
binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MODEHR_LIB", os.path.join(HERE, "libmodehr.so"))

ME_OK, ME_EINVAL, ME_ENOMEM, ME_EDEVICE, ME_ESTATE, ME_EUNSTABLE, ME_EUNSUPPORTED = range(7)
PRECISION = {"f64": 0, "f32": 1, "f32_bf16x3": 2}

SYMBOLS = [
    "me_workspace_size", "me_init_system", "me_destroy", "me_sync", "me_set_state",
    "me_get_state", "me_apply_H", "me_propagate_step", "me_report", "me_density",
    "me_forces", "me_get_ions", "me_get_potential", "me_set_static_potential",
    "me_timing_enable", "me_timing_read", "me_last_error", "me_strerror",
    "me_checkpoint_size", "me_save_checkpoint", "me_load_checkpoint",
    "me_set_static_potential_coarse", "me_dipole", "me_adjoint_begin", "me_adjoint_step",
    "me_adjoint_grad_v", "me_cp_begin", "me_cp_step",
    "me_batch_workspace_size", "me_init_batch", "me_batch_system", "me_batch_set_tuning",
    "me_batch_get_tuning", "me_batch_autotune", "me_propagate_batch", "me_batch_timing_enable",
    "me_batch_timing_read", "me_batch_last_error", "me_batch_destroy",
    "me_toy_run", "me_toy_distance", "me_dipole_noalloc", "me_timing_read_kind", "me_batch_timing_read_kind",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("n", c_int32 * 3), ("h", c_double), ("n_ions", c_int32),
        ("pos", POINTER(c_double)), ("vel", POINTER(c_double)),
        ("mass", POINTER(c_double)), ("zval", POINTER(c_double)),
        ("loc_a", c_double), ("kb_sigma", c_double), ("kb_rcut", c_double),
        ("kb_energy", c_double), ("n_orb", c_int32), ("occ", c_double),
        ("mu", c_double), ("dt", c_double), ("taylor_order", c_int32),
        ("precision", c_int32), ("freeze_ions", c_int32), ("enable_adjoint", c_int32),
        ("nl_force_form", c_int32), ("etrs_iterations", c_int32), ("finite_radius", c_double),
    ]


class StepReport(ctypes.Structure):
    _fields_ = [(k, c_double) for k in (
        "e_kinetic", "e_local", "e_hartree", "e_xc", "e_nonlocal", "e_ion", "e_ks",
        "e_ion_kinetic", "e_total", "max_norm_dev", "max_force", "charge")] + [("step", c_int64)] + [
        ("e_fictitious", c_double), ("cp_constraint_residual", c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchTuning(ctypes.Structure):
    _fields_ = [("block", c_int32), ("wg_per_cu", c_int32), ("zdiv", c_int32), ("stage_ms", c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ToyParams(ctypes.Structure):
    """me_toy_params: the constants of eq. L_toy."""
    _fields_ = [("R0", c_double), ("M_R", c_double), ("K_R", c_double),
                ("G0", c_double), ("M_G", c_double), ("K_G", c_double)]


class ModehrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"modehr status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library (once).  Raises if it is missing or lacks a symbol."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_0812_2801_amd.build")
    # torch first: it brings its own HIP runtime, rocFFT and rocBLAS under the
    # same sonames, and the library must bind to those.  Loaded the other way
    # round, the process maps two HIP runtimes (ROCm's and torch's), device
    # memory from one is handed to the other, and rocFFT plans fail.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for s in SYMBOLS:
        getattr(lib, s)
    lib.me_last_error.restype = c_char_p
    lib.me_last_error.argtypes = [c_void_p]
    lib.me_strerror.restype = c_char_p
    lib.me_strerror.argtypes = [c_int32]
    lib.me_workspace_size.argtypes = [POINTER(Params), POINTER(c_size_t)]
    lib.me_init_system.argtypes = [POINTER(Params), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]
    lib.me_destroy.argtypes = [c_void_p]
    lib.me_sync.argtypes = [c_void_p]
    lib.me_set_state.argtypes = [c_void_p, c_void_p, c_int64]
    lib.me_get_state.argtypes = [c_void_p, c_void_p, c_int64]
    lib.me_apply_H.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int64]
    lib.me_propagate_step.argtypes = [c_void_p, POINTER(c_double), POINTER(StepReport)]
    lib.me_report.argtypes = [c_void_p, POINTER(StepReport)]
    lib.me_density.argtypes = [c_void_p, c_void_p]
    lib.me_forces.argtypes = [c_void_p, POINTER(c_double)]
    lib.me_get_ions.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double)]
    lib.me_get_potential.argtypes = [c_void_p, c_int32, c_void_p]
    lib.me_set_static_potential.argtypes = [c_void_p, c_void_p]
    lib.me_timing_enable.argtypes = [c_void_p, c_int32]
    lib.me_timing_read.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_double), POINTER(c_double)]
    lib.me_timing_read_kind.argtypes = [c_void_p, c_int32, POINTER(c_int64), POINTER(c_double), POINTER(c_double)]
    lib.me_checkpoint_size.argtypes = [c_void_p, POINTER(c_size_t)]
    lib.me_save_checkpoint.argtypes = [c_void_p, c_void_p]
    lib.me_load_checkpoint.argtypes = [c_void_p, c_void_p]
    lib.me_set_static_potential_coarse.argtypes = [c_void_p, c_void_p, c_int32]
    lib.me_dipole.argtypes = [c_void_p, POINTER(c_double)]
    lib.me_dipole_noalloc.argtypes = [c_void_p, POINTER(c_int32), c_double, c_void_p, c_void_p]
    lib.me_adjoint_begin.argtypes = [c_void_p, c_void_p]
    lib.me_adjoint_step.argtypes = [c_void_p, c_double, POINTER(c_double)]
    lib.me_adjoint_grad_v.argtypes = [c_void_p, c_void_p, c_void_p, c_int32]
    lib.me_cp_begin.argtypes = [c_void_p, c_double, c_double]
    lib.me_cp_step.argtypes = [c_void_p, POINTER(StepReport)]
    lib.me_batch_workspace_size.argtypes = [POINTER(Params), c_int32, POINTER(c_size_t)]
    lib.me_init_batch.argtypes = [POINTER(Params), c_int32, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]
    lib.me_batch_system.argtypes = [c_void_p, c_int32, POINTER(c_void_p)]
    lib.me_batch_set_tuning.argtypes = [c_void_p, POINTER(BatchTuning)]
    lib.me_batch_get_tuning.argtypes = [c_void_p, POINTER(BatchTuning)]
    lib.me_batch_autotune.argtypes = [c_void_p, c_char_p, POINTER(BatchTuning)]
    lib.me_propagate_batch.argtypes = [c_void_p, c_int32, c_int32]
    lib.me_batch_timing_enable.argtypes = [c_void_p, c_int32]
    lib.me_batch_timing_read.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_double), POINTER(c_double)]
    lib.me_batch_timing_read_kind.argtypes = [c_void_p, c_int32, POINTER(c_int64), POINTER(c_double),
                                              POINTER(c_double)]
    lib.me_batch_last_error.restype = c_char_p
    lib.me_batch_last_error.argtypes = [c_void_p]
    lib.me_batch_destroy.argtypes = [c_void_p]
    lib.me_toy_run.argtypes = [POINTER(ToyParams), c_int32, c_int32, c_int32, c_double, c_int32, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.me_toy_distance.argtypes = [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
    for s in SYMBOLS:
        if s not in ("me_last_error", "me_strerror", "me_batch_last_error"):
            getattr(lib, s).restype = c_int32
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def make_params(*, n, h, pos, mass, zval, n_orb, mu, dt, vel=None, loc_a=0.5,
                kb_sigma=0.4, kb_rcut=1.2, kb_energy=2.0, occ=2.0, taylor_order=4,
                precision="f64", freeze_ions=False, enable_adjoint=False, nl_force_form=0,
                etrs_iterations=0, finite_radius=0.0):
    """Params plus the host arrays it points to (keep both alive)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float64).ravel()
    zval = np.ascontiguousarray(zval, dtype=np.float64).ravel()
    keep = [pos, mass, zval]
    p = Params()
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    p.n = (c_int32 * 3)(*nn)
    p.h = h
    p.n_ions = len(pos)
    p.pos = _dptr(pos)
    if vel is not None:
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        keep.append(vel)
        p.vel = _dptr(vel)
    p.mass = _dptr(mass)
    p.zval = _dptr(zval)
    p.loc_a, p.kb_sigma, p.kb_rcut, p.kb_energy = loc_a, kb_sigma, kb_rcut, kb_energy
    p.n_orb = n_orb
    p.occ, p.mu, p.dt = occ, mu, dt
    p.taylor_order = taylor_order
    p.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    p.freeze_ions = int(bool(freeze_ions))
    p.enable_adjoint = int(bool(enable_adjoint))
    p.nl_force_form = int(nl_force_form)
    p.etrs_iterations = int(etrs_iterations)
    p.finite_radius = float(finite_radius)
    return p, keep


def params_from_config(cfg, pos, vel=None, precision=None, **over):
    kw = dict(n=cfg.n, h=cfg.h, pos=pos, mass=np.full(cfg.n_ions, cfg.mass),
              zval=np.full(cfg.n_ions, cfg.zval), n_orb=cfg.n_orb, mu=cfg.mu, dt=cfg.dt,
              vel=vel, loc_a=cfg.loc_a, kb_sigma=cfg.kb_sigma, kb_rcut=cfg.kb_rcut,
              kb_energy=cfg.kb_energy, occ=cfg.occ,
              precision=precision or cfg.precision, freeze_ions=cfg.freeze_ions,
              finite_radius=getattr(cfg, "finite_radius", 0.0))
    kw.update(over)
    return make_params(**kw)


def workspace_size(p: Params) -> int:
    lib = load()
    out = c_size_t(0)
    st = lib.me_workspace_size(ctypes.byref(p), ctypes.byref(out))
    if st != ME_OK:
        raise ModehrError(st, lib.me_last_error(None).decode())
    return out.value


class System:
    """One system on one GPU; device memory from torch, work on torch's current stream."""

    def __init__(self, params: Params, keep=None, device="cuda:0", handle=None, stream=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.params = params
        self._keep = keep
        self.device = torch.device(device)
        self.cdtype = torch.complex128 if params.precision == 0 else torch.complex64
        self.N = params.n[0] * params.n[1] * params.n[2]
        self.n_orb = params.n_orb
        self.n_ions = params.n_ions
        self._owned = handle is None
        if handle is not None:          # a system owned by a Batch, on the batch's stream
            self.h = handle
            self.stream = stream
            return
        size = workspace_size(params)
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = c_void_p()
        st = self.lib.me_init_system(ctypes.byref(params), c_void_p(self.workspace.data_ptr()),
                                     c_size_t(size), c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h))
        if st != ME_OK:
            raise ModehrError(st, self.lib.me_last_error(None).decode())
        self.h = h

    # -------------------------------------------------------------- helpers
    def _check(self, st: int):
        self._post()
        if st != ME_OK:
            raise ModehrError(st, self.lib.me_last_error(self.h).decode())

    def _pre(self):
        """Order the handle's stream after torch's current stream (inputs ready)."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _post(self):
        """Order torch's current stream after the handle's (outputs ready)."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def close(self):
        if getattr(self, "h", None):
            if self._owned:
                self.lib.me_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _orbitals(self, psi):
        t = self.torch
        if not isinstance(psi, t.Tensor):
            psi = t.from_numpy(np.ascontiguousarray(psi))
        psi = psi.to(device=self.device, dtype=self.cdtype).reshape(psi.shape[0], -1).contiguous()
        if psi.shape[1] != self.N:
            raise ValueError("orbitals must have N grid points each")
        return psi

    # -------------------------------------------------------------- API
    def set_state(self, psi):
        psi = self._orbitals(psi)
        if psi.shape[0] != self.n_orb:
            raise ValueError("set_state needs n_orb orbitals")
        self._check(self._pre() or self.lib.me_set_state(self.h, c_void_p(psi.data_ptr()), c_int64(self.N)))

    def get_state(self):
        out = self.torch.empty((self.n_orb, self.N), dtype=self.cdtype, device=self.device)
        self._check(self._pre() or self.lib.me_get_state(self.h, c_void_p(out.data_ptr()), c_int64(self.N)))
        return out

    def apply_H(self, psi):
        psi = self._orbitals(psi)
        out = self.torch.empty_like(psi)
        self._check(self._pre() or self.lib.me_apply_H(self.h, c_void_p(psi.data_ptr()), c_void_p(out.data_ptr()),
                                        c_int32(psi.shape[0]), c_int64(self.N)))
        return out

    def step(self, ctrl: Optional[float] = None, report: bool = False):
        c = c_double(ctrl) if ctrl is not None else None
        rep = StepReport() if report else None
        self._pre()
        st = self.lib.me_propagate_step(self.h, ctypes.byref(c) if c is not None else None,
                                        ctypes.byref(rep) if rep is not None else None)
        self._check(st)
        return rep.as_dict() if rep is not None else None

    def cp_begin(self, mu_cp: float, dt: float):
        """Start Car-Parrinello steps from the current state (zero orbital velocities)."""
        self._check(self._pre() or self.lib.me_cp_begin(self.h, c_double(mu_cp), c_double(dt)))

    def cp_step(self, report: bool = False):
        rep = StepReport() if report else None
        self._pre()
        self._check(self.lib.me_cp_step(self.h, ctypes.byref(rep) if rep is not None else None))
        return rep.as_dict() if rep is not None else None

    def report(self) -> dict:
        rep = StepReport()
        self._check(self._pre() or self.lib.me_report(self.h, ctypes.byref(rep)))
        return rep.as_dict()

    def sync(self):
        self._check(self._pre() or self.lib.me_sync(self.h))

    def density(self):
        out = self.torch.empty(self.N, dtype=self.torch.float64, device=self.device)
        self._check(self._pre() or self.lib.me_density(self.h, c_void_p(out.data_ptr())))
        return out

    def forces(self) -> np.ndarray:
        f = np.zeros((self.n_ions, 3))
        self._check(self._pre() or self.lib.me_forces(self.h, _dptr(f)))
        return f

    def ions(self):
        p = np.zeros((self.n_ions, 3))
        v = np.zeros((self.n_ions, 3))
        self._check(self._pre() or self.lib.me_get_ions(self.h, _dptr(p), _dptr(v)))
        return p, v

    def potential(self, which: int):
        out = self.torch.empty(self.N, dtype=self.torch.float64, device=self.device)
        self._check(self._pre() or self.lib.me_get_potential(self.h, c_int32(which), c_void_p(out.data_ptr())))
        return out

    def set_static_potential(self, dv):
        if dv is None:
            self._check(self._pre() or self.lib.me_set_static_potential(self.h, None))
            return
        dv = self.torch.as_tensor(dv, dtype=self.torch.float64).to(self.device).reshape(-1).contiguous()
        self._dv = dv
        self._check(self._pre() or self.lib.me_set_static_potential(self.h, c_void_p(dv.data_ptr())))

    # -------------------------------------------------------------- adjoint
    def checkpoint_size(self) -> int:
        out = c_size_t(0)
        self._check(self._pre() or self.lib.me_checkpoint_size(self.h, ctypes.byref(out)))
        return out.value

    def new_checkpoint(self):
        return self.torch.empty(self.checkpoint_size(), dtype=self.torch.uint8, device=self.device)

    def save_checkpoint(self, buf):
        self._check(self._pre() or self.lib.me_save_checkpoint(self.h, c_void_p(buf.data_ptr())))

    def load_checkpoint(self, buf):
        self._check(self._pre() or self.lib.me_load_checkpoint(self.h, c_void_p(buf.data_ptr())))

    def set_static_potential_coarse(self, coarse):
        if coarse is None:
            self._check(self._pre() or self.lib.me_set_static_potential_coarse(self.h, None, c_int32(1)))
            return
        c = self.torch.as_tensor(coarse, dtype=self.torch.float64).to(self.device).contiguous()
        self._coarse = c
        self._check(self._pre() or self.lib.me_set_static_potential_coarse(self.h, c_void_p(c.data_ptr()),
                                                            c_int32(c.shape[0])))

    def dipole(self) -> float:
        d = c_double(0)
        self._check(self._pre() or self.lib.me_dipole(self.h, ctypes.byref(d)))
        return d.value

    def adjoint_begin(self, rhobar=None):
        ptr = None
        if rhobar is not None:
            rhobar = self.torch.as_tensor(rhobar, dtype=self.torch.float64).to(self.device).contiguous()
            self._rhobar = rhobar
            ptr = c_void_p(rhobar.data_ptr())
        self._check(self._pre() or self.lib.me_adjoint_begin(self.h, ptr))

    def adjoint_step(self, ctrl: float) -> float:
        g = c_double(0)
        self._check(self._pre() or self.lib.me_adjoint_step(self.h, c_double(ctrl), ctypes.byref(g)))
        return g.value

    def adjoint_grad_v(self, m: Optional[int] = None):
        t = self.torch
        if m is None:
            out = t.empty(self.N, dtype=t.float64, device=self.device)
            self._check(self._pre() or self.lib.me_adjoint_grad_v(self.h, c_void_p(out.data_ptr()), None, c_int32(0)))
        else:
            out = t.empty((m, m, m), dtype=t.float64, device=self.device)
            self._check(self._pre() or self.lib.me_adjoint_grad_v(self.h, None, c_void_p(out.data_ptr()), c_int32(m)))
        return out

    def timing_enable(self, on: bool = True):
        self._check(self._pre() or self.lib.me_timing_enable(self.h, c_int32(1 if on else 0)))

    def timing_read(self, streams: int = 0):
        """(launches, total ms, algorithmic bytes) of the timed Horner stages:
        streams 2 the first stages, 3 the others, 0 all."""
        n = c_int64(0)
        ms = c_double(0)
        by = c_double(0)
        self._check(self._pre() or self.lib.me_timing_read_kind(self.h, c_int32(streams), ctypes.byref(n),
                                                               ctypes.byref(ms), ctypes.byref(by)))
        return n.value, ms.value, by.value


class Batch:
    """Several systems advanced together (persistent stencil launches, graph
    replay); device memory from torch, work on torch's current stream.
    ``systems[i]`` is a System view of system i, owned by the batch."""

    def __init__(self, params_list, keep=None, device="cuda:0"):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device(device)
        n = len(params_list)
        self._params = (Params * n)(*params_list)
        self._keep = keep
        size = c_size_t(0)
        st = self.lib.me_batch_workspace_size(self._params, c_int32(n), ctypes.byref(size))
        if st != ME_OK:
            raise ModehrError(st, self.lib.me_batch_last_error(None).decode())
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority): graphs cannot be captured
        # on the legacy default stream
        self.stream = torch.cuda.Stream(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        h = c_void_p()
        st = self.lib.me_init_batch(self._params, c_int32(n), c_void_p(self.workspace.data_ptr()), size,
                                    c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != ME_OK:
            raise ModehrError(st, self.lib.me_batch_last_error(None).decode())
        self.h = h
        self.systems = []
        for i in range(n):
            sh = c_void_p()
            self._check(self.lib.me_batch_system(self.h, c_int32(i), ctypes.byref(sh)))
            self.systems.append(System(params_list[i], device=device, handle=sh, stream=self.stream))

    def _check(self, st: int):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        if st != ME_OK:
            raise ModehrError(st, self.lib.me_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            for s in self.systems:
                s.close()
            self.lib.me_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def propagate(self, n_steps: int, use_graph: bool = True):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        self._check(self.lib.me_propagate_batch(self.h, c_int32(n_steps), c_int32(1 if use_graph else 0)))

    def tuning(self) -> dict:
        t = BatchTuning()
        self._check(self.lib.me_batch_get_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, block: int, wg_per_cu: int, zdiv: int = 1):
        t = BatchTuning(block, wg_per_cu, zdiv, 0.0)
        self._check(self.lib.me_batch_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, cache_path: Optional[str] = None) -> dict:
        t = BatchTuning()
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.me_batch_autotune(self.h, path, ctypes.byref(t)))
        return t.as_dict()

    def timing_enable(self, on: bool = True):
        self._check(self.lib.me_batch_timing_enable(self.h, c_int32(1 if on else 0)))

    def timing_read(self, streams: int = 0):
        """(launches, total ms, algorithmic bytes) of the timed stencil
        launches: streams 2 the first stages, 3 the others, 0 all."""
        n = c_int64(0)
        ms = c_double(0)
        by = c_double(0)
        self._check(self.lib.me_batch_timing_read_kind(self.h, c_int32(streams), ctypes.byref(n), ctypes.byref(ms),
                                                       ctypes.byref(by)))
        return n.value, ms.value, by.value


# ------------------------------------------------------------- toy model
TOY_SCHEMES = {"ehrenfest": 0, "cp": 1}


def toy_params(R0, M_R, K_R, G0, M_G, K_G) -> ToyParams:
    return ToyParams(R0, M_R, K_R, G0, M_G, K_G)


def toy_run(p: ToyParams, scheme: str, mu, substeps, window, n_samples: int, t_total: float,
            max_substeps: Optional[int] = None, samples: bool = True, device="cuda:0"):
    """me_toy_run over len(mu) trajectories (mu, substeps, window: sequences
    or tensors).  Returns {"d_R", "d_F", "samples" ([n_samples + 1, NV, n_traj],
    NV = 6 for Ehrenfest, 8 for CP, or None)} as device tensors, ordered on
    torch's current stream."""
    import torch
    lib = load()
    mu = torch.as_tensor(mu, dtype=torch.float64, device=device).contiguous()
    n = mu.numel()
    sub = torch.as_tensor(substeps, dtype=torch.int32, device=device).reshape(-1).expand(n).contiguous()
    win = torch.as_tensor(window, dtype=torch.int32, device=device).reshape(-1).expand(n).contiguous()
    if max_substeps is None:
        max_substeps = int(sub.max().item()) if n else 1
    d_R = torch.empty(n, dtype=torch.float64, device=device)
    d_F = torch.empty(n, dtype=torch.float64, device=device)
    nv = 8 if scheme == "cp" else 6
    S = torch.empty((n_samples + 1, nv, n), dtype=torch.float64, device=device) if samples else None
    stream = torch.cuda.current_stream(mu.device).cuda_stream
    st = lib.me_toy_run(ctypes.byref(p), c_int32(TOY_SCHEMES[scheme]), c_int32(n), c_int32(n_samples),
                        c_double(t_total), c_int32(max_substeps), c_void_p(mu.data_ptr()), c_void_p(sub.data_ptr()),
                        c_void_p(win.data_ptr()), c_void_p(S.data_ptr()) if S is not None else None,
                        c_void_p(d_R.data_ptr()), c_void_p(d_F.data_ptr()), c_void_p(stream))
    if st != ME_OK:
        raise ModehrError(st, lib.me_last_error(None).decode())
    return {"d_R": d_R, "d_F": d_F, "samples": S}


def toy_distance(samples, ref):
    """me_toy_distance: samples [n_samples + 1, NV, n_traj] (device), ref the
    reference trajectory of each; returns the distances (device tensor)."""
    import torch
    lib = load()
    n_samples = samples.shape[0] - 1
    n = samples.shape[2]
    ref = torch.as_tensor(ref, dtype=torch.int32, device=samples.device).reshape(-1).expand(n).contiguous()
    dist = torch.empty(n, dtype=torch.float64, device=samples.device)
    stream = torch.cuda.current_stream(samples.device).cuda_stream
    st = lib.me_toy_distance(c_int32(n), c_int32(n_samples), c_int32(samples.shape[1]), c_void_p(samples.data_ptr()),
                             c_void_p(ref.data_ptr()), c_void_p(dist.data_ptr()), c_void_p(stream))
    if st != ME_OK:
        raise ModehrError(st, lib.me_last_error(None).decode())
    return dist


# ------------------------------------------------------------- no allocation
def dipole_noalloc(rho, n, h: float, out):
    """me_dipole_noalloc: out[0] = h^3 sum (h*ix - L/2) rho for a device FP64
    density rho (n = (n_x, n_y, n_z), x fastest) into the device FP64 tensor
    out, on torch's current stream, without allocating or synchronising."""
    import torch
    lib = load()
    if rho.dtype != torch.float64 or out.dtype != torch.float64 or not rho.is_contiguous():
        raise ValueError("rho must be contiguous float64 and out float64")
    n3 = (c_int32 * 3)(*[int(v) for v in n])
    stream = torch.cuda.current_stream(rho.device).cuda_stream
    st = lib.me_dipole_noalloc(c_void_p(rho.data_ptr()), n3, c_double(h), c_void_p(out.data_ptr()),
                               c_void_p(stream))
    if st != ME_OK:
        raise ModehrError(st, lib.me_last_error(None).decode())
    return out
