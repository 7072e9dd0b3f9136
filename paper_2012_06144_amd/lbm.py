"""ctypes binding of ``liblbm.so`` (C ABI declared in include/lbm.h).

Argument marshalling only: every step of the solver runs in the HIP
library.  PyTorch provides device memory (the workspace and field tensors)
and the stream.  Importing this module loads the library and raises if it
is not built: there is no fallback.

Module-level functions carry the C names (``lbm_step(ctx, n)`` ...); the
:class:`Solver` class wraps them for tensors shaped (nz, ny, nx) /
(q, nz, ny, nx), x fastest.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "liblbm.so")

LBM_OK, LBM_EARG, LBM_EHIP, LBM_ESTATE, LBM_ENONFINITE, LBM_ESIZE = 0, -1, -2, -3, -4, -5
STORAGE = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}
DTYPE_F64, DTYPE_F32 = 0, 1

EXPORTS = [
    "lbm_velocity_set", "lbm_workspace_bytes", "lbm_create", "lbm_set_stream", "lbm_init_fields",
    "lbm_step", "lbm_step_straightforward", "lbm_step_timed", "lbm_step_timed_fused", "lbm_reduce_mass", "lbm_reduce_stats", "lbm_get_macroscopic",
    "lbm_set_macroscopic", "lbm_shift_equilibrium", "lbm_get_pdfs", "lbm_set_pdfs", "lbm_stream_copy", "lbm_steps_done",
    "lbm_state_bytes", "lbm_save_state", "lbm_restore_state", "lbm_destroy", "lbm_last_error",
]


class LbmParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls_y", C.c_int32),
        ("phi_L", C.c_double), ("phi_H", C.c_double), ("xi", C.c_double),
        ("mobility", C.c_double), ("sigma", C.c_double),
        ("rho_L", C.c_double), ("rho_H", C.c_double), ("tau_L", C.c_double), ("tau_H", C.c_double),
        ("body_accel", C.c_double * 3), ("buoyancy_rho_ref", C.c_double), ("normal_eps", C.c_double),
        ("storage", C.c_int32), ("density_literal", C.c_int32),
        ("lattice_phase", C.c_int32), ("lattice_hydro", C.c_int32), ("phase_mrt", C.c_int32),
    ]


class LbmStats(C.Structure):
    _fields_ = [
        ("mass", C.c_double), ("momentum", C.c_double * 3), ("gas_volume", C.c_double),
        ("centroid", C.c_double * 3), ("rise_velocity", C.c_double),
        ("interface_sum", C.c_double), ("grad_sum", C.c_double), ("xi_eff", C.c_double),
        ("max_speed", C.c_double),
    ]


class LbmError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise LbmError(f"HIP library not built: {LIB_PATH} is missing "
                       "(run paper_2012_06144_amd/build.py or __graft_entry__.build())")
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes the library bind to that runtime, so the
    # process has one HIP runtime and torch's device pointers and streams
    # are valid in the library.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "lbm_velocity_set": ([C.c_int32, vp, vp], C.c_int),
        "lbm_workspace_bytes": ([C.POINTER(LbmParams)], C.c_size_t),
        "lbm_create": ([C.POINTER(LbmParams), vp, C.c_size_t, vp, C.POINTER(vp)], C.c_int),
        "lbm_set_stream": ([vp, vp], C.c_int),
        "lbm_init_fields": ([vp, vp, vp, vp], C.c_int),
        "lbm_step": ([vp, C.c_int32], C.c_int),
        "lbm_step_straightforward": ([vp, C.c_int32], C.c_int),
        "lbm_step_timed": ([vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
        "lbm_step_timed_fused": ([vp, C.c_int32, C.POINTER(C.c_double)], C.c_int),
        "lbm_reduce_mass": ([vp, C.POINTER(C.c_double)], C.c_int),
        "lbm_reduce_stats": ([vp, C.POINTER(LbmStats)], C.c_int),
        "lbm_get_macroscopic": ([vp, C.c_int32, vp, vp, vp], C.c_int),
        "lbm_set_macroscopic": ([vp, C.c_int32, vp, vp, vp], C.c_int),
        "lbm_shift_equilibrium": ([vp, C.c_int32, vp, vp, vp], C.c_int),
        "lbm_get_pdfs": ([vp, vp, vp], C.c_int),
        "lbm_set_pdfs": ([vp, vp, vp, vp, vp], C.c_int),
        "lbm_stream_copy": ([vp, vp, C.c_size_t, vp], C.c_int),
        "lbm_steps_done": ([vp], C.c_int64),
        "lbm_state_bytes": ([vp], C.c_size_t),
        "lbm_save_state": ([vp, vp], C.c_int),
        "lbm_restore_state": ([vp, vp], C.c_int),
        "lbm_destroy": ([vp], None),
        "lbm_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


_lib = _load()


def _check(status: int, what: str):
    if status != LBM_OK:
        msg = _lib.lbm_last_error().decode(errors="replace")
        raise LbmError(f"{what} failed with status {status}: {msg}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ---- C names -------------------------------------------------------------------

def lbm_velocity_set(q: int):
    e = np.zeros(3 * q, dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    _check(_lib.lbm_velocity_set(q, e.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p)),
           "lbm_velocity_set")
    return e.reshape(q, 3), w


def lbm_workspace_bytes(params: LbmParams) -> int:
    n = _lib.lbm_workspace_bytes(C.byref(params))
    if n == 0:
        raise LbmError("invalid parameters: " + _lib.lbm_last_error().decode(errors="replace"))
    return int(n)


def lbm_create(params: LbmParams, workspace, nbytes: int, stream) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(_lib.lbm_create(C.byref(params), C.c_void_p(workspace), nbytes, C.c_void_p(stream),
                           C.byref(ctx)), "lbm_create")
    return ctx


def lbm_set_stream(ctx, stream):
    _check(_lib.lbm_set_stream(ctx, C.c_void_p(stream)), "lbm_set_stream")


def lbm_init_fields(ctx, phi, u, p_star):
    _check(_lib.lbm_init_fields(ctx, _ptr(phi), _ptr(u), _ptr(p_star)), "lbm_init_fields")


def lbm_step(ctx, n: int):
    _check(_lib.lbm_step(ctx, int(n)), "lbm_step")


def lbm_step_straightforward(ctx, n: int):
    _check(_lib.lbm_step_straightforward(ctx, int(n)), "lbm_step_straightforward")


def lbm_step_timed_fused(ctx, n: int) -> float:
    f = C.c_double()
    _check(_lib.lbm_step_timed_fused(ctx, int(n), C.byref(f)), "lbm_step_timed_fused")
    return f.value


def lbm_step_timed(ctx, n: int):
    """Runs n steps; returns (mean phase-sweep ms, mean hydro-sweep ms)."""
    a, b = C.c_double(), C.c_double()
    _check(_lib.lbm_step_timed(ctx, int(n), C.byref(a), C.byref(b)), "lbm_step_timed")
    return a.value, b.value


def lbm_reduce_mass(ctx) -> float:
    v = C.c_double()
    _check(_lib.lbm_reduce_mass(ctx, C.byref(v)), "lbm_reduce_mass")
    return v.value


def lbm_reduce_stats(ctx) -> dict:
    s = LbmStats()
    _check(_lib.lbm_reduce_stats(ctx, C.byref(s)), "lbm_reduce_stats")
    return {
        "mass": s.mass, "momentum": tuple(s.momentum), "gas_volume": s.gas_volume,
        "centroid": tuple(s.centroid), "rise_velocity": s.rise_velocity,
        "interface_sum": s.interface_sum, "grad_sum": s.grad_sum, "xi_eff": s.xi_eff,
        "max_speed": s.max_speed,
    }


def lbm_get_macroscopic(ctx, dtype: int, phi, u, p):
    _check(_lib.lbm_get_macroscopic(ctx, dtype, _ptr(phi), _ptr(u), _ptr(p)), "lbm_get_macroscopic")


def lbm_set_macroscopic(ctx, dtype: int, phi, u, p):
    _check(_lib.lbm_set_macroscopic(ctx, dtype, _ptr(phi), _ptr(u), _ptr(p)), "lbm_set_macroscopic")


def lbm_shift_equilibrium(ctx, dtype: int, phi, u, p):
    _check(_lib.lbm_shift_equilibrium(ctx, dtype, _ptr(phi), _ptr(u), _ptr(p)), "lbm_shift_equilibrium")


def lbm_get_pdfs(ctx, H, G):
    _check(_lib.lbm_get_pdfs(ctx, _ptr(H), _ptr(G)), "lbm_get_pdfs")


def lbm_set_pdfs(ctx, H, G, phi, u):
    _check(_lib.lbm_set_pdfs(ctx, _ptr(H), _ptr(G), _ptr(phi), _ptr(u)), "lbm_set_pdfs")


def lbm_stream_copy(src, dst, nbytes: int, stream):
    _check(_lib.lbm_stream_copy(_ptr(src), _ptr(dst), nbytes, C.c_void_p(stream)), "lbm_stream_copy")


def lbm_steps_done(ctx) -> int:
    return int(_lib.lbm_steps_done(ctx))


def lbm_state_bytes(ctx) -> int:
    return int(_lib.lbm_state_bytes(ctx))


def lbm_save_state(ctx, dst):
    _check(_lib.lbm_save_state(ctx, _ptr(dst)), "lbm_save_state")


def lbm_restore_state(ctx, src):
    _check(_lib.lbm_restore_state(ctx, _ptr(src)), "lbm_restore_state")


def lbm_destroy(ctx):
    _lib.lbm_destroy(ctx)


def lbm_last_error() -> str:
    return _lib.lbm_last_error().decode(errors="replace")


# ---- convenience wrapper ---------------------------------------------------------

def make_params(nx, ny, nz, walls_y=False, phi_L=0.0, phi_H=1.0, xi=4.0, mobility=0.02,
                sigma=1e-3, rho_L=1.0, rho_H=10.0, tau_L=1.0, tau_H=1.0, accel=(0.0, 0.0, 0.0),
                buoyancy_rho_ref=0.0, normal_eps=1e-12, density_literal=False, storage="f64",
                lattice_phase=15, lattice_hydro=27, phase_mrt=False) -> LbmParams:
    p = LbmParams()
    p.nx, p.ny, p.nz, p.walls_y = int(nx), int(ny), int(nz), int(bool(walls_y))
    p.phi_L, p.phi_H, p.xi, p.mobility, p.sigma = phi_L, phi_H, xi, mobility, sigma
    p.rho_L, p.rho_H, p.tau_L, p.tau_H = rho_L, rho_H, tau_L, tau_H
    for a in range(3):
        p.body_accel[a] = float(accel[a])
    p.buoyancy_rho_ref = float(buoyancy_rho_ref)
    p.normal_eps = normal_eps
    p.density_literal = int(bool(density_literal))
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.lattice_phase, p.lattice_hydro = int(lattice_phase), int(lattice_hydro)
    p.phase_mrt = int(bool(phase_mrt))
    return p


class Solver:
    """One solver context on one device, with a torch-allocated workspace."""

    def __init__(self, physics: dict, storage: str = "f64", device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.physics = dict(physics)
        self.storage = storage
        self.params = make_params(storage=storage, **physics)
        self.qp, self.qh = self.params.lattice_phase, self.params.lattice_hydro
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.n = self.params.nx * self.params.ny * self.params.nz
        self.nbytes = lbm_workspace_bytes(self.params)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = lbm_create(self.params, self.workspace.data_ptr(), self.nbytes,
                              self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev64(self, a, shape):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        return a.to(device=self.device, dtype=t.float64).reshape(shape).contiguous()

    def init_fields(self, phi, u, p_star):
        phi_d = self._dev64(phi, self.shape)
        u_d = self._dev64(u, (3,) + self.shape)
        p_d = self._dev64(p_star, self.shape)
        lbm_init_fields(self.ctx, phi_d, u_d, p_d)
        self.stream.synchronize()

    def step(self, n: int = 1):
        lbm_step(self.ctx, n)

    def step_straightforward(self, n: int = 1):
        """n steps of the straightforward six-kernel algorithm (FP64, FP32)."""
        lbm_step_straightforward(self.ctx, n)

    def step_timed(self, n: int):
        return lbm_step_timed(self.ctx, n)

    def step_timed_fused(self, n: int) -> float:
        """Mean fused-kernel time (ms) over n steps run as lbm_step runs them."""
        return lbm_step_timed_fused(self.ctx, n)

    def reduce_mass(self) -> float:
        return lbm_reduce_mass(self.ctx)

    def stats(self) -> dict:
        return lbm_reduce_stats(self.ctx)

    def macroscopic(self, dtype=None, out=None):
        """(phi, u, p) as new tensors, or as views of `out`, a (5, nz, ny, nx)
        tensor holding phi, u_x, u_y, u_z, p as consecutive planes."""
        t = self.torch
        if out is not None:
            assert out.shape == (5,) + self.shape and out.is_contiguous()
            dtype = out.dtype
            phi, u, p = out[0], out[1:4], out[4]
        else:
            dtype = dtype or t.float64
            phi = t.empty(self.shape, dtype=dtype, device=self.device)
            u = t.empty((3,) + self.shape, dtype=dtype, device=self.device)
            p = t.empty(self.shape, dtype=dtype, device=self.device)
        code = DTYPE_F64 if dtype == t.float64 else DTYPE_F32
        lbm_get_macroscopic(self.ctx, code, phi, u, p)
        return phi, u, p

    def set_macroscopic(self, phi, u, p, keep_neq=False):
        """Equilibrium state of the fields (lbm_set_macroscopic), or with
        keep_neq the current state moved to them with every population's
        non-equilibrium part kept (lbm_shift_equilibrium)."""
        t = self.torch
        dtype = phi.dtype if hasattr(phi, "dtype") and phi.dtype in (t.float32, t.float64) else t.float64
        code = DTYPE_F64 if dtype == t.float64 else DTYPE_F32
        fn = lbm_shift_equilibrium if keep_neq else lbm_set_macroscopic
        fn(self.ctx, code, phi.contiguous(), u.contiguous(), p.contiguous())

    def pdfs(self):
        t = self.torch
        H = t.empty((self.qp,) + self.shape, dtype=t.float64, device=self.device)
        G = t.empty((self.qh,) + self.shape, dtype=t.float64, device=self.device)
        lbm_get_pdfs(self.ctx, H, G)
        return H, G

    def state(self):
        """Canonical state (H, G, phi, u) as float64 numpy arrays."""
        H, G = self.pdfs()
        phi, u, _ = self.macroscopic(self.torch.float64)
        self.stream.synchronize()
        return H.cpu().numpy(), G.cpu().numpy(), phi.cpu().numpy(), u.cpu().numpy()

    def set_state(self, H, G, phi, u):
        lbm_set_pdfs(self.ctx, self._dev64(H, (self.qp,) + self.shape), self._dev64(G, (self.qh,) + self.shape),
                     self._dev64(phi, self.shape), self._dev64(u, (3,) + self.shape))
        self.stream.synchronize()

    def new_state_buffer(self):
        """A device buffer for save_state / restore_state."""
        return self.torch.empty(lbm_state_bytes(self.ctx), dtype=self.torch.uint8, device=self.device)

    def save_state(self, buf):
        lbm_save_state(self.ctx, buf)

    def restore_state(self, buf):
        lbm_restore_state(self.ctx, buf)

    def pressure(self):
        _, _, p = self.macroscopic(self.torch.float64)
        self.stream.synchronize()
        return p.cpu().numpy()
