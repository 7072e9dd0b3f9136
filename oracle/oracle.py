"""ctypes wrapper of the FP64 CPU oracle (``liblbm_oracle.so``).

TEST INFRASTRUCTURE ONLY: this module is for the tests, the smoke check and
the CPU-baseline leg of the benchmark.  The GPU library never imports it and
it never imports the GPU library.

Fields are numpy float64 arrays in x-fastest order: a scalar field has shape
(nz, ny, nx), a vector or PDF field (q, nz, ny, nx).  The canonical state is
H (post-collision phase-field PDFs, not yet streamed), G (pre-collision
hydrodynamic PDFs, already streamed), phi (latest phase field) and u.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")

_lib = None


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls_y", C.c_int32),
        ("phi_L", C.c_double), ("phi_H", C.c_double), ("xi", C.c_double),
        ("mobility", C.c_double), ("sigma", C.c_double),
        ("rho_L", C.c_double), ("rho_H", C.c_double),
        ("tau_L", C.c_double), ("tau_H", C.c_double),
        ("accel", C.c_double * 3), ("rho_ref", C.c_double), ("normal_eps", C.c_double),
        ("density_literal", C.c_int32),
        ("lattice_phase", C.c_int32), ("lattice_hydro", C.c_int32), ("phase_mrt", C.c_int32),
    ]


class OrcStats(C.Structure):
    _fields_ = [
        ("mass", C.c_double), ("momentum", C.c_double * 3), ("gas_volume", C.c_double),
        ("centroid", C.c_double * 3), ("rise_velocity", C.c_double),
        ("interface_sum", C.c_double), ("grad_sum", C.c_double),
        ("xi_eff", C.c_double), ("max_speed", C.c_double),
    ]


_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    """Load the oracle library, building it with gcc if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    L = C.CDLL(LIB_PATH)
    L.orc_velocity_set.argtypes = [C.c_int32, _I, _D]
    L.orc_velocity_set.restype = C.c_int
    L.orc_gamma.argtypes = [C.c_int32, _D, _D]
    L.orc_hydro_equilibrium.argtypes = [C.c_double, _D, _D]
    L.orc_phase_forcing.argtypes = [C.c_double, _D, _D]
    L.orc_moment_matrix.argtypes = [_D, _D, _I]
    L.orc_moment_matrix.restype = C.c_int
    L.orc_viscous_bracket.argtypes = [_D, C.c_double, _D, _D]
    L.orc_viscous_bracket.restype = C.c_int
    L.orc_mrt_collide.argtypes = [_D, C.c_double, _D, _D, C.c_double, C.c_double, _D]
    L.orc_mrt_collide.restype = C.c_int
    L.orc_moment_matrix_q.argtypes = [C.c_int32, _D, _D, _D, _D, _I, _I]
    L.orc_moment_matrix_q.restype = C.c_int
    L.orc_hydro_equilibrium_q.argtypes = [C.c_int32, C.c_double, _D, _D]
    L.orc_hydro_equilibrium_q.restype = C.c_int
    L.orc_mrt_collide_q.argtypes = [C.c_int32, _D, C.c_double, _D, _D, C.c_double, C.c_double, _D]
    L.orc_mrt_collide_q.restype = C.c_int
    L.orc_viscous_bracket_q.argtypes = [C.c_int32, _D, C.c_double, _D, _D]
    L.orc_viscous_bracket_q.restype = C.c_int
    L.orc_phase_mrt_collide_q.argtypes = [C.c_int32, _D, _D, _D, C.c_double, _D]
    L.orc_phase_mrt_collide_q.restype = C.c_int
    L.orc_stencil.argtypes = [C.POINTER(OrcParams), _D, C.c_int32, C.c_int32, C.c_int32,
                              C.c_int32, _D, C.POINTER(C.c_double)]
    L.orc_create.argtypes = [C.POINTER(OrcParams)]
    L.orc_create.restype = C.c_void_p
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_init.argtypes = [C.c_void_p, _D, _D, _D]
    L.orc_step.argtypes = [C.c_void_p, C.c_int32]
    L.orc_step_naive.argtypes = [C.c_void_p, C.c_int32]
    L.orc_get_state.argtypes = [C.c_void_p] + [C.c_void_p] * 4
    L.orc_set_state.argtypes = [C.c_void_p] + [C.c_void_p] * 4
    L.orc_pressure.argtypes = [C.c_void_p, _D]
    L.orc_init_pressure.argtypes = [C.c_void_p, _D, _D, _D]
    L.orc_shift_equilibrium.argtypes = [C.c_void_p, _D, _D, _D]
    L.orc_stats_compute.argtypes = [C.c_void_p, C.POINTER(OrcStats)]
    L.orc_num_threads.argtypes = []
    L.orc_num_threads.restype = C.c_int
    L.orc_num_cells.argtypes = [C.c_void_p]
    L.orc_num_cells.restype = C.c_int64
    _lib = L
    return L


@dataclass
class Params:
    """Physical and grid parameters, in lattice units (dx = dt = 1)."""
    nx: int
    ny: int
    nz: int
    walls_y: bool = False
    phi_L: float = 0.0
    phi_H: float = 1.0
    xi: float = 4.0
    mobility: float = 0.02
    sigma: float = 1e-3
    rho_L: float = 1.0
    rho_H: float = 10.0
    tau_L: float = 1.0
    tau_H: float = 1.0
    accel: tuple = (0.0, 0.0, 0.0)
    buoyancy_rho_ref: float = 0.0
    normal_eps: float = 1e-12
    density_literal: bool = False
    lattice_phase: int = 15      # velocity set of the phase-field step (15, 19, 27)
    lattice_hydro: int = 27      # velocity set of the hydrodynamic step (27, 19, 15)
    phase_mrt: bool = False      # raw-moment MRT phase-field collision instead of SRT

    def to_c(self) -> OrcParams:
        p = OrcParams()
        p.nx, p.ny, p.nz, p.walls_y = self.nx, self.ny, self.nz, int(bool(self.walls_y))
        p.phi_L, p.phi_H, p.xi = self.phi_L, self.phi_H, self.xi
        p.mobility, p.sigma = self.mobility, self.sigma
        p.rho_L, p.rho_H, p.tau_L, p.tau_H = self.rho_L, self.rho_H, self.tau_L, self.tau_H
        for a in range(3):
            p.accel[a] = self.accel[a]
        p.rho_ref = self.buoyancy_rho_ref
        p.normal_eps = self.normal_eps
        p.density_literal = int(bool(self.density_literal))
        p.lattice_phase, p.lattice_hydro = int(self.lattice_phase), int(self.lattice_hydro)
        p.phase_mrt = int(bool(self.phase_mrt))
        return p


def velocity_set(q: int):
    e = np.zeros(3 * q, dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    if lib().orc_velocity_set(q, e, w) != 0:
        raise ValueError(f"no velocity set with q={q}")
    return e.reshape(q, 3), w


def num_threads() -> int:
    """OpenMP threads the oracle's cell loops use."""
    return int(lib().orc_num_threads())


def gamma(q: int, u) -> np.ndarray:
    out = np.zeros(q)
    lib().orc_gamma(q, np.ascontiguousarray(u, dtype=np.float64), out)
    return out


def hydro_equilibrium(pstar: float, u) -> np.ndarray:
    out = np.zeros(27)
    lib().orc_hydro_equilibrium(pstar, np.ascontiguousarray(u, dtype=np.float64), out)
    return out


def phase_forcing(theta: float, n) -> np.ndarray:
    out = np.zeros(15)
    lib().orc_phase_forcing(theta, np.ascontiguousarray(n, dtype=np.float64), out)
    return out


def moment_matrix():
    M = np.zeros(27 * 27)
    Mi = np.zeros(27 * 27)
    deg = np.zeros(27, dtype=np.int32)
    if lib().orc_moment_matrix(M, Mi, deg) != 0:
        raise RuntimeError("moment matrix construction failed")
    return M.reshape(27, 27), Mi.reshape(27, 27), deg


def viscous_bracket(g, s_nu: float, u) -> np.ndarray:
    V = np.zeros(9)
    lib().orc_viscous_bracket(np.ascontiguousarray(g, dtype=np.float64), s_nu,
                              np.ascontiguousarray(u, dtype=np.float64), V)
    return V.reshape(3, 3)


def mrt_collide(g, pstar: float, u, F, rho: float, s_nu: float) -> np.ndarray:
    out = np.zeros(27)
    lib().orc_mrt_collide(np.ascontiguousarray(g, dtype=np.float64), pstar,
                          np.ascontiguousarray(u, dtype=np.float64),
                          np.ascontiguousarray(F, dtype=np.float64), rho, s_nu, out)
    return out


def moment_matrix_q(q: int):
    """Weighted-orthogonal moment matrix M of the q-velocity set, its inverse,
    the raw monomial matrix R and its inverse, the degree and the exponents
    (a, b, c) of the monomial of each row."""
    M, Mi, R, Ri = (np.zeros(q * q) for _ in range(4))
    deg = np.zeros(q, dtype=np.int32)
    expo = np.zeros(3 * q, dtype=np.int32)
    if lib().orc_moment_matrix_q(q, M, Mi, R, Ri, deg, expo) != 0:
        raise RuntimeError(f"moment matrices of D3Q{q} failed")
    return M.reshape(q, q), Mi.reshape(q, q), R.reshape(q, q), Ri.reshape(q, q), deg, expo.reshape(q, 3)


def hydro_equilibrium_q(q: int, pstar: float, u) -> np.ndarray:
    out = np.zeros(q)
    if lib().orc_hydro_equilibrium_q(q, pstar, np.ascontiguousarray(u, dtype=np.float64), out) != 0:
        raise ValueError(q)
    return out


def mrt_collide_q(q: int, g, pstar: float, u, F, rho: float, s_nu: float) -> np.ndarray:
    out = np.zeros(q)
    if lib().orc_mrt_collide_q(q, np.ascontiguousarray(g, dtype=np.float64), pstar,
                               np.ascontiguousarray(u, dtype=np.float64),
                               np.ascontiguousarray(F, dtype=np.float64), rho, s_nu, out) != 0:
        raise ValueError(q)
    return out


def viscous_bracket_q(q: int, g, s_nu: float, u) -> np.ndarray:
    V = np.zeros(9)
    if lib().orc_viscous_bracket_q(q, np.ascontiguousarray(g, dtype=np.float64), s_nu,
                                   np.ascontiguousarray(u, dtype=np.float64), V) != 0:
        raise ValueError(q)
    return V.reshape(3, 3)


def phase_mrt_collide_q(q: int, h, heq, F, omega: float) -> np.ndarray:
    """Raw-moment MRT collision of the phase field (Sec. 3.1):
    h + R^-1 S R (heq - h - F/2) + F, first-order moments relaxed with omega."""
    out = np.zeros(q)
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in (h, heq, F)]
    if lib().orc_phase_mrt_collide_q(q, *args, omega, out) != 0:
        raise ValueError(q)
    return out


def stencil(params: Params, phi: np.ndarray, q: int, x: int, y: int, z: int):
    """Isotropic gradient and Laplacian of ``phi`` at (x, y, z) with the
    weights of the q-velocity set (and the wall mirror if walls_y)."""
    grad = np.zeros(3)
    lap = C.c_double(0.0)
    cp = params.to_c()
    lib().orc_stencil(C.byref(cp), np.ascontiguousarray(phi, dtype=np.float64), q, x, y, z,
                      grad, C.byref(lap))
    return grad, lap.value


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class Oracle:
    """A running oracle simulation."""

    def __init__(self, params: Params):
        self.params = params
        self._cp = params.to_c()
        self._h = lib().orc_create(C.byref(self._cp))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self.shape = (params.nz, params.ny, params.nx)
        self.n = params.nx * params.ny * params.nz
        self.qp, self.qh = int(params.lattice_phase), int(params.lattice_hydro)

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def init(self, phi, u, pstar):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.shape)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + self.shape)
        pstar = np.ascontiguousarray(pstar, dtype=np.float64).reshape(self.shape)
        lib().orc_init(self._h, phi, u, pstar)

    def init_pressure(self, phi, u, p):
        """Equilibrium state of (phi, u) and the pressure p, p* = p/(rho cs^2)."""
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.shape)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + self.shape)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(self.shape)
        lib().orc_init_pressure(self._h, phi, u, p)

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def step_straightforward(self, n: int = 1):
        """n steps of the straightforward algorithm (Alg. naiveAlgorithm,
        Sec. 4.2), read as a time-consistent scheme: the collisions take phi,
        its gradient and u of the new time."""
        lib().orc_step_naive(self._h, int(n))

    def state(self):
        H = np.zeros((self.qp,) + self.shape)
        G = np.zeros((self.qh,) + self.shape)
        phi = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().orc_get_state(self._h, _ptr(H), _ptr(G), _ptr(phi), _ptr(u))
        return H, G, phi, u

    def set_state(self, H, G, phi, u):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
                for a in (H, G, phi, u)]
        lib().orc_set_state(self._h, *[_ptr(a) for a in arrs])

    def shift_equilibrium(self, phi, u, p):
        """Moves the state to the fields (phi, u, pressure p) keeping every
        population's non-equilibrium part."""
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.shape)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + self.shape)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(self.shape)
        lib().orc_shift_equilibrium(self._h, phi, u, p)

    def pressure(self):
        p = np.zeros(self.shape)
        lib().orc_pressure(self._h, p)
        return p

    def stats(self) -> dict:
        s = OrcStats()
        lib().orc_stats_compute(self._h, C.byref(s))
        return {
            "mass": s.mass, "momentum": tuple(s.momentum), "gas_volume": s.gas_volume,
            "centroid": tuple(s.centroid), "rise_velocity": s.rise_velocity,
            "interface_sum": s.interface_sum, "grad_sum": s.grad_sum,
            "xi_eff": s.xi_eff, "max_speed": s.max_speed,
        }
