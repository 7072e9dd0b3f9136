"""Performance model of the coupled step (host arithmetic only).

Algorithmic bytes per cell update follow the paper's count (Section 5.1):
every PDF of a sweep is read and written once, the velocity is read by both
sweeps and written by the hydrodynamic one, and the phase field is read once
per sweep (the ideal case where the stencil neighbours come from cache) and
written by the phase-field sweep.  The paper's P_max = b_s / n_b turns bytes
into a lattice-update ceiling.
"""
from __future__ import annotations

PDF_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3


def field_bytes(storage: str) -> int:
    return 8 if storage == "f64" else 4


def bytes_per_cell(storage: str, qp: int = 15, qh: int = 27) -> dict:
    """Algorithmic HBM bytes per cell update of each sweep, for qp phase-field
    and qh hydrodynamic populations (D3Q15 and D3Q27 by default)."""
    p = PDF_BYTES[storage]
    r = field_bytes(storage)
    phase_r = qp * p + 3 * r + 1 * r      # h, u, phi (previous)
    phase_w = qp * p + 1 * r              # h, phi (new)
    hydro_r = qh * p + 3 * r + 1 * r      # g, u, phi (new)
    hydro_w = qh * p + 3 * r              # g, u
    return {
        "phase_read": phase_r, "phase_write": phase_w, "phase": phase_r + phase_w,
        "hydro_read": hydro_r, "hydro_write": hydro_w, "hydro": hydro_r + hydro_w,
        "total": phase_r + phase_w + hydro_r + hydro_w,
        # hydrodynamic sweep of one step fused with the phase sweep of the next:
        # the phase body takes u from registers and shares the phi stencil
        "fused": phase_r + phase_w + hydro_r + hydro_w - 3 * r - 1 * r,
        # the straightforward algorithm (six passes, Sec. 4.2): stream h
        # (15 + 15), phi = sum h (15 + 1), stream g (27 + 27), velocity update
        # (27 g + phi + 3 u read, 3 u written), collision of h (15 + phi + 3 u
        # read, 15 written), collision of g (27 + phi + 3 u read, 27 written)
        "straightforward": (2 * qp * p) + (qp * p + r) + (2 * qh * p) + (qh * p + 4 * r + 3 * r)
        + (qp * p + 4 * r + qp * p) + (qh * p + 4 * r + qh * p),
    }


def p_max_glups(b_s_gbs: float, n_b: float) -> float:
    """The paper's roofline P_max = b_s / n_b, in giga lattice updates/s."""
    return b_s_gbs / n_b


def balance(n_b: float, n_f: float, b_s_gbs: float, p_peak_tflops: float) -> dict:
    """Code balance B_c = n_b / n_f, machine balance B_m = b_s / p_peak and the
    light-speed factor l = min(1, B_m / B_c) (Section 5.1)."""
    B_c = n_b / n_f
    B_m = b_s_gbs / (p_peak_tflops * 1e3)
    return {"B_c": B_c, "B_m": B_m, "l": min(1.0, B_m / B_c)}


_KERNEL_SOURCES = ("csrc/lbm_kernels.hpp", "csrc/lbm_lattice.hpp", "csrc/lbm_api.hip", "csrc/lbm_sweeps_f32.hip",
                   "build.py")
_SURROGATE_SOURCES = ("csrc/sg_api.hip", "surrogate.py") + _KERNEL_SOURCES


def _hash_files(names) -> str:
    import hashlib
    import os
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in names:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    """Digest of the LBM kernel sources and their build script: a recorded
    measurement belongs to the current kernels only if its hash matches."""
    return _hash_files(_KERNEL_SOURCES)


def surrogate_source_hash() -> str:
    """Digest of the surrogate and LBM kernel sources, the jump driver and
    the build script (what a jump-study row depends on)."""
    return _hash_files(_SURROGATE_SOURCES)

