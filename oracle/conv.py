"""ctypes wrapper of the FP64 CPU oracle of the surrogate network's
operations (``conv_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Tensors are numpy float64 arrays, channels last:
activations (N, D, H, W, C); convolution weights (27, C_out, C_in) with tap
t = (a+1)*9 + (b+1)*3 + (c+1) for the offset (a, b, c) along (D, H, W).
"""
import ctypes as C

import numpy as np

from .oracle import lib as _lib_loader

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ready = False


def _lib():
    global _ready
    L = _lib_loader()
    if not _ready:
        i = C.c_int
        L.orc_conv3d_fwd.argtypes = [_D, i, i, i, i, i, _D, C.c_void_p, i, _D]
        L.orc_conv3d_bwd_data.argtypes = [_D, i, i, i, i, i, _D, i, _D]
        L.orc_conv3d_bwd_weight.argtypes = [_D, _D, i, i, i, i, i, i, _D, C.c_void_p]
        L.orc_pool2.argtypes = [_D, i, i, i, i, i, _D]
        L.orc_up2.argtypes = [_D, i, i, i, i, i, _D]
        L.orc_leaky.argtypes = [_D, C.c_size_t, C.c_double, _D]
        L.orc_mse.argtypes = [_D, _D, C.c_size_t, C.c_void_p]
        L.orc_mse.restype = C.c_double
        L.orc_adam.argtypes = [_D, _D, _D, _D, C.c_size_t, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_int]
        L.orc_advect_phase.argtypes = [_D, i, i, i, i, C.c_double, _D]
        L.orc_shift_boxes.argtypes = [_D, i, i, i, i, _D, _D]
        L.orc_box_moments.argtypes = [_D, i, i, i, i, C.c_double, C.c_double, _D]
        i64 = C.c_int64
        L.orc_projective_step.argtypes = [_D, _D, i64, i64, i64, C.c_double, C.c_double, C.c_double, i, i, i, _D]
        L.orc_mass_project.argtypes = [_D, i, i, i, i, C.c_double, C.c_double, C.c_double, _D]
        _ready = True
    return L


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def conv3d(x, w, b=None):
    x, w = _f(x), _f(w)
    N, D, H, W, Ci = x.shape
    Co = w.shape[1]
    assert w.shape == (27, Co, Ci)
    y = np.zeros((N, D, H, W, Co))
    bp = _f(b).ctypes.data_as(C.c_void_p) if b is not None else None
    bb = _f(b) if b is not None else None
    _lib().orc_conv3d_fwd(x, N, D, H, W, Ci, w, bb.ctypes.data_as(C.c_void_p) if bb is not None else None,
                          Co, y)
    return y


def conv3d_bwd_data(dy, w):
    dy, w = _f(dy), _f(w)
    N, D, H, W, Co = dy.shape
    Ci = w.shape[2]
    dx = np.zeros((N, D, H, W, Ci))
    _lib().orc_conv3d_bwd_data(dy, N, D, H, W, Co, w, Ci, dx)
    return dx


def conv3d_bwd_weight(x, dy):
    x, dy = _f(x), _f(dy)
    N, D, H, W, Ci = x.shape
    Co = dy.shape[-1]
    dw = np.zeros((27, Co, Ci))
    db = np.zeros(Co)
    _lib().orc_conv3d_bwd_weight(x, dy, N, D, H, W, Ci, Co, dw, db.ctypes.data_as(C.c_void_p))
    return dw, db


def pool2(x):
    x = _f(x)
    N, D, H, W, Cc = x.shape
    y = np.zeros((N, D // 2, H // 2, W // 2, Cc))
    _lib().orc_pool2(x, N, D, H, W, Cc, y)
    return y


def up2(x):
    x = _f(x)
    N, D, H, W, Cc = x.shape
    y = np.zeros((N, 2 * D, 2 * H, 2 * W, Cc))
    _lib().orc_up2(x, N, D, H, W, Cc, y)
    return y


def leaky(x, slope):
    x = _f(x)
    y = np.zeros_like(x)
    _lib().orc_leaky(x, x.size, slope, y)
    return y


def mse(pred, target, want_grad=True):
    pred, target = _f(pred), _f(target)
    g = np.zeros_like(pred) if want_grad else None
    v = _lib().orc_mse(pred, target, pred.size, g.ctypes.data_as(C.c_void_p) if g is not None else None)
    return v, g


def adam(p, g, m, v, lr, b1, b2, eps, t):
    """In-place Adam step on float64 arrays p, m, v."""
    assert p.dtype == np.float64 and p.flags.c_contiguous
    _lib().orc_adam(p, _f(g), m, v, p.size, lr, b1, b2, eps, int(t))


def advect_phase(state, K):
    """Semi-Lagrangian jump baseline on boxes of states shaped (count, bz, by,
    bx, 5): phi(x - K u(x)) by trilinear interpolation (departure point
    clamped to the box), u and p unchanged."""
    st = _f(state)
    if st.ndim == 4:
        st = st[None]
    n, bz, by, bx, c = st.shape
    assert c == 5
    out = np.zeros_like(st)
    _lib().orc_advect_phase(st, n, bx, by, bz, float(K), out)
    return out.reshape(np.shape(state))


def shift_boxes(state, shift):
    """Co-moving jump baseline on boxes of states shaped (count, bz, by, bx, 5):
    every channel translated by the box's displacement (dx, dy, dz), s(x - d)
    by trilinear interpolation with the departure point clamped to the box,
    then the velocity channels multiplied by f; shift shaped (count, 4) rows
    (dx, dy, dz, f), or (count, 3) for f = 1."""
    st = _f(state)
    if st.ndim == 4:
        st = st[None]
    n, bz, by, bx, c = st.shape
    assert c == 5
    d = _f(np.reshape(shift, (n, -1)))
    if d.shape[1] == 3:
        d = np.concatenate([d, np.ones((n, 1))], axis=1)
    d = _f(d)
    out = np.zeros_like(st)
    _lib().orc_shift_boxes(st, n, bx, by, bz, d, out)
    return out.reshape(np.shape(state))


def box_moments(state, phi_heavy, phi_light):
    """Gas-indicator moments of boxes of states (count, bz, by, bx, 5):
    rows of (sum chi, sum chi x, sum chi y, sum chi z, sum chi u_x,
    sum chi u_y, sum chi u_z, 0), chi = (phi_heavy - phi)/(phi_heavy -
    phi_light) clipped to [0, 1]."""
    st = _f(state)
    if st.ndim == 4:
        st = st[None]
    n, bz, by, bx, c = st.shape
    assert c == 5
    out = np.zeros((n, 8))
    _lib().orc_box_moments(st, n, bx, by, bz, float(phi_heavy), float(phi_light), out)
    return out


def projective_step(s, s_prev, ratio, phi_lo, phi_hi, u_by_phase=True, p_step=False, layout="last", phi_step=True):
    """Projective step s + ratio (s - s_prev) of field sets: layout "last"
    (..., 5) channels last, or "planar" (5, ...) one plane per channel;
    phi_step False carries phi over, p_step False the pressure."""
    a, b = _f(s), _f(s_prev)
    assert a.shape == b.shape
    if layout == "last":
        n = a.size // 5
        cs, vs = 1, 5
    else:
        n = a.size // 5
        cs, vs = n, 1
    out = np.zeros_like(a)
    _lib().orc_projective_step(a, b, n, cs, vs, float(ratio), float(phi_lo), float(phi_hi), int(u_by_phase),
                               int(phi_step), int(p_step), out)
    return out


def mass_project(phi, walls_y, target, phi_min, phi_max):
    """Mass projection of a phase field shaped (nz, ny, nx): phi + c 4q(1-q),
    q = clamp((phi - phi_min)/(phi_max - phi_min), 0, 1), c such that the sum
    over the fluid cells equals target; wall rows (walls_y) untouched."""
    a = _f(phi)
    nz, ny, nx = a.shape
    out = np.zeros_like(a)
    _lib().orc_mass_project(a, nx, ny, nz, int(bool(walls_y)), float(target), float(phi_min), float(phi_max), out)
    return out
