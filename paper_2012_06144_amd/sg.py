"""ctypes binding of the surrogate-network kernels (C ABI in include/sg.h).

Argument marshalling only; tensors are torch device tensors (BF16 activations
channels-last (N, D, H, W, C), BF16 weights (27, C_out, C_in), FP32 bias,
gradients and optimiser state).  The kernels live in the same ``liblbm.so``
as the solver; importing raises if it is not built.
"""
from __future__ import annotations

import ctypes as C

from .lbm import LIB_PATH, LbmError, _lib as _L  # noqa: F401  (loads the library)

EXPORTS = [
    "sg_conv3d_fwd", "sg_conv3d_fwd_up_cat", "sg_weight_mirror", "sg_conv3d_bwd_data", "sg_conv3d_bwd_data_noalloc", "sg_bwd_weight_workspace", "sg_conv3d_bwd_weight",
    "sg_leaky_bwd", "sg_pool2_fwd", "sg_pool2_bwd", "sg_up2_fwd", "sg_up2_bwd", "sg_concat",
    "sg_split", "sg_mse", "sg_adam", "sg_to_bf16", "sg_to_f32", "sg_add", "sg_fields_to_input",
    "sg_state_to_input", "sg_make_target", "sg_apply_prediction", "sg_advect_phase", "sg_projective_step",
    "sg_pair_to_input", "sg_channel_moments", "sg_shift_boxes", "sg_box_moments",
    "sg_mass_project", "sg_last_error",
]

_vp, _i, _i64, _f, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
_SIG = {
    "sg_conv3d_fwd": [_vp, _i, _i, _i, _i, _i, _vp, _vp, _i, _i, _i, _f, _vp, _i, _vp],
    "sg_conv3d_fwd_up_cat": [_vp, _i, _vp, _i, _i, _i, _i, _i, _vp, _vp, _i, _i, _i, _f, _vp, _i, _vp],
    "sg_weight_mirror": [_vp, _i, _i, _vp, _vp],
    "sg_conv3d_bwd_data": [_vp, _i, _i, _i, _i, _i, _vp, _i, _vp, _vp, _sz, _vp],
    "sg_conv3d_bwd_data_noalloc": [_vp, _i, _i, _i, _i, _i, _vp, _i, _vp, _vp],
    "sg_bwd_weight_workspace": [_i, _i, _i, _i, _i, _i],
    "sg_conv3d_bwd_weight": [_vp, _vp, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp, _sz, _vp],
    "sg_leaky_bwd": [_vp, _vp, _vp, _sz, _f, _vp],
    "sg_pool2_fwd": [_vp, _i, _i, _i, _i, _i, _vp, _vp],
    "sg_pool2_bwd": [_vp, _i, _i, _i, _i, _i, _vp, _vp],
    "sg_up2_fwd": [_vp, _i, _i, _i, _i, _i, _vp, _vp],
    "sg_up2_bwd": [_vp, _i, _i, _i, _i, _i, _vp, _vp],
    "sg_concat": [_vp, _i, _vp, _i, _i64, _vp, _vp],
    "sg_split": [_vp, _i, _i, _i64, _vp, _vp, _vp],
    "sg_mse": [_vp, _vp, _i64, _vp, _vp, _vp, _vp],
    "sg_adam": [_vp, _vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, _i, _vp],
    "sg_to_bf16": [_vp, _vp, _i64, _vp],
    "sg_to_f32": [_vp, _vp, _i64, _vp],
    "sg_add": [_vp, _vp, _vp, _i64, _vp],
    "sg_fields_to_input": [_vp, _vp, _vp, _i, _i, _i, _vp, _vp, _i, _vp, _vp, _vp],
    "sg_state_to_input": [_vp, _i64, _vp, _i, _vp, _vp],
    "sg_make_target": [_vp, _vp, _i64, _vp, _i, _vp, _vp],
    "sg_apply_prediction": [_vp, _i, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp, _i, _f, _f, _i, _vp],
    "sg_advect_phase": [_vp, _i64, _i, _i, _i, _f, _vp, _vp],
    "sg_projective_step": [_vp, _vp, _i64, _i64, _i64, _f, _f, _f, _i, _i, _i, _vp, _vp],
    "sg_pair_to_input": [_vp, _vp, _i64, _vp, _vp, _i, _vp, _vp],
    "sg_channel_moments": [_vp, _i64, _i, _vp, _vp, _vp],
    "sg_shift_boxes": [_vp, _i64, _i, _i, _i, _vp, _vp, _vp],
    "sg_box_moments": [_vp, _i64, _i, _i, _i, _f, _f, _vp, _vp],
    "sg_mass_project": [_vp, _i, _i, _i, _i, C.c_double, _f, _f, _vp, _vp],
    "sg_last_error": [],
}
for _name, _args in _SIG.items():
    _fn = getattr(_L, _name)
    _fn.argtypes = _args
    _fn.restype = C.c_char_p if _name == "sg_last_error" else (
        C.c_size_t if _name == "sg_bwd_weight_workspace" else C.c_int)


class SgError(RuntimeError):
    pass


def _check(status, what):
    if status != 0:
        raise SgError(f"{what} failed with status {status}: "
                      f"{_L.sg_last_error().decode(errors='replace')}")


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


def sg_conv3d_fwd(x, wt, bias, c_out, n_store, act, slope, y, y_f32, stream=None):
    n, d, h, w, c_in = x.shape
    _check(_L.sg_conv3d_fwd(_p(x), n, d, h, w, c_in, _p(wt), _p(bias), c_out, n_store, int(act),
                            float(slope), _p(y), int(y_f32), _stream(stream)), "sg_conv3d_fwd")


def sg_conv3d_fwd_up_cat(xa, xb, wt, bias, c_out, n_store, act, slope, y, y_f32, stream=None):
    """sg_conv3d_fwd of [up2(xa), xb] along the channels: xa (N, D/2, H/2, W/2, ca), xb (N, D, H, W, cb)."""
    n, d, h, w, cb = xb.shape
    ca = xa.shape[-1]
    assert tuple(xa.shape[:4]) == (n, d // 2, h // 2, w // 2)
    _check(_L.sg_conv3d_fwd_up_cat(_p(xa), ca, _p(xb), cb, n, d, h, w, _p(wt), _p(bias), c_out, n_store, int(act),
                                   float(slope), _p(y), int(y_f32), _stream(stream)), "sg_conv3d_fwd_up_cat")


def sg_weight_mirror(wt, wm, stream=None):
    _, c_out, c_in = wt.shape
    _check(_L.sg_weight_mirror(_p(wt), c_out, c_in, _p(wm), _stream(stream)), "sg_weight_mirror")


def sg_conv3d_bwd_data(dy, wt, dx, wm, stream=None):
    """dx (N, D, H, W, c_in) from dy (N, D, H, W, c_out) and wt (27, c_out, c_in);
    wm is a BF16 workspace of 27 c_in c_out elements."""
    n, d, h, w, c_out = dy.shape
    c_in = wt.shape[2]
    _check(_L.sg_conv3d_bwd_data(_p(dy), n, d, h, w, c_out, _p(wt), c_in, _p(dx), _p(wm),
                                 wm.numel() * wm.element_size(), _stream(stream)), "sg_conv3d_bwd_data")


def sg_conv3d_bwd_data_noalloc(dy, wt, dx, stream=None):
    """sg_conv3d_bwd_data with the library's fixed device array in place of
    the workspace (27 c_in c_out BF16 weights, at most 4 MiB)."""
    n, d, h, w, c_out = dy.shape
    c_in = wt.shape[2]
    _check(_L.sg_conv3d_bwd_data_noalloc(_p(dy), n, d, h, w, c_out, _p(wt), c_in, _p(dx), _stream(stream)),
           "sg_conv3d_bwd_data_noalloc")


def sg_bwd_weight_workspace(n, d, h, w, c_in, c_out) -> int:
    return int(_L.sg_bwd_weight_workspace(n, d, h, w, c_in, c_out))


def sg_conv3d_bwd_weight(x, dy, dw, db, workspace, stream=None):
    n, d, h, w, c_in = x.shape
    c_out = dy.shape[-1]
    _check(_L.sg_conv3d_bwd_weight(_p(x), _p(dy), n, d, h, w, c_in, c_out, _p(dw), _p(db),
                                   _p(workspace), workspace.numel() * workspace.element_size(),
                                   _stream(stream)), "sg_conv3d_bwd_weight")


def sg_leaky_bwd(y, dy, dpre, slope, stream=None):
    _check(_L.sg_leaky_bwd(_p(y), _p(dy), _p(dpre), y.numel(), float(slope), _stream(stream)), "sg_leaky_bwd")


def sg_pool2_fwd(x, y, stream=None):
    n, d, h, w, c = x.shape
    _check(_L.sg_pool2_fwd(_p(x), n, d, h, w, c, _p(y), _stream(stream)), "sg_pool2_fwd")


def sg_pool2_bwd(dy, dx, stream=None):
    n, d, h, w, c = dx.shape
    _check(_L.sg_pool2_bwd(_p(dy), n, d, h, w, c, _p(dx), _stream(stream)), "sg_pool2_bwd")


def sg_up2_fwd(x, y, stream=None):
    n, d, h, w, c = x.shape
    _check(_L.sg_up2_fwd(_p(x), n, d, h, w, c, _p(y), _stream(stream)), "sg_up2_fwd")


def sg_up2_bwd(dy, dx, stream=None):
    n, d, h, w, c = dx.shape
    _check(_L.sg_up2_bwd(_p(dy), n, d, h, w, c, _p(dx), _stream(stream)), "sg_up2_bwd")


def sg_concat(a, b, y, stream=None):
    ca, cb = a.shape[-1], b.shape[-1]
    v = a.numel() // ca
    _check(_L.sg_concat(_p(a), ca, _p(b), cb, v, _p(y), _stream(stream)), "sg_concat")


def sg_split(y, ca, cb, a, b, stream=None):
    v = y.numel() // (ca + cb)
    _check(_L.sg_split(_p(y), ca, cb, v, _p(a), _p(b), _stream(stream)), "sg_split")


def sg_mse(pred, target, loss, grad, scratch, stream=None):
    _check(_L.sg_mse(_p(pred), _p(target), pred.numel(), _p(loss), _p(grad), _p(scratch), _stream(stream)),
           "sg_mse")


def sg_adam(p, g, m, v, wt, lr, beta1, beta2, eps, step, stream=None):
    _check(_L.sg_adam(_p(p), _p(g), _p(m), _p(v), _p(wt), p.numel(), float(lr), float(beta1), float(beta2),
                      float(eps), int(step), _stream(stream)), "sg_adam")


def sg_to_bf16(x, y, stream=None):
    _check(_L.sg_to_bf16(_p(x), _p(y), x.numel(), _stream(stream)), "sg_to_bf16")


def sg_to_f32(x, y, stream=None):
    _check(_L.sg_to_f32(_p(x), _p(y), x.numel(), _stream(stream)), "sg_to_f32")


def sg_add(a, b, y, stream=None):
    _check(_L.sg_add(_p(a), _p(b), _p(y), a.numel(), _stream(stream)), "sg_add")


def _box(box):
    arr = (C.c_int32 * 6)(*[int(v) for v in box])
    return arr


def _f5(vals):
    return (C.c_float * 5)(*[float(v) for v in vals])


def sg_fields_to_input(phi, u, p, nx, ny, nz, box, scale_in, c_in, x, state=None, stream=None):
    _check(_L.sg_fields_to_input(_p(phi), _p(u), _p(p), nx, ny, nz, _box(box), _f5(scale_in), c_in, _p(x),
                                 _p(state), _stream(stream)), "sg_fields_to_input")


def sg_state_to_input(state, scale_in, c_in, x, stream=None):
    v = state.numel() // 5
    _check(_L.sg_state_to_input(_p(state), v, _f5(scale_in), c_in, _p(x), _stream(stream)), "sg_state_to_input")


def sg_make_target(s0, s1, scale_out, c_out, target, stream=None):
    v = s0.numel() // 5
    _check(_L.sg_make_target(_p(s0), _p(s1), v, _f5(scale_out), c_out, _p(target), _stream(stream)),
           "sg_make_target")


SG_APPLY_U_BY_PHASE = 1
SG_APPLY_PHI_AT_INTERFACE = 2
SG_APPLY_NO_CLIP = 4


def sg_apply_prediction(out, c_out, scale_out, phi, u, p, nx, ny, nz, box, walls_y, phi_min, phi_max,
                        base=None, u_by_phase=False, phi_at_interface=False, clip=True, stream=None):
    flags = ((SG_APPLY_U_BY_PHASE if u_by_phase else 0) | (SG_APPLY_PHI_AT_INTERFACE if phi_at_interface else 0)
             | (0 if clip else SG_APPLY_NO_CLIP))
    _check(_L.sg_apply_prediction(_p(out), c_out, _f5(scale_out), _p(base), _p(phi), _p(u), _p(p), nx, ny, nz,
                                  _box(box), int(walls_y), float(phi_min), float(phi_max), flags,
                                  _stream(stream)),
           "sg_apply_prediction")


def sg_advect_phase(state, count, bx, by, bz, K, out, stream=None):
    _check(_L.sg_advect_phase(_p(state), int(count), bx, by, bz, float(K), _p(out), _stream(stream)),
           "sg_advect_phase")


def sg_projective_step(s, s_prev, n, cs, vs, ratio, phi_lo, phi_hi, u_by_phase, phi_step, p_step, out, stream=None):
    _check(_L.sg_projective_step(_p(s), _p(s_prev), int(n), int(cs), int(vs), float(ratio), float(phi_lo),
                                 float(phi_hi), int(u_by_phase), int(phi_step), int(p_step), _p(out),
                                 _stream(stream)),
           "sg_projective_step")


def sg_pair_to_input(state, state_prev, scale_in, trend_scale, c_in, x, stream=None):
    v = state.numel() // 5
    _check(_L.sg_pair_to_input(_p(state), _p(state_prev), v, _f5(scale_in), _f5(trend_scale), c_in, _p(x),
                               _stream(stream)), "sg_pair_to_input")


def sg_channel_moments(a, rows, c, out, scratch, stream=None):
    _check(_L.sg_channel_moments(_p(a), int(rows), int(c), _p(out), _p(scratch), _stream(stream)),
           "sg_channel_moments")


def sg_shift_boxes(state, count, bx, by, bz, shift, out, stream=None):
    _check(_L.sg_shift_boxes(_p(state), int(count), bx, by, bz, _p(shift), _p(out), _stream(stream)),
           "sg_shift_boxes")


def sg_box_moments(state, count, bx, by, bz, phi_heavy, phi_light, out, stream=None):
    _check(_L.sg_box_moments(_p(state), int(count), bx, by, bz, float(phi_heavy), float(phi_light), _p(out),
                             _stream(stream)), "sg_box_moments")


def sg_mass_project(phi, walls_y, target_mass, phi_min, phi_max, scratch, stream=None):
    """phi: FP32 field shaped (nz, ny, nx)."""
    nz, ny, nx = phi.shape
    _check(_L.sg_mass_project(_p(phi), nx, ny, nz, int(bool(walls_y)), float(target_mass), float(phi_min),
                              float(phi_max), _p(scratch), _stream(stream)), "sg_mass_project")


def sg_last_error() -> str:
    return _L.sg_last_error().decode(errors="replace")
