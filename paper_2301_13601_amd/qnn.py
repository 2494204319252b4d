"""Python binding of the surrogate kernels (C ABI in include/qla_nn.h).

Functions carry the C names and only marshal arguments (device pointers as
integers, the caller's stream); the arithmetic runs in libqla.so.
"""
from __future__ import annotations

import ctypes

from . import qla

QNN_ACT_NONE, QNN_ACT_LEAKY = 0, 1

_i32, _i64, _f32, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p

_SIGNATURES = {
    "qnn_conv3x3_fwd": [_i32, _i32, _i32, _vp, _i32, _vp, _vp, _i32, _i32, _vp, _i32, _i32, _i32, _vp],
    "qnn_conv3x3_fwd_fused": [_i32, _i32, _i32, _vp, _i32, _i32, _vp, _vp, _i32, _i32, _vp, _vp, _i32, _vp],
    "qnn_conv3x3_fwd_planes": [_i32, _i32, _i32, _vp, _i32, _vp, _vp, _i32, _i32, _vp, _i32, _vp, _vp],
    "qnn_conv3x3_fwd_pool": [_i32, _i32, _i32, _vp, _i32, _vp, _vp, _i32, _i32, _vp, _vp, _vp],
    "qnn_conv3x3_flip": [_vp, _i32, _i32, _vp, _vp],
    "qnn_conv3x3_wgrad": [_i32, _i32, _i32, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp],
    "qnn_leaky_bwd": [_i64, _vp, _vp, _vp, _vp],
    "qnn_add": [_i64, _vp, _vp, _vp, _vp],
    "qnn_avgpool2": [_i32, _i32, _i32, _i32, _vp, _vp, _vp],
    "qnn_avgpool2_bwd": [_i32, _i32, _i32, _i32, _vp, _vp, _i32, _vp],
    "qnn_upsample2": [_i32, _i32, _i32, _i32, _vp, _vp, _vp],
    "qnn_upsample2_bwd": [_i32, _i32, _i32, _i32, _vp, _vp, _vp],
    "qnn_absmax": [_i32, _i32, _i32, _vp, _vp, _vp, _vp],
    "qnn_pack_input": [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _f32, _f32, _i32, _vp, _vp],
    "qnn_unpack_output": [_i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp],
    "qnn_rel_l2": [_i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp],
    "qnn_adam": [_i64, _vp, _vp, _vp, _vp, _vp, _f32, _f32, _f32, _f32, _i32, _vp],
    "qnn_to_bf16": [_i64, _vp, _vp, _vp],
    "qnn_compare": [_i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp],
}

_bound = False


def _lib():
    global _bound
    L = qla.lib()
    if not _bound:
        for name, argtypes in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = argtypes
            fn.restype = ctypes.c_int
        L.qnn_wgrad_work_floats.argtypes = [_i32, _i32, _i32, _i32, _i32]
        L.qnn_wgrad_work_floats.restype = ctypes.c_int64
        L.qnn_compare_work_doubles.argtypes = [_i32]
        L.qnn_compare_work_doubles.restype = ctypes.c_int64
        _bound = True
    return L


def _call(name, *args):
    rc = getattr(_lib(), name)(*args)
    if rc != 0:
        raise qla.QlaError(rc, qla.qla_last_error())


def _p(t):
    """Device pointer of a tensor (or None)."""
    return None if t is None else t.data_ptr()


def _s(stream):
    return stream.cuda_stream if stream is not None else None


def qnn_conv3x3_fwd(B, H, W, x, c_in, w, bias, c_out, act, y, y_fp32, y_ld, c_store, stream=None):
    _call("qnn_conv3x3_fwd", B, H, W, _p(x), c_in, _p(w), _p(bias), c_out, act, _p(y), int(y_fp32),
          y_ld, c_store, _s(stream))


def qnn_conv3x3_fwd_fused(B, H, W, x, c_in, up, w, bias, c_out, act, add, y, y_ld, stream=None):
    _call("qnn_conv3x3_fwd_fused", B, H, W, _p(x), c_in, int(up), _p(w), _p(bias), c_out, act, _p(add), _p(y),
          y_ld, _s(stream))


def qnn_conv3x3_fwd_planes(B, H, W, x, c_in, w, bias, c_out, act, scale, n_planes, q, stream=None):
    _call("qnn_conv3x3_fwd_planes", B, H, W, _p(x), c_in, _p(w), _p(bias), c_out, act, _p(scale), n_planes, _p(q),
          _s(stream))


def qnn_conv3x3_fwd_pool(B, H, W, x, c_in, w, bias, c_out, act, y, pool, stream=None):
    _call("qnn_conv3x3_fwd_pool", B, H, W, _p(x), c_in, _p(w), _p(bias), c_out, act, _p(y), _p(pool), _s(stream))


def qnn_conv3x3_flip(w, c_out, c_in, wt, stream=None):
    _call("qnn_conv3x3_flip", _p(w), c_out, c_in, _p(wt), _s(stream))


def qnn_wgrad_work_floats(B, H, W, c_in, c_out) -> int:
    return int(_lib().qnn_wgrad_work_floats(B, H, W, c_in, c_out))


def qnn_conv3x3_wgrad(B, H, W, x, c_in, dy, c_out, dw, dbias, work, stream=None):
    _call("qnn_conv3x3_wgrad", B, H, W, _p(x), c_in, _p(dy), c_out, _p(dw), _p(dbias), _p(work), _s(stream))


def qnn_leaky_bwd(n, y, dy, dz, stream=None):
    _call("qnn_leaky_bwd", n, _p(y), _p(dy), _p(dz), _s(stream))


def qnn_add(n, a, b, y, stream=None):
    _call("qnn_add", n, _p(a), _p(b), _p(y), _s(stream))


def qnn_avgpool2(B, H, W, C, x, y, stream=None):
    _call("qnn_avgpool2", B, H, W, C, _p(x), _p(y), _s(stream))


def qnn_avgpool2_bwd(B, H, W, C, dy, dx, accumulate, stream=None):
    _call("qnn_avgpool2_bwd", B, H, W, C, _p(dy), _p(dx), int(accumulate), _s(stream))


def qnn_upsample2(B, h, w, C, x, y, stream=None):
    _call("qnn_upsample2", B, h, w, C, _p(x), _p(y), _s(stream))


def qnn_upsample2_bwd(B, h, w, C, dy, dx, stream=None):
    _call("qnn_upsample2_bwd", B, h, w, C, _p(dy), _p(dx), _s(stream))


def qnn_absmax(B, H, W, q, idx, scale, stream=None):
    _call("qnn_absmax", B, H, W, _p(q), _p(idx), _p(scale), _s(stream))


def qnn_pack_input(B, H, W, q, idx_q, n, idx_n, scale, n_shift, n_scale, shift, x, stream=None):
    _call("qnn_pack_input", B, H, W, _p(q), _p(idx_q), _p(n), _p(idx_n), _p(scale), float(n_shift),
          float(n_scale), int(shift), _p(x), _s(stream))


def qnn_unpack_output(B, H, W, y, y_ld, scale, q, stream=None):
    _call("qnn_unpack_output", B, H, W, _p(y), y_ld, _p(scale), _p(q), _s(stream))


def qnn_rel_l2(B, H, W, pred, pred_ld, target, idx_t, scale, dpred, d_ld, loss, per_sample, work,
               stream=None):
    _call("qnn_rel_l2", B, H, W, _p(pred), pred_ld, _p(target), _p(idx_t), _p(scale), _p(dpred), d_ld,
          _p(loss), _p(per_sample), _p(work), _s(stream))


def qnn_adam(n, p, m, v, g, p_bf16, lr, b1, b2, eps, t, stream=None):
    _call("qnn_adam", n, _p(p), _p(m), _p(v), _p(g), _p(p_bf16), float(lr), float(b1), float(b2),
          float(eps), int(t), _s(stream))


def qnn_to_bf16(n, x, y, stream=None):
    _call("qnn_to_bf16", n, _p(x), _p(y), _s(stream))


def qnn_compare_work_doubles(B) -> int:
    return int(_lib().qnn_compare_work_doubles(B))


def qnn_compare(B, m, a, r, rel, en, work, stream=None):
    _call("qnn_compare", B, m, _p(a), _p(r), _p(rel), _p(en), _p(work), _s(stream))
