"""MI355X data-parallel volume renderer: Python binding of ``libdpvr.so``.

Every ``vr_*`` function here has the name and meaning of the C entry point
declared in ``include/dpvr.h`` and only marshals arguments (torch tensors
for device memory, torch streams, host arrays); a non-OK status raises
:class:`VRError` with the library's message.  All rendering work runs in the
HIP kernels of the library -- there is no fallback: importing this package
raises if the library has not been built.

:class:`Renderer` is plumbing on top: it keeps the caller-owned device
buffers (brick workspaces, partial images, the frame) as torch tensors and
issues the calls of one frame: render every brick's partial, then composite.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpvr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2501_01628_amd.build` "
                      "(hipcc, gfx950); there is no CPU fallback")

# torch brings its own HIP runtime (SONAME libamdhip64.so.7).  Loading it
# first makes libdpvr.so's dependency on libamdhip64.so.7 resolve to that same
# runtime, so device memory and streams from torch are valid in the library;
# two runtimes in one process would not see each other's devices.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

VR_OK, VR_ERR_INVALID_ARG, VR_ERR_INVALID_HANDLE, VR_ERR_WORKSPACE = 0, -1, -2, -3
VR_ERR_UNSUPPORTED, VR_ERR_DEVICE, VR_ERR_STATE, VR_ERR_OUT_OF_MEMORY = -4, -5, -6, -7
VR_F32, VR_F16 = 0, 1
VR_PATH_STAGED, VR_PATH_DIRECT = 0, 1
VR_STAGING_SLAB, VR_STAGING_RING = 0, 1
TF_ENTRIES = 256
MAX_PARTIALS = 64
STATIC_MAX_PARTIALS = 64


class vr_partial(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("w", C.c_int32), ("h", C.c_int32),
                ("rgba", C.c_void_p), ("depth", C.c_void_p), ("samples", C.c_void_p)]


class vr_camera_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("pad_", C.c_int32),
                ("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fovy_deg", C.c_double)]


class vr_tf_desc(C.Structure):
    _fields_ = [("rgba", C.c_void_p), ("vmin", C.c_float), ("vmax", C.c_float),
                ("opacity_scale", C.c_float), ("pad_", C.c_int32)]


class vr_batch_job(C.Structure):
    _fields_ = [("brick", C.c_void_p), ("camera", C.c_int32), ("tf", C.c_int32), ("part", vr_partial)]


class vr_batch_frame(C.Structure):
    _fields_ = [("camera", C.c_int32), ("first_job", C.c_int32), ("n_jobs", C.c_int32),
                ("pad_", C.c_int32), ("bg", C.c_float * 4), ("out", C.c_void_p)]


class vr_brick_desc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("ghost", C.c_int32), ("origin", C.c_double * 3),
                ("spacing", C.c_double * 3), ("storage", C.c_int), ("pad_", C.c_int32)]


class vr_light(C.Structure):
    _fields_ = [("direction", C.c_double * 3), ("ambient", C.c_float), ("pad_", C.c_int32)]


_i3 = C.c_int32 * 3
_d3 = C.c_double * 3
_f4 = C.c_float * 4
_st = C.c_int

_SIGS = {
    "vr_abi_version": ([], C.c_int32),
    "vr_status_string": ([C.c_int], C.c_char_p),
    "vr_last_error": ([C.c_void_p], C.c_char_p),
    "vr_context_create": ([C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)], _st),
    "vr_context_release": ([C.c_void_p], _st),
    "vr_context_set_stream": ([C.c_void_p, C.c_void_p], _st),
    "vr_synchronize": ([C.c_void_p], _st),
    "vr_brick_workspace_size": ([_i3, C.c_int32, C.c_int, C.POINTER(C.c_size_t)], _st),
    "vr_brick_create": ([C.c_void_p, _i3, C.c_int32, _d3, _d3, C.c_int, C.c_void_p, C.c_size_t,
                         C.POINTER(C.c_void_p)], _st),
    "vr_brick_set_data": ([C.c_void_p, C.c_void_p], _st),
    "vr_brick_release": ([C.c_void_p], _st),
    "vr_set_transfer_function": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_float,
                                  C.c_float], _st),
    "vr_set_camera_perspective": ([C.c_void_p, _d3, _d3, _d3, C.c_double, C.c_int32, C.c_int32],
                                  _st),
    "vr_set_camera_orthographic": ([C.c_void_p, _d3, _d3, _d3, C.c_double, C.c_int32, C.c_int32],
                                   _st),
    "vr_set_render_params": ([C.c_void_p, C.c_double, C.c_float], _st),
    "vr_partial_roi": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)], _st),
    "vr_render_partial": ([C.c_void_p, C.c_void_p, C.POINTER(vr_partial)], _st),
    "vr_composite": ([C.c_void_p, C.POINTER(vr_partial), C.c_int32, _f4, C.c_void_p], _st),
    "vr_brick_set_data_global": ([C.c_void_p, C.c_void_p, _i3, _i3], _st),
    "vr_set_march_path": ([C.c_void_p, C.c_int], _st),
    "vr_frame_workspace_size": ([C.c_int32, C.POINTER(C.c_size_t)], _st),
    "vr_camera_roi": ([C.c_void_p, C.c_void_p, C.POINTER(vr_camera_desc), C.POINTER(C.c_int32)], _st),
    "vr_batch_workspace_size": ([C.c_int32, C.c_int32, C.POINTER(C.c_size_t)], _st),
    "vr_batch_create": ([C.c_void_p, C.c_int32, C.POINTER(vr_camera_desc), C.c_int32,
                         C.POINTER(vr_tf_desc), C.c_int32, C.POINTER(vr_batch_job), C.c_int32,
                         C.POINTER(vr_batch_frame), C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)], _st),
    "vr_batch_launch": ([C.c_void_p], _st),
    "vr_batch_autotune": ([C.c_void_p, C.c_int32, C.POINTER(C.c_double)], _st),
    "vr_batch_config": ([C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                         C.POINTER(C.c_int32), C.POINTER(C.c_int32)], _st),
    "vr_set_march_config": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32], _st),
    "vr_batch_release": ([C.c_void_p], _st),
    "vr_batch_set_groups": ([C.c_void_p, C.c_int32], _st),
    "vr_batch_group": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], _st),
    "vr_batch_wait_group": ([C.c_void_p, C.c_int32, C.c_void_p], _st),
    "vr_batch_group_done": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int32)], _st),
    "vr_render_partials": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(vr_partial),
                            C.c_void_p, C.c_size_t], _st),
    "vr_render_partials_static": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                   C.POINTER(vr_partial)], _st),
    "vr_checkpoint_size": ([C.c_void_p, C.c_void_p, C.POINTER(vr_partial), C.c_int32,
                            C.POINTER(C.c_size_t)], _st),
    "vr_render_partial_checkpointed": ([C.c_void_p, C.c_void_p, C.POINTER(vr_partial), C.c_int32,
                                        C.c_void_p, C.c_size_t], _st),
    "vr_composite_backward": ([C.c_void_p, C.POINTER(vr_partial), C.c_int32, _f4, C.c_void_p,
                               C.POINTER(C.c_void_p)], _st),
    "vr_render_partial_backward": ([C.c_void_p, C.c_void_p, C.POINTER(vr_partial), C.c_int32,
                                    C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                                    _i3, _i3], _st),
    "vr_timeseries_workspace_size": ([C.c_int32, C.POINTER(vr_brick_desc), C.c_int32, C.POINTER(C.c_size_t)],
                                     _st),
    "vr_timeseries_create": ([C.c_void_p, C.c_int32, C.POINTER(vr_brick_desc), C.c_int32,
                              C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)],
                             _st),
    "vr_timeseries_prefetch": ([C.c_void_p, C.c_int32], _st),
    "vr_timeseries_acquire": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)], _st),
    "vr_timeseries_stats": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)], _st),
    "vr_timeseries_release": ([C.c_void_p], _st),
    "vr_backward_workspace_size": ([C.c_int32, C.POINTER(C.c_size_t)], _st),
    "vr_checkpointed_workspace_size": ([C.c_int32, C.POINTER(C.c_size_t)], _st),
    "vr_render_partials_checkpointed": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(vr_partial),
                                         C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_size_t), C.c_void_p,
                                         C.c_size_t], _st),
    "vr_render_partials_backward": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(vr_partial), C.c_int32,
                                     C.POINTER(C.c_void_p), C.POINTER(C.c_size_t), C.POINTER(C.c_void_p),
                                     C.c_void_p, C.c_void_p, _i3, C.POINTER(C.c_int32), C.c_void_p, C.c_size_t],
                                    _st),
    "vr_rqc_workspace_size": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_size_t)], _st),
    "vr_rqc_plan": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t,
                     C.POINTER(C.c_int64)], _st),
    "vr_render_rqc": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(vr_light), _f4, C.c_void_p,
                       C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p], _st),
    "vr_tetpart_create": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)], _st),
    "vr_tetpart_info": ([C.c_void_p, _d3, _d3, _i3, C.POINTER(C.c_int64), C.POINTER(C.c_size_t),
                         C.POINTER(C.c_int32)], _st),
    "vr_tetpart_create_cells": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.POINTER(C.c_void_p)], _st),
    "vr_set_tet_locator": ([C.c_void_p, C.c_int], _st),
    "vr_tetpart_attach": ([C.c_void_p, C.c_void_p, C.c_size_t], _st),
    "vr_tetpart_set_values": ([C.c_void_p, C.c_void_p], _st),
    "vr_tetpart_release": ([C.c_void_p], _st),
    "vr_tetparts_workspace_size": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_int32,
                                    C.POINTER(C.c_size_t)], _st),
    "vr_render_tetparts": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_int32, _f4, C.c_void_p, C.c_size_t,
                            C.c_void_p, C.c_void_p], _st),
    "vr_march_tetparts": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_size_t,
                           C.c_void_p], _st),
    "vr_resolve_tetparts": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_int32, _f4, C.c_void_p, C.c_size_t,
                             C.c_void_p], _st),
    "vr_tetparts_shadow_plan_size": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_size_t)], _st),
    "vr_tetparts_shadow_plan": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_size_t,
                                 C.c_void_p, C.c_size_t, C.POINTER(C.c_int64)], _st),
    "vr_tetparts_slot_bytes": ([C.c_int64, C.POINTER(C.c_size_t)], _st),
    "vr_render_tetparts_shadowed": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_int32, C.POINTER(vr_light),
                                     _f4, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t,
                                     C.c_void_p, C.c_void_p], _st),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class VRError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_lib.vr_status_string(status).decode()}: {message}")
        self.status = status


def _check(status, ctx=None):
    if status != VR_OK:
        raise VRError(status, _lib.vr_last_error(ctx).decode(errors="replace"))


def _ptr(x):
    """Device (or host) address of a torch tensor / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------------- C entry points
def vr_abi_version():
    return _lib.vr_abi_version()


def vr_status_string(status):
    return _lib.vr_status_string(status).decode()


def vr_last_error(ctx=None):
    return _lib.vr_last_error(ctx).decode(errors="replace")


def vr_context_create(device=0, stream=None):
    h = C.c_void_p()
    _check(_lib.vr_context_create(int(device), _stream_ptr(stream), C.byref(h)))
    return h.value


def vr_context_release(ctx):
    _check(_lib.vr_context_release(ctx))


def vr_context_set_stream(ctx, stream):
    _check(_lib.vr_context_set_stream(ctx, _stream_ptr(stream)), ctx)


def vr_synchronize(ctx):
    _check(_lib.vr_synchronize(ctx), ctx)


def vr_brick_workspace_size(dims, ghost=1, storage=VR_F32):
    n = C.c_size_t()
    _check(_lib.vr_brick_workspace_size(_i3(*dims), int(ghost), int(storage), C.byref(n)))
    return n.value


def vr_brick_create(ctx, dims, ghost, origin, spacing, storage, workspace, workspace_bytes):
    h = C.c_void_p()
    _check(_lib.vr_brick_create(ctx, _i3(*dims), int(ghost), _d3(*origin), _d3(*spacing),
                                int(storage), _ptr(workspace), int(workspace_bytes), C.byref(h)),
           ctx)
    return h.value


def vr_brick_set_data(brick, voxels, ctx=None):
    _check(_lib.vr_brick_set_data(brick, _ptr(voxels)), ctx)


def vr_brick_release(brick):
    _check(_lib.vr_brick_release(brick))


def vr_set_transfer_function(ctx, rgba, n=TF_ENTRIES, vmin=0.0, vmax=1.0, opacity_scale=1.0):
    _check(_lib.vr_set_transfer_function(ctx, _ptr(rgba), int(n), float(vmin), float(vmax),
                                         float(opacity_scale)), ctx)


def vr_set_camera_perspective(ctx, eye, target, up, fovy_deg, width, height):
    _check(_lib.vr_set_camera_perspective(ctx, _d3(*eye), _d3(*target), _d3(*up), float(fovy_deg),
                                          int(width), int(height)), ctx)


def vr_set_camera_orthographic(ctx, pos, dir, up, view_height, width, height):
    _check(_lib.vr_set_camera_orthographic(ctx, _d3(*pos), _d3(*dir), _d3(*up),
                                           float(view_height), int(width), int(height)), ctx)


def vr_set_render_params(ctx, dt=0.5, ert_epsilon=2.0 ** -20):
    _check(_lib.vr_set_render_params(ctx, float(dt), float(ert_epsilon)), ctx)


def vr_partial_roi(ctx, brick):
    roi = (C.c_int32 * 4)()
    _check(_lib.vr_partial_roi(ctx, brick, roi), ctx)
    return tuple(roi)


def make_partial(roi, rgba, depth, samples=None):
    x0, y0, w, h = roi
    return vr_partial(int(x0), int(y0), int(w), int(h), _ptr(rgba), _ptr(depth), _ptr(samples))


def vr_render_partial(ctx, brick, part):
    _check(_lib.vr_render_partial(ctx, brick, C.byref(part)), ctx)


def vr_composite(ctx, parts, bg, out):
    n = len(parts)
    arr = (vr_partial * max(n, 1))(*parts)
    _check(_lib.vr_composite(ctx, arr, n, _f4(*bg), _ptr(out)), ctx)


def _brick_descs(descs):
    arr = (vr_brick_desc * len(descs))()
    for i, (dims, origin, spacing, storage) in enumerate(descs):
        arr[i] = vr_brick_desc(_i3(*dims), 1, _d3(*origin), _d3(*spacing), int(storage), 0)
    return arr


def vr_timeseries_workspace_size(descs, slots):
    """descs: [(dims, origin, spacing, storage)] (ghost 1)."""
    n = C.c_size_t()
    _check(_lib.vr_timeseries_workspace_size(len(descs), _brick_descs(descs), int(slots), C.byref(n)))
    return n.value


def vr_timeseries_create(ctx, descs, host_ptrs, n_steps, slots, workspace, workspace_bytes):
    hp = (C.c_void_p * len(host_ptrs))(*host_ptrs)
    h = C.c_void_p()
    _check(_lib.vr_timeseries_create(ctx, len(descs), _brick_descs(descs), int(n_steps), hp, int(slots),
                                     _ptr(workspace), int(workspace_bytes), C.byref(h)), ctx)
    return h.value


def vr_timeseries_prefetch(ts, step, ctx=None):
    _check(_lib.vr_timeseries_prefetch(ts, int(step)), ctx)


def vr_timeseries_acquire(ts, step, n_bricks, ctx=None):
    out = (C.c_void_p * n_bricks)()
    _check(_lib.vr_timeseries_acquire(ts, int(step), out), ctx)
    return list(out)


def vr_timeseries_stats(ts, slots, ctx=None):
    loads = C.c_int64()
    res = (C.c_int32 * slots)()
    _check(_lib.vr_timeseries_stats(ts, C.byref(loads), res), ctx)
    return loads.value, list(res)


def vr_timeseries_release(ts, ctx=None):
    _check(_lib.vr_timeseries_release(ts), ctx)


def vr_checkpointed_workspace_size(n):
    b = C.c_size_t()
    _check(_lib.vr_checkpointed_workspace_size(int(n), C.byref(b)))
    return b.value


def vr_render_partials_checkpointed(ctx, bricks, parts, interval, ckpts, workspace, workspace_bytes):
    """ckpts: [(tensor, nbytes)] per partial."""
    n = len(bricks)
    hb = (C.c_void_p * max(n, 1))(*bricks)
    hp = (vr_partial * max(n, 1))(*parts)
    hc = (C.c_void_p * max(n, 1))(*[_ptr(c) for c, _ in ckpts])
    hcb = (C.c_size_t * max(n, 1))(*[int(b) for _, b in ckpts])
    _check(_lib.vr_render_partials_checkpointed(ctx, n, hb, hp, int(interval), hc, hcb, _ptr(workspace),
                                                int(workspace_bytes)), ctx)


def vr_backward_workspace_size(n):
    b = C.c_size_t()
    _check(_lib.vr_backward_workspace_size(int(n), C.byref(b)))
    return b.value


def vr_render_partials_backward(ctx, bricks, parts, interval, ckpts, d_parts, grad_tf, grad_volume, vol_dims, los,
                                workspace, workspace_bytes):
    """ckpts: [(tensor, nbytes)] per partial; los: [(x, y, z)] per partial."""
    n = len(bricks)
    hb = (C.c_void_p * max(n, 1))(*bricks)
    hp = (vr_partial * max(n, 1))(*parts)
    hc = (C.c_void_p * max(n, 1))(*[_ptr(c) for c, _ in ckpts])
    hcb = (C.c_size_t * max(n, 1))(*[int(b) for _, b in ckpts])
    hd = (C.c_void_p * max(n, 1))(*[_ptr(d) for d in d_parts])
    hl = (C.c_int32 * max(3 * n, 1))(*[int(v) for lo in los for v in lo])
    _check(_lib.vr_render_partials_backward(ctx, n, hb, hp, int(interval), hc, hcb, hd, _ptr(grad_tf),
                                            _ptr(grad_volume), _i3(*vol_dims), hl, _ptr(workspace),
                                            int(workspace_bytes)), ctx)


def vr_rqc_workspace_size(ctx, bricks):
    arr = (C.c_void_p * len(bricks))(*bricks)
    b = C.c_size_t()
    _check(_lib.vr_rqc_workspace_size(ctx, len(bricks), arr, C.byref(b)), ctx)
    return b.value


def vr_rqc_plan(ctx, bricks, ws, nbytes):
    arr = (C.c_void_p * len(bricks))(*bricks)
    total = C.c_int64()
    _check(_lib.vr_rqc_plan(ctx, len(bricks), arr, _ptr(ws), nbytes, C.byref(total)), ctx)
    return total.value


def vr_render_rqc(ctx, bricks, light_dir, ambient, bg, ws, nbytes, shade, shade_bytes, out, samples=None):
    arr = (C.c_void_p * len(bricks))(*bricks)
    lt = vr_light((C.c_double * 3)(*[float(v) for v in light_dir]), float(ambient), 0)
    _check(_lib.vr_render_rqc(ctx, len(bricks), arr, C.byref(lt), _f4(*bg), _ptr(ws), nbytes,
                              _ptr(shade) if shade is not None else None, shade_bytes, _ptr(out),
                              _ptr(samples)), ctx)


def vr_tetpart_create(ctx, vertices, tets):
    """A tetrahedral part from host arrays (vertices (V, 3) float64, tets
    (T, 4) int32); the location tables are built on the host."""
    v = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
    h = C.c_void_p()
    _check(_lib.vr_tetpart_create(ctx, v.ctypes.data, len(v), t.ctypes.data, len(t), C.byref(h)), ctx)
    return h


def vr_tetpart_create_cells(ctx, vertices, sizes, cell_vertices, vertex_ids=None):
    """A part from mixed cells (host arrays: vertices (V, 3) float64, sizes
    (C,) uint8 in {4, 5, 6, 8}, cell_vertices int32, optional vertex_ids (V,)
    int64 global ids for the quadrilateral cuts)."""
    v = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1, 3)
    sz = np.ascontiguousarray(sizes, dtype=np.uint8)
    cv = np.ascontiguousarray(cell_vertices, dtype=np.int32)
    ids = None if vertex_ids is None else np.ascontiguousarray(vertex_ids, dtype=np.int64)
    h = C.c_void_p()
    _check(_lib.vr_tetpart_create_cells(ctx, v.ctypes.data, len(v), None if ids is None else ids.ctypes.data,
                                        sz.ctypes.data, cv.ctypes.data, len(sz), C.byref(h)), ctx)
    return h


VR_TET_GRID, VR_TET_BVH = 0, 1


def vr_set_tet_locator(ctx, locator):
    _check(_lib.vr_set_tet_locator(ctx, int(locator)), ctx)


def vr_tetpart_info(part, ctx=None):
    lo, hi, grid = _d3(), _d3(), _i3()
    entries, nbytes, nt = C.c_int64(), C.c_size_t(), C.c_int32()
    _check(_lib.vr_tetpart_info(part, lo, hi, grid, C.byref(entries), C.byref(nbytes), C.byref(nt)), ctx)
    return dict(lo=tuple(lo), hi=tuple(hi), grid=tuple(grid), grid_entries=entries.value,
                workspace_bytes=nbytes.value, n_tets=nt.value)


def vr_tetpart_attach(part, workspace, workspace_bytes, ctx=None):
    _check(_lib.vr_tetpart_attach(part, _ptr(workspace), int(workspace_bytes)), ctx)


def vr_tetpart_set_values(part, values, ctx=None):
    _check(_lib.vr_tetpart_set_values(part, _ptr(values)), ctx)


def vr_tetpart_release(part, ctx=None):
    _check(_lib.vr_tetpart_release(part), ctx)


def vr_tetparts_workspace_size(ctx, parts, max_runs):
    arr = (C.c_void_p * len(parts))(*[p.value if isinstance(p, C.c_void_p) else p for p in parts])
    b = C.c_size_t()
    _check(_lib.vr_tetparts_workspace_size(ctx, len(parts), arr, int(max_runs), C.byref(b)), ctx)
    return b.value


def vr_render_tetparts(ctx, parts, max_runs, bg, workspace, workspace_bytes, out, samples=None):
    arr = (C.c_void_p * len(parts))(*[p.value if isinstance(p, C.c_void_p) else p for p in parts])
    _check(_lib.vr_render_tetparts(ctx, len(parts), arr, int(max_runs), _f4(*bg), _ptr(workspace),
                                   int(workspace_bytes), _ptr(out), _ptr(samples)), ctx)


def vr_march_tetparts(ctx, parts, max_runs, workspace, workspace_bytes, samples=None):
    arr = (C.c_void_p * len(parts))(*[p.value if isinstance(p, C.c_void_p) else p for p in parts])
    _check(_lib.vr_march_tetparts(ctx, len(parts), arr, int(max_runs), _ptr(workspace), int(workspace_bytes),
                                  _ptr(samples)), ctx)


def vr_resolve_tetparts(ctx, parts, max_runs, bg, workspace, workspace_bytes, out):
    arr = (C.c_void_p * len(parts))(*[p.value if isinstance(p, C.c_void_p) else p for p in parts])
    _check(_lib.vr_resolve_tetparts(ctx, len(parts), arr, int(max_runs), _f4(*bg), _ptr(workspace),
                                    int(workspace_bytes), _ptr(out)), ctx)


def _parts_array(parts):
    return (C.c_void_p * len(parts))(*[p.value if isinstance(p, C.c_void_p) else p for p in parts])


def vr_tetparts_shadow_plan_size(ctx, parts):
    b = C.c_size_t()
    _check(_lib.vr_tetparts_shadow_plan_size(ctx, len(parts), _parts_array(parts), C.byref(b)), ctx)
    return b.value


def vr_tetparts_shadow_plan(ctx, parts, max_runs, workspace, workspace_bytes, plan, plan_bytes):
    total = C.c_int64()
    _check(_lib.vr_tetparts_shadow_plan(ctx, len(parts), _parts_array(parts), int(max_runs), _ptr(workspace),
                                        int(workspace_bytes), _ptr(plan), int(plan_bytes), C.byref(total)), ctx)
    return total.value


def vr_tetparts_slot_bytes(total):
    b = C.c_size_t()
    _check(_lib.vr_tetparts_slot_bytes(int(total), C.byref(b)))
    return b.value


def vr_render_tetparts_shadowed(ctx, parts, max_runs, light_dir, ambient, bg, workspace, workspace_bytes, plan,
                                plan_bytes, slots, slot_bytes, out, samples=None):
    lt = vr_light((C.c_double * 3)(*[float(x) for x in light_dir]), float(ambient), 0)
    _check(_lib.vr_render_tetparts_shadowed(ctx, len(parts), _parts_array(parts), int(max_runs), C.byref(lt),
                                            _f4(*bg), _ptr(workspace), int(workspace_bytes), _ptr(plan),
                                            int(plan_bytes), _ptr(slots), int(slot_bytes), _ptr(out),
                                            _ptr(samples)), ctx)


def vr_set_march_path(ctx, path):
    _check(_lib.vr_set_march_path(ctx, int(path)), ctx)


def vr_set_march_config(ctx, storage, staging, tile_width, chunk_slices=4):
    _check(_lib.vr_set_march_config(ctx, int(storage), int(staging), int(tile_width), int(chunk_slices)), ctx)


def vr_frame_workspace_size(n):
    b = C.c_size_t()
    _check(_lib.vr_frame_workspace_size(int(n), C.byref(b)))
    return b.value


def vr_render_partials(ctx, bricks, parts, workspace, workspace_bytes):
    n = len(bricks)
    hb = (C.c_void_p * max(n, 1))(*bricks)
    hp = (vr_partial * max(n, 1))(*parts)
    _check(_lib.vr_render_partials(ctx, n, hb, hp, _ptr(workspace), int(workspace_bytes)), ctx)


def vr_render_partials_static(ctx, bricks, parts):
    n = len(bricks)
    hb = (C.c_void_p * max(n, 1))(*bricks)
    hp = (vr_partial * max(n, 1))(*parts)
    _check(_lib.vr_render_partials_static(ctx, n, hb, hp), ctx)


def camera_desc(cam: dict) -> vr_camera_desc:
    d = vr_camera_desc()
    persp = cam.get("kind", "perspective") == "perspective"
    d.kind = 0 if persp else 1
    d.width, d.height = int(cam["width"]), int(cam["height"])
    d.eye[:] = [float(v) for v in cam["eye"]]
    d.target[:] = [float(v) for v in (cam["target"] if persp else cam["dir"])]
    d.up[:] = [float(v) for v in cam["up"]]
    d.fovy_deg = float(cam["fovy_deg"] if persp else cam["view_height"])
    return d


def vr_camera_roi(ctx, brick, cam):
    roi = (C.c_int32 * 4)()
    d = cam if isinstance(cam, vr_camera_desc) else camera_desc(cam)
    _check(_lib.vr_camera_roi(ctx, brick, C.byref(d), roi), ctx)
    return tuple(roi)


def vr_batch_workspace_size(n_jobs, n_frames):
    b = C.c_size_t()
    _check(_lib.vr_batch_workspace_size(int(n_jobs), int(n_frames), C.byref(b)))
    return b.value


def vr_batch_create(ctx, cameras, tfs, jobs, frames, workspace, workspace_bytes):
    hc = (vr_camera_desc * max(len(cameras), 1))(*cameras)
    ht = (vr_tf_desc * max(len(tfs), 1))(*tfs)
    hj = (vr_batch_job * max(len(jobs), 1))(*jobs)
    hf = (vr_batch_frame * max(len(frames), 1))(*frames)
    h = C.c_void_p()
    _check(_lib.vr_batch_create(ctx, len(cameras), hc, len(tfs), ht, len(jobs), hj, len(frames), hf,
                                _ptr(workspace), int(workspace_bytes), C.byref(h)), ctx)
    return h.value


def vr_batch_launch(batch, ctx=None):
    _check(_lib.vr_batch_launch(batch), ctx)


def vr_batch_autotune(batch, reps=3, ctx=None):
    ms = C.c_double()
    _check(_lib.vr_batch_autotune(batch, int(reps), C.byref(ms)), ctx)
    return ms.value


def vr_batch_config(batch, ctx=None):
    """(workgroups per CU, job order, staging, tile width, chunk slices)."""
    w, o, g, t, c = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.vr_batch_config(batch, C.byref(w), C.byref(o), C.byref(g), C.byref(t), C.byref(c)), ctx)
    return w.value, o.value, g.value, t.value, c.value


def vr_batch_set_groups(batch, n_groups, ctx=None):
    _check(_lib.vr_batch_set_groups(batch, int(n_groups)), ctx)


def vr_batch_group(batch, group, ctx=None):
    f0, n = C.c_int32(), C.c_int32()
    _check(_lib.vr_batch_group(batch, int(group), C.byref(f0), C.byref(n)), ctx)
    return f0.value, n.value


def vr_batch_wait_group(batch, group, stream=None, ctx=None):
    _check(_lib.vr_batch_wait_group(batch, int(group), stream), ctx)


def vr_batch_group_done(batch, group, ctx=None):
    d = C.c_int32()
    _check(_lib.vr_batch_group_done(batch, int(group), C.byref(d)), ctx)
    return bool(d.value)


def vr_batch_release(batch):
    _check(_lib.vr_batch_release(batch))


def vr_brick_set_data_global(brick, volume, vol_dims, lo, ctx=None):
    _check(_lib.vr_brick_set_data_global(brick, _ptr(volume), _i3(*vol_dims), _i3(*lo)), ctx)


def vr_checkpoint_size(ctx, brick, part, interval):
    n = C.c_size_t()
    _check(_lib.vr_checkpoint_size(ctx, brick, C.byref(part), int(interval), C.byref(n)), ctx)
    return n.value


def vr_render_partial_checkpointed(ctx, brick, part, interval, ckpt, ckpt_bytes):
    _check(_lib.vr_render_partial_checkpointed(ctx, brick, C.byref(part), int(interval), _ptr(ckpt),
                                               int(ckpt_bytes)), ctx)


def vr_composite_backward(ctx, parts, bg, d_out, d_parts):
    n = len(parts)
    arr = (vr_partial * max(n, 1))(*parts)
    dps = (C.c_void_p * max(n, 1))(*[_ptr(d) for d in d_parts])
    _check(_lib.vr_composite_backward(ctx, arr, n, _f4(*bg), _ptr(d_out), dps), ctx)


def vr_render_partial_backward(ctx, brick, part, interval, ckpt, ckpt_bytes, d_part, grad_tf,
                               grad_volume, vol_dims, lo):
    _check(_lib.vr_render_partial_backward(ctx, brick, C.byref(part), int(interval), _ptr(ckpt),
                                           int(ckpt_bytes), _ptr(d_part), _ptr(grad_tf),
                                           _ptr(grad_volume), _i3(*vol_dims), _i3(*lo)), ctx)


def set_camera(ctx, cam: dict):
    """Apply a camera dict (``kind``, ``eye``, ``target``/``dir``, ``up``,
    ``fovy_deg``/``view_height``, ``width``, ``height``)."""
    if cam.get("kind", "perspective") == "perspective":
        vr_set_camera_perspective(ctx, cam["eye"], cam["target"], cam["up"], cam["fovy_deg"],
                                  cam["width"], cam["height"])
    else:
        vr_set_camera_orthographic(ctx, cam["eye"], cam["dir"], cam["up"], cam["view_height"],
                                   cam["width"], cam["height"])


# ------------------------------------------------------------ frame helpers
class TetRenderer:
    """Torch buffers and C-ABI calls for a volume given as tetrahedral parts
    on one device.  ``parts`` is a list of (vertices (V, 3) float64, tets
    (T, 4) int32) host arrays, or of (vertices, sizes, cell_vertices,
    vertex_ids) for mixed cells; vertex values come per part through
    :meth:`set_values`."""

    def __init__(self, parts, tf, vrange=(0.0, 1.0), opacity_scale=1.0, dt=0.5, device=0, stream=None,
                 max_runs=8, locator=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = vr_context_create(device, self.stream)
        self.tf = torch.as_tensor(np.ascontiguousarray(tf, dtype=np.float32)).to(self.device)
        vr_set_transfer_function(self.ctx, self.tf, TF_ENTRIES, vrange[0], vrange[1], opacity_scale)
        vr_set_render_params(self.ctx, dt, 0.0)
        if locator is not None:
            vr_set_tet_locator(self.ctx, locator)
        self.max_runs = int(max_runs)
        self.parts, self.workspaces, self.values, self.info = [], [], [], []
        for part in parts:
            h = vr_tetpart_create(self.ctx, *part) if len(part) == 2 else vr_tetpart_create_cells(self.ctx, *part)
            inf = vr_tetpart_info(h, self.ctx)
            n = inf["workspace_bytes"]
            ws = torch.empty(n // 4 + 64, dtype=torch.float32, device=self.device)
            base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
            vr_tetpart_attach(h, base, n, self.ctx)
            self.parts.append(h)
            self.workspaces.append(ws)
            self.values.append(None)
            self.info.append(inf)
        self.frame = None
        self._fws, self._fws_bytes = None, 0
        self.samples = torch.zeros(1, dtype=torch.int64, device=self.device)

    def set_values(self, k, values):
        v = self.torch.as_tensor(values).to(self.device, self.torch.float32).contiguous()
        vr_tetpart_set_values(self.parts[k], v, self.ctx)
        self.values[k] = v                    # kept alive until the next sync

    def set_camera(self, cam):
        set_camera(self.ctx, cam)
        self.width, self.height = int(cam["width"]), int(cam["height"])
        need = vr_tetparts_workspace_size(self.ctx, self.parts, self.max_runs)
        if self._fws is None or self._fws_bytes < need:
            self._fws = self.torch.empty(need // 4 + 64, dtype=self.torch.float32, device=self.device)
            self._fws_bytes = need
        if self.frame is None or self.frame.numel() != self.width * self.height * 4:
            self.frame = self.torch.empty(self.height, self.width, 4, dtype=self.torch.float32,
                                          device=self.device)

    def _base(self):
        return self._fws.data_ptr() + ((-self._fws.data_ptr()) % 256)

    def render(self, bg=(0.0, 0.0, 0.0, 0.0), count=False):
        vr_render_tetparts(self.ctx, self.parts, self.max_runs, bg, self._base(), self._fws_bytes, self.frame,
                           self.samples if count else None)
        return self.frame

    def march(self, count=False):
        """The march stage alone (runs of every part into the workspace)."""
        vr_march_tetparts(self.ctx, self.parts, self.max_runs, self._base(), self._fws_bytes,
                          self.samples if count else None)

    def resolve(self, bg=(0.0, 0.0, 0.0, 0.0)):
        """The resolve stage alone (after :meth:`march`)."""
        vr_resolve_tetparts(self.ctx, self.parts, self.max_runs, bg, self._base(), self._fws_bytes, self.frame)
        return self.frame

    def shadow_plan(self):
        """Plan the shadow rays of the current camera (plan and slot buffers
        allocated here; synchronises); returns the number of slots."""
        torch = self.torch
        pb = vr_tetparts_shadow_plan_size(self.ctx, self.parts)
        plan = torch.empty(pb // 4 + 64, dtype=torch.float32, device=self.device)
        pbase = plan.data_ptr() + ((-plan.data_ptr()) % 256)
        total = vr_tetparts_shadow_plan(self.ctx, self.parts, self.max_runs, self._base(), self._fws_bytes, pbase,
                                        pb)
        sb = vr_tetparts_slot_bytes(total)
        slots = torch.empty(sb // 4 + 64, dtype=torch.float32, device=self.device)
        sbase = slots.data_ptr() + ((-slots.data_ptr()) % 256)
        self._shadow = (plan, pbase, pb, slots, sbase, sb)
        return total

    def render_shadowed(self, light_dir, ambient, bg=(0.0, 0.0, 0.0, 0.0), count=False):
        """The frame with one directional light (plan first with
        :meth:`shadow_plan`)."""
        _, pbase, pb, _, sbase, sb = self._shadow
        vr_render_tetparts_shadowed(self.ctx, self.parts, self.max_runs, light_dir, ambient, bg, self._base(),
                                    self._fws_bytes, pbase, pb, sbase, sb, self.frame,
                                    self.samples if count else None)
        return self.frame

    def synchronize(self):
        vr_synchronize(self.ctx)

    def close(self):
        for h in self.parts:
            vr_tetpart_release(h, self.ctx)
        self.parts = []
        if self.ctx is not None:
            vr_context_release(self.ctx)
            self.ctx = None


class Renderer:
    """Owns the torch buffers of one scene on one device and issues the
    C-ABI calls of a frame.  ``bricks`` is a list of (voxels, lo) with voxels a
    ghost-padded float32 array (numpy or torch, (nz+2, ny+2, nx+2)) and lo
    the owned box's integer min corner; spacing is 1 (voxel units)."""

    def __init__(self, bricks, tf, vrange=(0.0, 1.0), opacity_scale=1.0, dt=0.5,
                 ert_eps=2.0 ** -20, storage=VR_F32, device=0, stream=None, spacing=(1.0, 1.0, 1.0),
                 path=VR_PATH_STAGED, march_config=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = vr_context_create(device, self.stream)
        self.storage = storage
        self.bricks, self.workspaces, self.meta = [], [], []
        self.tf = torch.as_tensor(np.ascontiguousarray(tf, dtype=np.float32)).to(self.device)
        vr_set_transfer_function(self.ctx, self.tf, TF_ENTRIES, vrange[0], vrange[1], opacity_scale)
        vr_set_render_params(self.ctx, dt, ert_eps)
        vr_set_march_path(self.ctx, path)
        if march_config is not None:     # (staging, tile_width, chunk_slices) for both storages
            for st in (VR_F32, VR_F16):
                vr_set_march_config(self.ctx, st, *march_config)
        for vox, lo in bricks:
            self.add_brick(vox, lo, spacing)
        self._parts = {}
        self.frame = None
        self.samples = torch.zeros(max(len(self.bricks), 1), dtype=torch.int64, device=self.device)

    def add_brick(self, vox, lo, spacing=(1.0, 1.0, 1.0)):
        torch = self.torch
        v = torch.as_tensor(vox).to(self.device, torch.float32).contiguous()
        nz, ny, nx = (int(s) - 2 for s in v.shape)
        dims = (nx, ny, nz)
        nbytes = vr_brick_workspace_size(dims, 1, self.storage)
        ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.device)
        base = ws.data_ptr()
        off = (-base) % 256
        h = vr_brick_create(self.ctx, dims, 1, tuple(float(x) for x in lo), spacing, self.storage,
                            base + off, nbytes)
        vr_brick_set_data(h, v, self.ctx)
        self.bricks.append(h)
        self.workspaces.append((ws, v))       # source kept alive until the next sync
        self.meta.append((dims, tuple(lo)))
        return h

    def set_data(self, k, vox):
        v = self.torch.as_tensor(vox).to(self.device, self.torch.float32).contiguous()
        vr_brick_set_data(self.bricks[k], v, self.ctx)
        self.workspaces[k] = (self.workspaces[k][0], v)

    def set_camera(self, cam):
        set_camera(self.ctx, cam)
        self.width, self.height = int(cam["width"]), int(cam["height"])
        self.rois = [vr_partial_roi(self.ctx, b) for b in self.bricks]
        torch = self.torch
        self.partials = []
        for k, roi in enumerate(self.rois):
            key = (k, roi[2], roi[3])
            if key not in self._parts:
                n = max(roi[2] * roi[3], 1)
                self._parts[key] = (torch.empty(n * 4, dtype=torch.float32, device=self.device),
                                    torch.empty(n, dtype=torch.float32, device=self.device))
            rgba, depth = self._parts[key]
            if self.samples.numel() < len(self.bricks):
                self.samples = torch.zeros(len(self.bricks), dtype=torch.int64, device=self.device)
            self.partials.append(make_partial(roi, rgba, depth, self.samples[k:k + 1]))
        if self.frame is None or self.frame.numel() != self.width * self.height * 4:
            self.frame = torch.empty(self.height, self.width, 4, dtype=torch.float32,
                                     device=self.device)

    def render_partials(self):
        """All partials of the frame in one persistent launch."""
        n = len(self.bricks)
        need = vr_frame_workspace_size(n)
        if getattr(self, "_fws", None) is None or self._fws_bytes < need:
            buf = self.torch.empty(need // 4 + 64, dtype=self.torch.float32, device=self.device)
            self._fws, self._fws_bytes = buf, need
        base = self._fws.data_ptr() + ((-self._fws.data_ptr()) % 256)
        vr_render_partials(self.ctx, self.bricks, self.partials, base, need)

    def render_partials_each(self):
        """One launch per partial (vr_render_partial)."""
        for b, p in zip(self.bricks, self.partials):
            vr_render_partial(self.ctx, b, p)

    def reset_samples(self):
        self.samples.zero_()

    def sample_counts(self):
        """Samples evaluated per brick since the last reset (synchronises)."""
        return self.samples[: len(self.bricks)].cpu().numpy().astype(np.int64)

    def composite(self, bg=(0.0, 0.0, 0.0, 0.0)):
        vr_composite(self.ctx, self.partials, bg, self.frame)
        return self.frame

    def render(self, bg=(0.0, 0.0, 0.0, 0.0)):
        self.render_partials()
        return self.composite(bg)

    def rqc_plan(self):
        """Plan the ray-queue-cycling frame of the current camera (workspace
        and shade buffer allocated here; synchronises)."""
        torch = self.torch
        nbytes = vr_rqc_workspace_size(self.ctx, self.bricks)
        ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.device)
        base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
        total = vr_rqc_plan(self.ctx, self.bricks, base, nbytes)
        shade = torch.empty(max(total, 1), dtype=torch.float32, device=self.device)
        self._rqc = (ws, base, nbytes, shade, total)
        return total

    def render_rqc(self, light_dir, ambient, bg=(0.0, 0.0, 0.0, 0.0), samples=None):
        """The frame by ray-queue cycling with one directional light (plan
        first with :meth:`rqc_plan`); returns the (H, W, 4) frame tensor.
        ``samples``: optional int64 device tensor that counts the primary and
        shadow samples evaluated."""
        _, base, nbytes, shade, total = self._rqc
        vr_render_rqc(self.ctx, self.bricks, light_dir, ambient, bg, base, nbytes, shade, shade.numel() * 4,
                      self.frame, samples)
        return self.frame

    def partial_arrays(self, k):
        """(rgba (h, w, 4), depth (h, w)) torch views of partial k."""
        x0, y0, w, h = self.rois[k]
        rgba, depth = self._parts[(k, w, h)]
        return rgba[: w * h * 4].view(h, w, 4), depth[: w * h].view(h, w)

    def synchronize(self):
        vr_synchronize(self.ctx)

    def close(self):
        if self.ctx is None:
            return
        self.synchronize()
        for b in self.bricks:
            vr_brick_release(b)
        vr_context_release(self.ctx)
        self.ctx = None
        self.bricks = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ batch helper
class BatchRenderer:
    """Plumbing for the batch entry points: bricks (each with its own data:
    a brick x time step x field), cameras, transfer functions and frames
    (a camera, the bricks composited into it and a background).  build()
    allocates every caller-owned buffer as a torch tensor and creates the
    batch; launch() enqueues it."""

    def __init__(self, dt=0.5, ert_eps=2.0 ** -20, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = vr_context_create(device, self.stream)
        vr_set_render_params(self.ctx, dt, ert_eps)
        self.bricks, self._keep, self.cameras, self.cam_dicts = [], [], [], []
        self.tfs, self._tf_keep, self.frame_specs = [], [], []
        self.batch = None

    def add_brick(self, vox, lo, storage=VR_F32, spacing=(1.0, 1.0, 1.0)):
        torch = self.torch
        v = torch.as_tensor(vox).to(self.device, torch.float32).contiguous()
        nz, ny, nx = (int(x) - 2 for x in v.shape)
        nbytes = vr_brick_workspace_size((nx, ny, nz), 1, storage)
        ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.device)
        base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
        h = vr_brick_create(self.ctx, (nx, ny, nz), 1, tuple(float(x) for x in lo), spacing, storage,
                            base, nbytes)
        vr_brick_set_data(h, v, self.ctx)
        self.bricks.append(h)
        self._keep.append((ws, v))
        return len(self.bricks) - 1

    def drop_uploads(self):
        """Free the float32 upload copies once ingest has run (synchronises)."""
        vr_synchronize(self.ctx)
        self._keep = [(ws, None) for ws, _ in self._keep]

    def add_camera(self, cam):
        self.cameras.append(camera_desc(cam))
        self.cam_dicts.append(cam)
        return len(self.cameras) - 1

    def add_tf(self, table, vrange=(0.0, 1.0), opacity_scale=1.0):
        t = self.torch.as_tensor(np.ascontiguousarray(table, dtype=np.float32)).to(self.device)
        self._tf_keep.append(t)
        self.tfs.append(vr_tf_desc(t.data_ptr(), float(vrange[0]), float(vrange[1]),
                                   float(opacity_scale), 0))
        return len(self.tfs) - 1

    def add_frame(self, camera, bricks, tf=0, bg=(0.0, 0.0, 0.0, 0.0)):
        self.frame_specs.append((int(camera), list(bricks), tf, tuple(float(x) for x in bg)))
        return len(self.frame_specs) - 1

    def build(self):
        torch = self.torch
        jobs, frames, self.parts, self.frames, self.job_meta = [], [], [], [], []
        self.samples = torch.zeros(sum(len(b) for _, b, _, _ in self.frame_specs) + 1,
                                   dtype=torch.int64, device=self.device)
        for cam, bricks, tf, bg in self.frame_specs:
            first = len(jobs)
            for k, bi in enumerate(bricks):
                roi = vr_camera_roi(self.ctx, self.bricks[bi], self.cameras[cam])
                n = max(roi[2] * roi[3], 1)
                rgba = torch.empty(n * 4, dtype=torch.float32, device=self.device)
                depth = torch.empty(n, dtype=torch.float32, device=self.device)
                t = tf[k] if isinstance(tf, (list, tuple)) else tf
                part = make_partial(roi, rgba, depth, self.samples[len(jobs):len(jobs) + 1])
                jobs.append(vr_batch_job(self.bricks[bi], cam, int(t), part))
                self.parts.append((roi, rgba, depth))
                self.job_meta.append((bi, cam))
            W, H = self.cameras[cam].width, self.cameras[cam].height
            out = torch.empty(H, W, 4, dtype=torch.float32, device=self.device)
            self.frames.append(out)
            f = vr_batch_frame(cam, first, len(bricks), 0, (C.c_float * 4)(*bg), out.data_ptr())
            frames.append(f)
        need = vr_batch_workspace_size(len(jobs), len(frames))
        self._ws = torch.empty(need // 4 + 64, dtype=torch.float32, device=self.device)
        base = self._ws.data_ptr() + ((-self._ws.data_ptr()) % 256)
        self.batch = vr_batch_create(self.ctx, self.cameras, self.tfs, jobs, frames, base, need)
        self.n_jobs = len(jobs)
        return self

    def launch(self):
        vr_batch_launch(self.batch, self.ctx)

    def autotune(self, reps=3):
        return vr_batch_autotune(self.batch, reps, self.ctx)

    def config(self):
        return vr_batch_config(self.batch, self.ctx)

    def set_groups(self, n_groups):
        """Split the frames into n_groups release groups (vr_batch_set_groups)."""
        vr_batch_set_groups(self.batch, n_groups, self.ctx)

    def group(self, g):
        """(first frame, number of frames) of release group g."""
        return vr_batch_group(self.batch, g, self.ctx)

    def wait_group(self, g, stream=None):
        """Block until group g of the latest launch is written, or make
        `stream` (a torch.cuda.Stream) wait for it on the device."""
        vr_batch_wait_group(self.batch, g, None if stream is None else stream.cuda_stream, self.ctx)

    def group_done(self, g):
        return vr_batch_group_done(self.batch, g, self.ctx)

    def partial_arrays(self, j):
        (x0, y0, w, h), rgba, depth = self.parts[j]
        return rgba[: w * h * 4].view(h, w, 4), depth[: w * h].view(h, w)

    def synchronize(self):
        vr_synchronize(self.ctx)

    def close(self):
        if self.ctx is None:
            return
        vr_synchronize(self.ctx)
        if self.batch is not None:
            vr_batch_release(self.batch)
            self.batch = None
        for b in self.bricks:
            vr_brick_release(b)
        vr_context_release(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------ time-step streaming
class StreamRenderer:
    """Plays a time series of bricked volumes with only ``slots`` time steps
    resident on the device.  ``steps[t]`` is a list of (voxels, lo) per brick
    (ghost-padded float32 arrays, the same brick boxes at every step); the
    arrays are copied once into pinned host memory, from which the library
    uploads a step when it is needed (on its own copy stream)."""

    def __init__(self, steps, tf, vrange=(0.0, 1.0), opacity_scale=1.0, dt=0.5, slots=2,
                 ert_eps=2.0 ** -20, storage=VR_F32, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = vr_context_create(device, self.stream)
        self.tf = torch.as_tensor(np.ascontiguousarray(tf, dtype=np.float32)).to(self.device)
        vr_set_transfer_function(self.ctx, self.tf, TF_ENTRIES, vrange[0], vrange[1], opacity_scale)
        vr_set_render_params(self.ctx, dt, ert_eps)
        self.n_steps, self.n_bricks, self.slots = len(steps), len(steps[0]), int(slots)
        descs = []
        for vox, lo in steps[0]:
            nz, ny, nx = (int(v) - 2 for v in np.shape(vox))
            descs.append(((nx, ny, nz), tuple(float(x) for x in lo), (1.0, 1.0, 1.0), storage))
        self._host = [torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).pin_memory()
                      for step in steps for v, _ in step]
        nbytes = vr_timeseries_workspace_size(descs, self.slots)
        self._ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.device)
        base = self._ws.data_ptr() + ((-self._ws.data_ptr()) % 256)
        self.ts = vr_timeseries_create(self.ctx, descs, [h.data_ptr() for h in self._host], self.n_steps,
                                       self.slots, base, nbytes)
        self._bufs = {}
        self.frame = None

    def set_camera(self, cam):
        set_camera(self.ctx, cam)
        self.width, self.height = int(cam["width"]), int(cam["height"])
        self.frame = self.torch.empty(self.height, self.width, 4, dtype=self.torch.float32, device=self.device)

    def prefetch(self, step):
        vr_timeseries_prefetch(self.ts, step, self.ctx)

    def render(self, step, bg=(0.0, 0.0, 0.0, 0.0), prefetch=None):
        """Frame of time step ``step`` (loaded now if it is not resident);
        ``prefetch``: a step whose upload should start behind this frame."""
        torch = self.torch
        bricks = vr_timeseries_acquire(self.ts, step, self.n_bricks, self.ctx)
        parts = []
        for k, b in enumerate(bricks):
            roi = vr_partial_roi(self.ctx, b)
            key = (k, roi[2], roi[3])
            if key not in self._bufs:
                n = max(roi[2] * roi[3], 1)
                self._bufs[key] = (torch.empty(n * 4, dtype=torch.float32, device=self.device),
                                   torch.empty(n, dtype=torch.float32, device=self.device))
            rgba, depth = self._bufs[key]
            parts.append(make_partial(roi, rgba, depth))
        need = vr_frame_workspace_size(len(bricks))
        if getattr(self, "_fws", None) is None or self._fws_bytes < need:
            self._fws = torch.empty(need // 4 + 64, dtype=torch.float32, device=self.device)
            self._fws_bytes = need
        base = self._fws.data_ptr() + ((-self._fws.data_ptr()) % 256)
        vr_render_partials(self.ctx, bricks, parts, base, need)
        vr_composite(self.ctx, parts, bg, self.frame)
        # after the frame's work is enqueued: a load that evicts this step's
        # slot waits for it
        if prefetch is not None:
            vr_timeseries_prefetch(self.ts, prefetch, self.ctx)
        return self.frame

    def stats(self):
        return vr_timeseries_stats(self.ts, self.slots, self.ctx)

    def synchronize(self):
        vr_synchronize(self.ctx)

    def close(self):
        if self.ctx is None:
            return
        vr_synchronize(self.ctx)
        vr_timeseries_release(self.ts, self.ctx)
        vr_context_release(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- differentiable path
class DiffRenderer:
    """Differentiable frame of a bricked volume: ``render(tf, volume, cam)``
    returns the composited frame as a torch tensor whose backward runs the
    library's composite backward and adjoint march, giving gradients with
    respect to the (256, 4) transfer-function table and the (nz, ny, nx)
    global voxel array.  ``boxes`` = [(lo, hi), ...] integer owned boxes of
    the global grid (x, y, z order); early termination is off."""

    def __init__(self, vol_dims, boxes, vrange=(0.0, 1.0), opacity_scale=1.0, dt=0.5,
                 interval=64, storage=VR_F32, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = vr_context_create(device, self.stream)
        self.vol_dims = tuple(int(v) for v in vol_dims)
        self.vrange, self.opacity_scale, self.dt = vrange, float(opacity_scale), float(dt)
        self.interval = int(interval)
        self.batched_backward = True     # all bricks' checkpointed forwards, and adjoints, in one launch each
        self.bricks, self.los, self._ws = [], [], []
        vr_set_render_params(self.ctx, self.dt, 0.0)
        for lo, hi in boxes:
            dims = tuple(int(h - l) for l, h in zip(lo, hi))
            nbytes = vr_brick_workspace_size(dims, 1, storage)
            ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.device)
            base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
            self.bricks.append(vr_brick_create(self.ctx, dims, 1, tuple(float(x) for x in lo),
                                               (1.0, 1.0, 1.0), storage, base, nbytes))
            self.los.append(tuple(int(x) for x in lo))
            self._ws.append(ws)

    def _load(self, tf, volume, cam):
        vr_set_transfer_function(self.ctx, tf, TF_ENTRIES, self.vrange[0], self.vrange[1],
                                 self.opacity_scale)
        # the bricks are re-gathered unless the volume is the tensor of the
        # last gather (held here, so its memory cannot be another tensor's)
        # with an unchanged version counter (in-place updates bump it)
        last = getattr(self, "_loaded", None)
        if (last is None or last[0].data_ptr() != volume.data_ptr() or last[1] != volume._version or
                tuple(last[0].shape) != tuple(volume.shape)):
            for b, lo in zip(self.bricks, self.los):
                vr_brick_set_data_global(b, volume, self.vol_dims, lo, self.ctx)
            self._loaded = (volume, volume._version)
        set_camera(self.ctx, cam)

    def render(self, tf, volume, cam, bg=(0.0, 0.0, 0.0, 0.0)):
        return _RenderFn.apply(tf, volume, self, cam, tuple(float(x) for x in bg))

    def close(self):
        if self.ctx is None:
            return
        vr_synchronize(self.ctx)
        self._loaded = None
        for b in self.bricks:
            vr_brick_release(b)
        vr_context_release(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class RenderFn(torch.autograd.Function):
        @staticmethod
        def forward(fctx, tf, volume, dr, cam, bg):
            torch_ = dr.torch
            tf_c = tf.detach().to(dr.device, torch_.float32).contiguous()
            vol_c = volume.detach().to(dr.device, torch_.float32).contiguous()
            dr._load(tf_c, vol_c, cam)
            W, H = int(cam["width"]), int(cam["height"])
            parts, keep, ckpts = [], [], []
            for b in dr.bricks:
                roi = vr_partial_roi(dr.ctx, b)
                n = max(roi[2] * roi[3], 1)
                rgba = torch_.empty(n * 4, dtype=torch_.float32, device=dr.device)
                depth = torch_.empty(n, dtype=torch_.float32, device=dr.device)
                part = make_partial(roi, rgba, depth)
                nb = max(vr_checkpoint_size(dr.ctx, b, part, dr.interval), 4)
                ck = torch_.empty(nb // 4, dtype=torch_.float32, device=dr.device)
                if not dr.batched_backward:
                    vr_render_partial_checkpointed(dr.ctx, b, part, dr.interval, ck, nb)
                parts.append(part)
                keep.append((rgba, depth))
                ckpts.append((ck, nb))
            if dr.batched_backward:     # every brick's checkpointed forward in one launch
                need = vr_checkpointed_workspace_size(len(dr.bricks))
                ws = torch_.empty(need // 4 + 64, dtype=torch_.float32, device=dr.device)
                vr_render_partials_checkpointed(dr.ctx, dr.bricks, parts, dr.interval, ckpts,
                                                ws.data_ptr() + ((-ws.data_ptr()) % 256), need)
                keep.append(ws)
            out = torch_.empty(H, W, 4, dtype=torch_.float32, device=dr.device)
            vr_composite(dr.ctx, parts, bg, out)
            fctx.dr, fctx.cam, fctx.bg = dr, cam, bg
            fctx.parts, fctx.keep, fctx.ckpts = parts, keep, ckpts
            fctx.save_for_backward(tf_c, vol_c)
            return out

        @staticmethod
        def backward(fctx, g_out):
            dr = fctx.dr
            torch_ = dr.torch
            tf_c, vol_c = fctx.saved_tensors
            # another forward may have changed the context state since
            dr._load(tf_c, vol_c, fctx.cam)
            g = g_out.detach().to(dr.device, torch_.float32).contiguous()
            d_parts = [torch_.empty(max(p.w * p.h, 1) * 4, dtype=torch_.float32, device=dr.device)
                       for p in fctx.parts]
            vr_composite_backward(dr.ctx, fctx.parts, fctx.bg, g, d_parts)
            grad_tf = torch_.zeros(TF_ENTRIES, 4, dtype=torch_.float32, device=dr.device)
            grad_vol = torch_.zeros_like(vol_c)
            if not dr.batched_backward:
                for b, lo, part, (ck, nb), dp in zip(dr.bricks, dr.los, fctx.parts, fctx.ckpts, d_parts):
                    vr_render_partial_backward(dr.ctx, b, part, dr.interval, ck, nb, dp, grad_tf, grad_vol,
                                               dr.vol_dims, lo)
                return grad_tf, grad_vol, None, None, None
            # all bricks' adjoints in one launch (per storage precision)
            need = vr_backward_workspace_size(len(dr.bricks))
            ws = torch_.empty(need // 4 + 64, dtype=torch_.float32, device=dr.device)
            base = ws.data_ptr() + ((-ws.data_ptr()) % 256)
            vr_render_partials_backward(dr.ctx, dr.bricks, fctx.parts, dr.interval, fctx.ckpts, d_parts, grad_tf,
                                        grad_vol, dr.vol_dims, dr.los, base, need)
            fctx.bwd_ws = ws      # borrowed until the enqueued work has run (the stream orders its reuse)
            return grad_tf, grad_vol, None, None, None

    return RenderFn


class _LazyFn:
    _fn = None

    def apply(self, *args):
        if _LazyFn._fn is None:
            _LazyFn._fn = _autograd_function()
        return _LazyFn._fn.apply(*args)


_RenderFn = _LazyFn()
