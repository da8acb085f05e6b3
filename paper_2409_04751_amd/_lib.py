"""ctypes binding of libfgs (include/fgs.h).

Argument marshalling only: every step of the rasterizer runs in the HIP
library.  The names match the C entry points.  Importing this module loads
``libfgs.so`` from the package directory and raises if it is missing; there
is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfgs.so")

FGS_OK = 0
FGS_ERR_ARG = -1
FGS_ERR_WORKSPACE = -2
FGS_ERR_HIP = -3
FGS_ERR_OVERFLOW = -4
FGS_MODEL_EQUIDISTANT = 0
FGS_MODEL_PINHOLE = 1
FGS_MODEL_PANORAMA = 2
FGS_MODEL_EQUISOLID = 3
FGS_MODEL_ORTHOGRAPHIC = 4
FGS_MODEL_STEREOGRAPHIC = 5
FGS_SAVE_PIXEL_STATE = 1
FGS_RECT_BINNING = 2
FGS_MAX_BATCH = 8
FGS_L1_PARTIALS = 1024

c_size = ctypes.c_size_t


class fgs_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("model", ctypes.c_int32),
                ("near_dist", ctypes.c_double), ("theta_max", ctypes.c_double)]


class fgs_pose(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3)]


class fgs_gaussians(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("sh_degree", ctypes.c_int32)]


class fgs_grads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("means2d", ctypes.c_void_p),
                ("accumulate", ctypes.c_int32)]


class fgs_layout(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32), ("k_capacity", ctypes.c_int64),
                ("bytes", c_size), ("splats", c_size), ("colors", c_size), ("depth_keys", c_size), ("tiles", c_size), ("rects", c_size),
                ("radii", c_size), ("depth_order", c_size), ("offsets", c_size), ("tile_keys", c_size),
                ("tile_ids", c_size), ("ranges", c_size), ("grad2d", c_size), ("pixel_T", c_size),
                ("pixel_last", c_size), ("counters", c_size)]


FGS_PROF_MAX_KERNELS = 32


class fgs_profile(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("names", ctypes.c_char_p * FGS_PROF_MAX_KERNELS),
                ("launches", ctypes.c_int64 * FGS_PROF_MAX_KERNELS),
                ("total_ms", ctypes.c_double * FGS_PROF_MAX_KERNELS)]


# Exported symbols, argtypes and restype.  Kept in one table so a CPU test can
# check it against the header.
SIGNATURES = {
    "fgs_version": ([], ctypes.c_char_p),
    "fgs_last_error": ([], ctypes.c_char_p),
    "fgs_workspace_bytes": ([ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(c_size)],
                            ctypes.c_int),
    "fgs_workspace_layout": ([ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, c_size, ctypes.POINTER(fgs_layout)],
                             ctypes.c_int),
    "fgs_render_forward": ([ctypes.POINTER(fgs_gaussians), ctypes.POINTER(fgs_pose), ctypes.POINTER(fgs_camera),
                            ctypes.POINTER(ctypes.c_float), ctypes.c_uint32, ctypes.c_void_p, c_size, ctypes.c_void_p,
                            ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p], ctypes.c_int),
    "fgs_render_backward": ([ctypes.POINTER(fgs_gaussians), ctypes.POINTER(fgs_pose), ctypes.POINTER(fgs_camera),
                             ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, c_size, ctypes.c_void_p,
                             ctypes.POINTER(fgs_grads), ctypes.c_void_p], ctypes.c_int),
    "fgs_deterministic_workspace_bytes": ([ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(c_size)], ctypes.c_int),
    "fgs_render_backward_deterministic": ([ctypes.POINTER(fgs_gaussians), ctypes.POINTER(fgs_pose),
                                           ctypes.POINTER(fgs_camera), ctypes.POINTER(ctypes.c_float),
                                           ctypes.c_void_p, c_size, ctypes.c_void_p, ctypes.POINTER(fgs_grads),
                                           ctypes.c_void_p, c_size, ctypes.c_void_p], ctypes.c_int),
    "fgs_batch_workspace_bytes": ([ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(fgs_camera), ctypes.c_int64,
                                   ctypes.POINTER(c_size)], ctypes.c_int),
    "fgs_render_forward_batch": ([ctypes.POINTER(fgs_gaussians), ctypes.c_int32, ctypes.POINTER(fgs_pose),
                                  ctypes.POINTER(fgs_camera), ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, c_size,
                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p], ctypes.c_int),
    "fgs_l1_loss": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_void_p], ctypes.c_int),
    "fgs_l1_loss_backward": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p], ctypes.c_int),
    "fgs_l1_loss_noalloc": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
                            ctypes.c_int),
    "fgs_spatial_order_workspace_bytes": ([ctypes.c_int64, ctypes.POINTER(c_size)], ctypes.c_int),
    "fgs_spatial_order": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, c_size,
                           ctypes.c_void_p], ctypes.c_int),
    "fgs_gather_planes": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                           ctypes.c_void_p], ctypes.c_int),
    "fgs_profile_enable": ([ctypes.c_int32], ctypes.c_int),
    "fgs_profile_read": ([ctypes.POINTER(fgs_profile)], ctypes.c_int),
}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(_LIB_PATH)
        for name, (argtypes, restype) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = argtypes
            fn.restype = restype
        _lib = L
    return _lib


class FgsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fgs error {code}: {msg}")
        self.code = code


def fgs_version() -> str:
    return lib().fgs_version().decode()


def fgs_last_error() -> str:
    return lib().fgs_last_error().decode()


def check(rc: int) -> int:
    if rc != FGS_OK:
        raise FgsError(rc, fgs_last_error())
    return rc


def fgs_workspace_bytes(n: int, width: int, height: int, k_capacity: int) -> int:
    out = c_size(0)
    check(lib().fgs_workspace_bytes(n, width, height, k_capacity, ctypes.byref(out)))
    return int(out.value)


def fgs_workspace_layout(n: int, width: int, height: int, nbytes: int) -> fgs_layout:
    out = fgs_layout()
    check(lib().fgs_workspace_layout(n, width, height, nbytes, ctypes.byref(out)))
    return out


def _bg(bg):
    return (ctypes.c_float * 3)(*[float(v) for v in bg])


def fgs_render_forward(g: fgs_gaussians, pose: fgs_pose, cam: fgs_camera, bg, flags: int, workspace: int,
                       workspace_bytes: int, out_rgb: int, stream: int) -> tuple[int, int]:
    """Returns (return code, K).  Does not raise: FGS_ERR_WORKSPACE is part of
    the protocol (grow and retry)."""
    k = ctypes.c_int64(0)
    rc = lib().fgs_render_forward(ctypes.byref(g), ctypes.byref(pose), ctypes.byref(cam), _bg(bg), flags, workspace,
                                  workspace_bytes, out_rgb, ctypes.byref(k), stream)
    return rc, int(k.value)


def fgs_render_backward(g: fgs_gaussians, pose: fgs_pose, cam: fgs_camera, bg, workspace: int, workspace_bytes: int,
                        dL_drgb: int, grads: fgs_grads, stream: int) -> int:
    return lib().fgs_render_backward(ctypes.byref(g), ctypes.byref(pose), ctypes.byref(cam), _bg(bg), workspace,
                                     workspace_bytes, dL_drgb, ctypes.byref(grads), stream)


def fgs_deterministic_workspace_bytes(n: int, k_capacity: int) -> int:
    out = c_size(0)
    check(lib().fgs_deterministic_workspace_bytes(n, k_capacity, ctypes.byref(out)))
    return int(out.value)


def fgs_render_backward_deterministic(g: fgs_gaussians, pose: fgs_pose, cam: fgs_camera, bg, workspace: int,
                                      workspace_bytes: int, dL_drgb: int, grads: fgs_grads, det_workspace: int,
                                      det_workspace_bytes: int, stream: int) -> int:
    return lib().fgs_render_backward_deterministic(ctypes.byref(g), ctypes.byref(pose), ctypes.byref(cam), _bg(bg),
                                                   workspace, workspace_bytes, dL_drgb, ctypes.byref(grads),
                                                   det_workspace, det_workspace_bytes, stream)


def fgs_batch_workspace_bytes(n: int, cams, k_capacity: int) -> int:
    arr = (fgs_camera * len(cams))(*cams)
    out = c_size(0)
    check(lib().fgs_batch_workspace_bytes(n, len(cams), arr, k_capacity, ctypes.byref(out)))
    return int(out.value)


def fgs_render_forward_batch(g: fgs_gaussians, poses, cams, bgs, workspace: int, workspace_bytes: int, out_rgb,
                             stream: int) -> tuple[int, list[int], int]:
    """Returns (return code, K per view, K total); does not raise."""
    nv = len(cams)
    P = (fgs_pose * nv)(*poses)
    C = (fgs_camera * nv)(*cams)
    B = (ctypes.c_float * (3 * nv))(*[float(x) for bg in bgs for x in bg])
    O = (ctypes.c_void_p * nv)(*out_rgb)
    kv = (ctypes.c_int64 * nv)()
    kt = ctypes.c_int64(0)
    rc = lib().fgs_render_forward_batch(ctypes.byref(g), nv, P, C, B, workspace, workspace_bytes, O, kv,
                                        ctypes.byref(kt), stream)
    return rc, [int(x) for x in kv], int(kt.value)


def fgs_l1_loss(image: int, target: int, count: int, partials: int, loss: int, stream: int) -> None:
    check(lib().fgs_l1_loss(image, target, count, partials, loss, stream))


def fgs_l1_loss_noalloc(image: int, target: int, count: int, loss: int, stream: int) -> int:
    """Returns the library's status code (the caller checks it)."""
    return lib().fgs_l1_loss_noalloc(image, target, count, loss, stream)


def fgs_l1_loss_backward(image: int, target: int, count: int, dL_dloss: int, dL_dimage: int, stream: int) -> None:
    check(lib().fgs_l1_loss_backward(image, target, count, dL_dloss, dL_dimage, stream))


def fgs_spatial_order_workspace_bytes(n: int) -> int:
    out = c_size(0)
    check(lib().fgs_spatial_order_workspace_bytes(n, ctypes.byref(out)))
    return int(out.value)


def fgs_spatial_order(means: int, n: int, order: int, workspace: int, workspace_bytes: int, stream: int) -> None:
    check(lib().fgs_spatial_order(means, n, order, workspace, workspace_bytes, stream))


def fgs_gather_planes(src: int, dst: int, planes: int, n: int, order: int, stream: int) -> None:
    check(lib().fgs_gather_planes(src, dst, planes, n, order, stream))


def fgs_profile_enable(on: bool) -> None:
    check(lib().fgs_profile_enable(1 if on else 0))


def fgs_profile_read() -> dict:
    """{kernel name: (launches, total ms)} for kernels launched while enabled."""
    out = fgs_profile()
    check(lib().fgs_profile_read(ctypes.byref(out)))
    return {out.names[k].decode(): (int(out.launches[k]), float(out.total_ms[k])) for k in range(out.count)
            if out.launches[k] > 0}
