"""CPU oracle for the fisheye Gaussian-splatting rasterizer (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The
rendering library (``paper_2409_04751_amd``) never imports it, and it imports
nothing from the library: scene, pose and camera arguments are any objects
with the fields of the input generators' dataclasses.

All arithmetic lives in ``fgs_oracle.c`` (double precision); this file only
marshals numpy arrays.  See that file's header for the paper passages each
step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fgs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TILE = 16


_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc: IEEE double, no FMA contraction, OpenMP.
    With sanitize, a separate copy instrumented with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only; loading it needs the ASan
    runtime preloaded)."""
    out = _SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        extra = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"])
        cmd = ["gcc", *extra, "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-o", out + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return out


class _Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("near_dist", ctypes.c_double), ("theta_max", ctypes.c_double), ("model", ctypes.c_int32)]


class _Tol(ctypes.Structure):
    _fields_ = [("tol_alpha", ctypes.c_double), ("tol_T", ctypes.c_double), ("tol_clamp", ctypes.c_double),
                ("err_scale", ctypes.c_double)]


_lib = None


def lib():
    """The oracle library; FGS_ORACLE_LIB=sanitized loads the instrumented
    copy (built by build(sanitize=True))."""
    global _lib
    if _lib is None:
        if os.environ.get("FGS_ORACLE_LIB") == "sanitized":
            path = _SAN_LIB
        else:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        _lib = ctypes.CDLL(path)
        _lib.orc_count_pairs.restype = ctypes.c_int64
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _cam(cam) -> _Cam:
    return _Cam(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.near, cam.theta_max, cam.model)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _params(scene, pose):
    """Parameters as doubles (float32 inputs convert exactly)."""
    return (_f64(scene.means), _f64(scene.scales), _f64(scene.quats), _f64(scene.opacity), _f64(scene.sh),
            _f64(pose.R).reshape(9), _f64(pose.t).reshape(3))


# -- math primitives -------------------------------------------------------

def project(p, fx, fy, cx, cy) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(2)
    lib().orc_project(_p(p), ctypes.c_double(fx), ctypes.c_double(fy), ctypes.c_double(cx), ctypes.c_double(cy),
                      _p(out))
    return out


def jacobian(p, fx, fy) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    J = np.zeros(6)
    lib().orc_jacobian(_p(p), ctypes.c_double(fx), ctypes.c_double(fy), _p(J))
    return J.reshape(2, 3)


def jacobian_grad(p, fx, fy) -> np.ndarray:
    """[3, 2, 3]: d J / d(x_c, y_c, z_c)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    dJ = np.zeros(18)
    lib().orc_jacobian_grad(_p(p), ctypes.c_double(fx), ctypes.c_double(fy), _p(dJ))
    return dJ.reshape(3, 2, 3)


def project_model(model: int, p, fx, fy, cx, cy) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(2)
    lib().orc_project_model(ctypes.c_int(model), _p(p), ctypes.c_double(fx), ctypes.c_double(fy),
                            ctypes.c_double(cx), ctypes.c_double(cy), _p(out))
    return out


def jacobian_model(model: int, p, fx, fy) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    J = np.zeros(6)
    lib().orc_jacobian_model(ctypes.c_int(model), _p(p), ctypes.c_double(fx), ctypes.c_double(fy), _p(J))
    return J.reshape(2, 3)


def jacobian_grad_model(model: int, p, fx, fy) -> np.ndarray:
    """[3, 2, 3]: d J / d(x_c, y_c, z_c) for camera model `model`."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    dJ = np.zeros(18)
    lib().orc_jacobian_grad_model(ctypes.c_int(model), _p(p), ctypes.c_double(fx), ctypes.c_double(fy), _p(dJ))
    return dJ.reshape(3, 2, 3)


def cull_angle(model: int, p) -> float:
    p = np.ascontiguousarray(p, dtype=np.float64)
    f = lib().orc_cull_angle
    f.restype = ctypes.c_double
    return float(f(ctypes.c_int(model), _p(p)))


def sh_basis(degree: int, d) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(16)
    lib().orc_sh_basis(ctypes.c_int(degree), _p(d), _p(out))
    return out[: (degree + 1) ** 2]


# -- pipeline --------------------------------------------------------------

# tie bits: 1 the radius or rect (fp64 decisions) within 1e-9 of a boundary;
# 2 another rounding of the float record keeps other tiles (fp32 recipe);
# 4 the fp64 tight rule's tiles move with its margins (rule only)
TIE_RECT, TIE_RECORD, TIE_RULE = 1, 2, 4

_BIN_MODE = {"rect": 0, "tight": 1, "tight64": 2}


def preprocess(scene, pose, cam, binning: str = "tight") -> dict:
    """binning "tight": each Gaussian keeps only the tiles of its 3-sigma rect
    that its (margin-grown) alpha >= 1/255 ellipse reaches, decided by the
    binary32 key recipe from the float record of the splat; "tight64": the
    same rule decided in fp64 (its definition); "rect": every tile of the rect
    (vanilla lists).  Images and gradients are the same."""
    assert binning in _BIN_MODE
    n = scene.n
    o = dict(
        visible=np.zeros(n, np.uint8), mu_p=np.zeros((n, 2)), conic=np.zeros((n, 3)), rgb=np.zeros((n, 3)),
        clamped=np.zeros(n, np.uint8), radius=np.zeros(n, np.int32), rect=np.zeros((n, 4), np.int32),
        depth=np.zeros(n, np.float32), tiles=np.zeros(n, np.uint32), tie=np.zeros(n, np.uint8),
        cov2d=np.zeros((n, 3)))
    means, scales, quats, opac, sh, R, t = _params(scene, pose)
    c = _cam(cam)
    lib().orc_preprocess(ctypes.c_int64(n), _p(means), _p(scales), _p(quats), _p(opac), _p(sh),
                         ctypes.c_int(scene.sh_degree), _p(R), _p(t), ctypes.byref(c), _p(o["visible"]),
                         _p(o["mu_p"]), _p(o["conic"]), _p(o["rgb"]), _p(o["clamped"]), _p(o["radius"]),
                         _p(o["rect"]), _p(o["depth"]), _p(o["tiles"]), _p(o["tie"]), _p(o["cov2d"]))
    o["opacity"] = opac
    o["binning"] = binning
    if binning == "tight":
        lib().orc_tighten32(ctypes.c_int64(n), _p(o["visible"]), _p(o["mu_p"]), _p(o["conic"]), _p(o["cov2d"]),
                            _p(opac), _p(o["rect"]), _p(o["tiles"]), _p(o["tie"]))
    elif binning == "tight64":
        lib().orc_tighten(ctypes.c_int64(n), _p(o["visible"]), _p(o["mu_p"]), _p(o["conic"]), _p(opac),
                          _p(o["rect"]), _p(o["tiles"]), _p(o["tie"]))
    return o


def tight_alternatives(pre: dict, i: int, max_alt: int = 64) -> list:
    """Kept tile columns per rect row of Gaussian i under the binary32 recipe,
    one [rows, 2] array per rounding of its float record that the renderer's
    fp64 geometry could produce (one array unless a value is near a float
    rounding midpoint)."""
    rect = np.ascontiguousarray(pre["rect"][i], dtype=np.int32)
    rows = int(rect[3] - rect[1])
    out = np.zeros((max_alt, max(rows, 1), 2), np.int32)
    cnt = lib().orc_tight32_alternatives(_p(np.ascontiguousarray(pre["mu_p"][i])),
                                         _p(np.ascontiguousarray(pre["conic"][i])),
                                         _p(np.ascontiguousarray(pre["cov2d"][i])),
                                         ctypes.c_double(float(pre["opacity"][i])), _p(rect), ctypes.c_int(max_alt),
                                         _p(out))
    return [out[k, :rows] for k in range(cnt)]


def bin_and_sort(pre: dict, cam) -> dict:
    n = pre["visible"].shape[0]
    k = lib().orc_count_pairs(ctypes.c_int64(n), _p(pre["visible"]), _p(pre["tiles"]))
    keys = np.zeros(max(k, 1), np.uint64)
    vals = np.zeros(max(k, 1), np.uint32)
    ranges = np.zeros((cam.tiles_x * cam.tiles_y, 2), np.uint32)
    lib().orc_bin(ctypes.c_int64(n), _p(pre["visible"]), _p(pre["rect"]), _p(pre["depth"]),
                  ctypes.c_int32(cam.width), ctypes.c_int32(cam.height), ctypes.c_int64(k), _p(keys), _p(vals),
                  _p(ranges), ctypes.c_int(_BIN_MODE[pre.get("binning", "rect")]), _p(pre["mu_p"]),
                  _p(pre["conic"]), _p(pre["cov2d"]), _p(pre["opacity"]))
    return dict(K=int(k), keys=keys[:k], vals=vals[:k], ranges=ranges)


# flag bands: no fixed margin, twice the binary32 error bound of each
# decision (fgs_oracle.c, "Ambiguity flags")
DEFAULT_TOL = (0.0, 0.0, 0.0, 2.0)


def blend(pre: dict, bins: dict, cam, bg=(0.0, 0.0, 0.0), tol=DEFAULT_TOL) -> dict:
    H, W = cam.height, cam.width
    image = np.zeros((3, H, W))
    T = np.zeros((H, W))
    last = np.zeros((H, W), np.int32)
    flags = np.zeros((H, W), np.uint8)
    evals = ctypes.c_int64(0)
    bgv = _f32(bg)
    vals = bins["vals"] if bins["K"] > 0 else np.zeros(1, np.uint32)
    tl = _Tol(*tol)
    lib().orc_blend(ctypes.c_int32(W), ctypes.c_int32(H), _p(bins["ranges"]), _p(vals), _p(pre["mu_p"]),
                    _p(pre["conic"]), _p(pre["opacity"]), _p(pre["rgb"]), _p(bgv), ctypes.byref(tl), _p(image),
                    _p(T), _p(last), _p(flags), ctypes.byref(evals))
    return dict(image=image, T_final=T, last=last, flags=flags, evals=int(evals.value))


def blend_bruteforce(pre: dict, cam, bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    n = pre["visible"].shape[0]
    image = np.zeros((3, cam.height, cam.width))
    tl = _Tol(*DEFAULT_TOL)
    lib().orc_blend_bruteforce(ctypes.c_int64(n), ctypes.c_int32(cam.width), ctypes.c_int32(cam.height),
                               _p(pre["visible"]), _p(pre["rect"]), _p(pre["depth"]), _p(pre["mu_p"]),
                               _p(pre["conic"]), _p(pre["opacity"]), _p(pre["rgb"]), _p(_f32(bg)),
                               ctypes.byref(tl), _p(image))
    return image


def blend_backward(pre: dict, bins: dict, cam, dL_dimg, bg=(0.0, 0.0, 0.0), abs_sums: bool = False) -> dict:
    """Per-Gaussian 2D gradients; with abs_sums also `abs` [n, 9] (operand
    magnitudes summed over pixels) and `pos` [n, 9] (sensitivity to the pixel
    offset) for (mu_x, mu_y, A, B, C, o, r, g, b)."""
    n = pre["visible"].shape[0]
    g = dict(mu_p=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n), rgb=np.zeros((n, 3)))
    if abs_sums:
        g["abs18"] = np.zeros((n, 18))
    vals = bins["vals"] if bins["K"] > 0 else np.zeros(1, np.uint32)
    lib().orc_blend_backward(ctypes.c_int32(cam.width), ctypes.c_int32(cam.height), _p(bins["ranges"]), _p(vals),
                             _p(pre["mu_p"]), _p(pre["conic"]), _p(pre["opacity"]), _p(pre["rgb"]), _p(_f32(bg)),
                             _p(_f32(dL_dimg)), _p(g["mu_p"]), _p(g["conic"]), _p(g["opacity"]), _p(g["rgb"]),
                             _p(g["abs18"]) if abs_sums else None)
    if abs_sums:
        g["abs"] = np.ascontiguousarray(g["abs18"][:, :9])
        g["pos"] = np.ascontiguousarray(g["abs18"][:, 9:])
        del g["abs18"]
    return g


def preprocess_backward(scene, pose, cam, pre: dict, g2d: dict) -> dict:
    n = scene.n
    S = scene.sh.shape[0]
    out = dict(means=np.zeros((3, n)), scales=np.zeros((3, n)), quats=np.zeros((4, n)), opacity=np.zeros(n),
               sh=np.zeros((S, n)))
    means, scales, quats, opac, sh, R, t = _params(scene, pose)
    c = _cam(cam)
    lib().orc_preprocess_backward(ctypes.c_int64(n), _p(means), _p(scales), _p(quats), _p(opac), _p(sh),
                                  ctypes.c_int(scene.sh_degree), _p(R), _p(t), ctypes.byref(c),
                                  _p(pre["visible"]), _p(np.ascontiguousarray(g2d["mu_p"])),
                                  _p(np.ascontiguousarray(g2d["conic"])), _p(np.ascontiguousarray(g2d["opacity"])),
                                  _p(np.ascontiguousarray(g2d["rgb"])), _p(out["means"]), _p(out["scales"]),
                                  _p(out["quats"]), _p(out["opacity"]), _p(out["sh"]))
    return out


def chain_error_scale(scene, pose, cam, pre: dict, g2d_abs) -> dict:
    """The rounding-error scale of each parameter gradient: the preprocess
    backward is linear in the nine 2D gradients of a Gaussian, dL/dp = M g2d,
    so an error of g2d bounded by its operand magnitudes `g2d_abs` [n, 9]
    (mu_x, mu_y, A, B, C, o, r, g, b) reaches dL/dp as at most |M| g2d_abs.
    |M| is taken column by column, one backward per unit 2D gradient."""
    n = scene.n
    out = None
    for k in range(9):
        unit = np.zeros((n, 9))
        unit[:, k] = 1.0
        g2d = dict(mu_p=np.ascontiguousarray(unit[:, 0:2]), conic=np.ascontiguousarray(unit[:, 2:5]),
                   opacity=np.ascontiguousarray(unit[:, 5]), rgb=np.ascontiguousarray(unit[:, 6:9]))
        col = preprocess_backward(scene, pose, cam, pre, g2d)
        w = np.asarray(g2d_abs)[:, k]
        term = {b: np.abs(v) * w for b, v in col.items()}
        out = term if out is None else {b: out[b] + term[b] for b in out}
    return out


def render(scene, pose, cam, bg=(0.0, 0.0, 0.0), tol=DEFAULT_TOL, binning: str = "tight") -> dict:
    """Full forward: preprocess, bin + sort, blend."""
    pre = preprocess(scene, pose, cam, binning)
    bins = bin_and_sort(pre, cam)
    out = blend(pre, bins, cam, bg, tol)
    out.update(pre=pre, bins=bins)
    return out


def render_backward(scene, pose, cam, fwd: dict, dL_dimg, bg=(0.0, 0.0, 0.0), abs_sums: bool = False) -> dict:
    g2d = blend_backward(fwd["pre"], fwd["bins"], cam, dL_dimg, bg, abs_sums)
    grads = preprocess_backward(scene, pose, cam, fwd["pre"], g2d)
    grads["g2d"] = g2d
    return grads
