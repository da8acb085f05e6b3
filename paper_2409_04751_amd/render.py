"""PyTorch-facing entry points.

PyTorch supplies device memory (tensors, the workspace) and the stream; every
step of the rasterizer runs in libfgs through the C ABI.  Tensors must be
float32, contiguous, on the GPU, in the structure-of-arrays layout of
include/fgs.h: means [3, N], scales [3, N], quats [4, N], opacities [N],
sh [S, N].
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib as L

FGS_SAVE_PIXEL_STATE = L.FGS_SAVE_PIXEL_STATE


def _check_param(name, t, rows, n):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous float32")
    shape = (rows, n) if rows else (n,)
    if tuple(t.shape) != shape:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")


def gaussians_struct(means, scales, quats, opacities, sh, sh_degree: int) -> L.fgs_gaussians:
    n = int(means.shape[1]) if means.dim() == 2 else -1
    S = 3 * (sh_degree + 1) ** 2
    _check_param("means", means, 3, n)
    _check_param("scales", scales, 3, n)
    _check_param("quats", quats, 4, n)
    _check_param("opacities", opacities, 0, n)
    _check_param("sh", sh, S, n)
    return L.fgs_gaussians(means.data_ptr(), scales.data_ptr(), quats.data_ptr(), opacities.data_ptr(),
                           sh.data_ptr(), n, sh_degree)


def camera_struct(cam) -> L.fgs_camera:
    return L.fgs_camera(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy),
                        int(getattr(cam, "model", 0)), float(cam.near), float(cam.theta_max))


def pose_struct(pose) -> L.fgs_pose:
    R = [float(v) for v in torch.as_tensor(pose.R, dtype=torch.float64).reshape(9).tolist()]
    t = [float(v) for v in torch.as_tensor(pose.t, dtype=torch.float64).reshape(3).tolist()]
    return L.fgs_pose((ctypes.c_double * 9)(*R), (ctypes.c_double * 3)(*t))


class Workspace:
    """Device scratch of one view, owned by PyTorch.  Keep it alive from a
    forward to its backward; it grows when a view needs more intersections.
    `generation` counts the forwards rendered into it: a backward checks that
    no other forward has overwritten the state of its own."""

    def __init__(self, device=None, deterministic: bool = False):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.buf: torch.Tensor | None = None
        self.generation = 0
        # backwards on this workspace reduce the 2D gradients in a fixed order
        # (bit-identical from run to run) instead of with float atomics; they
        # then need about 36 K + 4 N bytes more scratch, kept in det_buf
        self.deterministic = deterministic
        self.det_buf: torch.Tensor | None = None
        self.k = 0  # intersections of the last forward rendered into it

    def ensure_det(self, n: int) -> None:
        nbytes = L.fgs_deterministic_workspace_bytes(n, self.k)
        if self.det_buf is None or self.det_buf.numel() < nbytes:
            self.det_buf = None
            self.det_buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)

    @property
    def nbytes(self) -> int:
        return 0 if self.buf is None else int(self.buf.numel())

    @property
    def ptr(self) -> int:
        return 0 if self.buf is None else int(self.buf.data_ptr())

    def ensure(self, nbytes: int) -> None:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)

    def layout(self, n: int, width: int, height: int) -> L.fgs_layout:
        return L.fgs_workspace_layout(n, width, height, self.nbytes)

    def view(self, offset: int, count: int, dtype: torch.dtype) -> torch.Tensor:
        """A typed view of `count` elements at byte `offset`."""
        size = torch.empty((), dtype=dtype).element_size()
        return self.buf[offset:offset + count * size].view(dtype)


def _stream_handle(device) -> int:
    return int(torch.cuda.current_stream(device).cuda_stream)


def render_forward(means, scales, quats, opacities, sh, sh_degree: int, pose, cam, bg=(0.0, 0.0, 0.0),
                   workspace: Workspace | None = None, save_pixel_state: bool = False, out: torch.Tensor | None = None,
                   k_hint: int | None = None, binning: str = "tight"):
    """Render one view.  Returns (image [3, H, W], workspace, K).  binning
    "rect" lists every tile of each Gaussian's 3-sigma rectangle, "tight"
    only the tiles its alpha >= 1/255 ellipse reaches (same image)."""
    g = gaussians_struct(means, scales, quats, opacities, sh, sh_degree)
    c = camera_struct(cam)
    p = pose_struct(pose)
    dev = means.device
    ws = workspace if workspace is not None else Workspace(dev)
    if out is None:
        out = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device=dev)
    if ws.buf is None:
        kcap = k_hint if k_hint is not None else 8 * g.n + 65536
        ws.ensure(L.fgs_workspace_bytes(g.n, cam.width, cam.height, kcap))
    flags = (FGS_SAVE_PIXEL_STATE if save_pixel_state else 0) | (L.FGS_RECT_BINNING if binning == "rect" else 0)
    for _ in range(3):
        ws.generation += 1
        rc, K = L.fgs_render_forward(g, p, c, bg, flags, ws.ptr, ws.nbytes, out.data_ptr(), _stream_handle(dev))
        if rc == L.FGS_ERR_WORKSPACE and K >= 0:
            ws.ensure(L.fgs_workspace_bytes(g.n, cam.width, cam.height, int(math.ceil(K * 1.15)) + 65536))
            continue
        L.check(rc)
        ws.k = K
        return out, ws, K
    raise L.FgsError(L.FGS_ERR_WORKSPACE, "workspace did not converge")


def render_backward(means, scales, quats, opacities, sh, sh_degree: int, pose, cam, bg, workspace: Workspace,
                    dL_dimg: torch.Tensor, want_means2d: bool = False, accumulate_into: dict | None = None,
                    deterministic: bool | None = None) -> dict:
    """Gradients of one view for the workspace of its forward.  With
    accumulate_into (a dict of gradient tensors from an earlier call), the
    view's gradients are added to those tensors, which are returned.
    deterministic (default: the workspace's setting) reduces the per-tile
    sums in a fixed order, so repeated calls give identical bits."""
    g = gaussians_struct(means, scales, quats, opacities, sh, sh_degree)
    if not dL_dimg.is_contiguous() or dL_dimg.dtype != torch.float32 or tuple(dL_dimg.shape) != (3, cam.height, cam.width):
        raise ValueError("dL_dimg must be contiguous float32 [3, H, W]")
    if accumulate_into is not None:
        out = accumulate_into
        for k, ref in (("means", means), ("scales", scales), ("quats", quats), ("opacities", opacities), ("sh", sh)):
            t = out[k]
            if t.shape != ref.shape or t.dtype != torch.float32 or not t.is_contiguous() or t.device != ref.device:
                raise ValueError(f"accumulated gradient {k} does not match its parameter")
        if want_means2d and "means2d" not in out:
            raise ValueError("accumulate_into has no means2d")
    else:
        out = dict(means=torch.empty_like(means), scales=torch.empty_like(scales), quats=torch.empty_like(quats),
                   opacities=torch.empty_like(opacities), sh=torch.empty_like(sh))
        if want_means2d:
            out["means2d"] = torch.empty((2, g.n), dtype=torch.float32, device=means.device)
    gr = L.fgs_grads(out["means"].data_ptr(), out["scales"].data_ptr(), out["quats"].data_ptr(),
                     out["opacities"].data_ptr(), out["sh"].data_ptr(),
                     out["means2d"].data_ptr() if want_means2d else None, 1 if accumulate_into is not None else 0)
    det = workspace.deterministic if deterministic is None else deterministic
    if det:
        workspace.ensure_det(g.n)
        rc = L.fgs_render_backward_deterministic(g, pose_struct(pose), camera_struct(cam), bg, workspace.ptr,
                                                 workspace.nbytes, dL_dimg.data_ptr(), gr,
                                                 int(workspace.det_buf.data_ptr()), int(workspace.det_buf.numel()),
                                                 _stream_handle(means.device))
    else:
        rc = L.fgs_render_backward(g, pose_struct(pose), camera_struct(cam), bg, workspace.ptr,
                                   workspace.nbytes, dL_dimg.data_ptr(), gr, _stream_handle(means.device))
    L.check(rc)
    return out


class WorkspaceReused(RuntimeError):
    """A backward found its view's forward state overwritten by a later
    forward on the same workspace."""


def _check_generation(ws: Workspace, gen: int) -> None:
    if ws.generation != gen:
        raise WorkspaceReused(
            "the workspace of this view was used by another forward before its backward "
            f"(generation {ws.generation}, expected {gen}); give every view of a step its own Workspace")


class _FisheyeRasterize(torch.autograd.Function):
    """Forward keeps the sorted lists and 2D records in the workspace but no
    per-pixel transmittance; the backward recomputes it with a front-to-back
    re-sweep before the reverse pass."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, sh_degree, pose, cam, bg, workspace):
        img, ws, K = render_forward(means, scales, quats, opacities, sh, sh_degree, pose, cam, bg, workspace)
        ctx.save_for_backward(means, scales, quats, opacities, sh)
        ctx.meta = (sh_degree, pose, cam, bg, ws, ws.generation)
        return img

    @staticmethod
    def backward(ctx, dL):
        means, scales, quats, opacities, sh = ctx.saved_tensors
        sh_degree, pose, cam, bg, ws, gen = ctx.meta
        _check_generation(ws, gen)
        g = render_backward(means, scales, quats, opacities, sh, sh_degree, pose, cam, bg, ws, dL.contiguous())
        return g["means"], g["scales"], g["quats"], g["opacities"], g["sh"], None, None, None, None, None


def rasterize(means, scales, quats, opacities, sh, sh_degree: int, pose, cam, bg=(0.0, 0.0, 0.0),
              workspace: Workspace | None = None) -> torch.Tensor:
    """Differentiable fisheye render of one view, [3, H, W]."""
    return _FisheyeRasterize.apply(means, scales, quats, opacities, sh, sh_degree, pose, cam, tuple(bg),
                                   workspace if workspace is not None else Workspace(means.device))


class _FisheyeRasterizeViews(torch.autograd.Function):
    """B views of one scene: each forward keeps its lists and 2D records in
    its own workspace (no per-pixel transmittance); the backward runs the
    views' backwards into one set of gradient buffers, the first writing and
    the others adding, so B views cost one set of parameter gradients."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, sh_degree, poses, cams, bgs, workspaces):
        imgs = []
        gens = []
        for v, (pose, cam, bg, ws) in enumerate(zip(poses, cams, bgs, workspaces)):
            img, _, _ = render_forward(means, scales, quats, opacities, sh, sh_degree, pose, cam, bg, ws)
            imgs.append(img)
            gens.append(ws.generation)
        ctx.save_for_backward(means, scales, quats, opacities, sh)
        ctx.meta = (sh_degree, poses, cams, bgs, workspaces, gens)
        return tuple(imgs)

    @staticmethod
    def backward(ctx, *dLs):
        means, scales, quats, opacities, sh = ctx.saved_tensors
        sh_degree, poses, cams, bgs, workspaces, gens = ctx.meta
        for ws, gen in zip(workspaces, gens):
            _check_generation(ws, gen)
        g = None
        for pose, cam, bg, ws, dL in zip(poses, cams, bgs, workspaces, dLs):
            if dL is None:
                continue
            g = render_backward(means, scales, quats, opacities, sh, sh_degree, pose, cam, bg, ws, dL.contiguous(),
                                accumulate_into=g)
        if g is None:
            return (None,) * 10
        return g["means"], g["scales"], g["quats"], g["opacities"], g["sh"], None, None, None, None, None


def rasterize_views(means, scales, quats, opacities, sh, sh_degree: int, poses, cams, bgs=None,
                    workspaces: list | None = None) -> tuple:
    """Differentiable fisheye render of several views of one scene (a training
    step's batch of poses); returns one [3, H_v, W_v] image per view.  Each
    view needs its own Workspace (created if not given), since a view's
    backward reads the state its forward left there."""
    B = len(poses)
    if len(cams) != B:
        raise ValueError("one camera per pose")
    bgs = [tuple(b) for b in bgs] if bgs is not None else [(0.0, 0.0, 0.0)] * B
    if workspaces is None:
        workspaces = [Workspace(means.device) for _ in range(B)]
    if len(workspaces) != B or len({id(w) for w in workspaces}) != B:
        raise ValueError("rasterize_views needs one distinct Workspace per view")
    return _FisheyeRasterizeViews.apply(means, scales, quats, opacities, sh, sh_degree, list(poses), list(cams),
                                        bgs, list(workspaces))


def spatial_order(means: torch.Tensor) -> torch.Tensor:
    """Permutation (int64 [N], on the device) that sorts a scene by the Morton
    code of its means (fgs_spatial_order); ties in id order."""
    if means.dim() != 2 or means.shape[0] != 3 or means.dtype != torch.float32 or not means.is_contiguous():
        raise ValueError("means must be contiguous float32 [3, N]")
    n = int(means.shape[1])
    order = torch.empty(n, dtype=torch.int32, device=means.device)
    ws = torch.empty(L.fgs_spatial_order_workspace_bytes(n), dtype=torch.uint8, device=means.device)
    L.fgs_spatial_order(means.data_ptr(), n, order.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(means.device))
    return order.long()


def gather_planes(t: torch.Tensor, order: torch.Tensor) -> torch.Tensor:
    """t[:, order] for a parameter array of planes [P, N] (or [N]) through
    fgs_gather_planes."""
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("gather_planes takes contiguous float32 tensors")
    n = int(t.shape[-1])
    planes = 1 if t.dim() == 1 else int(t.shape[0])
    idx = order.to(torch.int32).contiguous()
    if idx.numel() != n:
        raise ValueError("order and tensor differ in length")
    out = torch.empty_like(t)
    L.fgs_gather_planes(t.data_ptr(), out.data_ptr(), planes, n, idx.data_ptr(), _stream_handle(t.device))
    return out


def spatially_ordered(means, scales, quats, opacities, sh):
    """The scene's parameter arrays permuted into Morton order of the means,
    and the permutation: what a resident scene is stored as, so that a view's
    culled Gaussians come in long runs of memory."""
    order = spatial_order(means)
    return tuple(gather_planes(t, order) for t in (means, scales, quats, opacities, sh)) + (order,)


class _L1Loss(torch.autograd.Function):
    """mean |image - target| in the library's kernels: one deterministic
    two-stage sum forward, one streaming pass for the gradient."""

    @staticmethod
    def forward(ctx, image, target):
        for t in (image, target):
            if not t.is_contiguous() or t.dtype != torch.float32 or not t.is_cuda:
                raise ValueError("l1_loss takes contiguous float32 device tensors")
        if image.shape != target.shape:
            raise ValueError("l1_loss: image and target differ in shape")
        dev = image.device
        partials = torch.empty(L.FGS_L1_PARTIALS, dtype=torch.float64, device=dev)
        loss = torch.empty((), dtype=torch.float32, device=dev)
        L.fgs_l1_loss(image.data_ptr(), target.data_ptr(), image.numel(), partials.data_ptr(), loss.data_ptr(),
                      _stream_handle(dev))
        ctx.save_for_backward(image, target)
        return loss

    @staticmethod
    def backward(ctx, g):
        image, target = ctx.saved_tensors
        g = g.to(torch.float32).contiguous()
        out = torch.empty_like(image)
        L.fgs_l1_loss_backward(image.data_ptr(), target.data_ptr(), image.numel(), g.data_ptr(), out.data_ptr(),
                               _stream_handle(image.device))
        return out, None


def l1_loss(image: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """L1 photometric loss (mean absolute difference), differentiable in image."""
    return _L1Loss.apply(image, target)
