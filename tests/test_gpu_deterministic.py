"""Deterministic backward (fgs_render_backward_deterministic) through the C ABI.

  * Two calls on the same forward state give bit-identical gradients (all
    five parameter blocks and dL/dmu_p), at small sizes and at the 3M-Gaussian
    1752x1168 benchmark view.
  * Against the oracle it meets the same bars as the atomic backward
    (per-block rel-L2, per-element, per-Gaussian 2D sums, preprocess chain).
  * Against the atomic backward only the order of the float additions
    differs: per block rel-L2 <= 1e-5.
  * A view with no intersections gives zero gradients; a scratch buffer one
    byte too small is refused with FGS_ERR_WORKSPACE.
  * A deterministic Workspace makes the autograd path deterministic.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2409_04751_amd import _lib as L  # noqa: E402
from paper_2409_04751_amd import render as R  # noqa: E402
from paper_2409_04751_amd import synth  # noqa: E402

from parity import gpu_forward, gradient_parity, masked_upstream, to_gpu  # noqa: E402

pytestmark = pytest.mark.gpu

_KEYS = ("means", "scales", "quats", "opacities", "sh", "means2d")


def _params(gs):
    return gs["means"], gs["scales"], gs["quats"], gs["opacities"], gs["sh"], gs["sh_degree"]


def _backward(gs, pose, cam, bg, ws, up, det):
    g = R.render_backward(*_params(gs), pose, cam, bg, ws, up, want_means2d=True, deterministic=det)
    torch.cuda.synchronize()
    return g


def _identical(a, b):
    for k in _KEYS:
        assert torch.equal(a[k], b[k]), f"{k} differs between two deterministic backwards"


def _close_to_atomic(det, atom, tol=1e-5):
    for k in _KEYS:
        d, a = det[k].double(), atom[k].double()
        na = float(torch.linalg.vector_norm(a))
        err = float(torch.linalg.vector_norm(d - a))
        print(f"  {k}: rel-L2 deterministic vs atomic {err / max(na, 1e-30):.2e}", flush=True)
        assert err <= tol * max(na, 1e-30), k


def test_deterministic_matches_oracle_and_repeats():
    scene = synth.room_scene(20_003, 4, 0.01, 3)  # ragged n
    cam = synth.fisheye_camera(160, 128, 200.0)
    pose = synth.identity_pose()
    bg = (0.1, 0.2, 0.3)
    print(f"case n={scene.n} cam={cam.width}x{cam.height}", flush=True)
    gs = to_gpu(scene)
    _, ws, K = gpu_forward(gs, pose, cam, bg)
    ora = oracle.render(scene, pose, cam, bg)
    up_np = masked_upstream(ora, np.random.default_rng(0), cam)
    up = torch.from_numpy(up_np).cuda()
    d1 = _backward(gs, pose, cam, bg, ws, up, True)
    stats, _ = gradient_parity(scene, pose, cam, ws, d1, ora, up_np, bg)
    print(stats, flush=True)
    d2 = _backward(gs, pose, cam, bg, ws, up, True)
    _identical(d1, d2)
    a = _backward(gs, pose, cam, bg, ws, up, False)
    _close_to_atomic(d1, a)


def test_deterministic_long_lists():
    """Faint splats: long lists, many tiles per Gaussian, several staged
    chunks per tile."""
    scene = synth.room_scene(30_000, 9, 0.01, 1)
    scene.opacity = np.random.default_rng(5).uniform(0.01, 0.04, scene.n).astype(np.float32)
    cam = synth.fisheye_camera(96, 64, 190.0)
    pose = synth.identity_pose()
    print(f"case n={scene.n} faint cam={cam.width}x{cam.height}", flush=True)
    gs = to_gpu(scene)
    _, ws, K = gpu_forward(gs, pose, cam)
    ora = oracle.render(scene, pose, cam)
    up_np = masked_upstream(ora, np.random.default_rng(1), cam)
    up = torch.from_numpy(up_np).cuda()
    d1 = _backward(gs, pose, cam, (0.0, 0.0, 0.0), ws, up, True)
    stats, _ = gradient_parity(scene, pose, cam, ws, d1, ora, up_np)
    print(stats, flush=True)
    _identical(d1, _backward(gs, pose, cam, (0.0, 0.0, 0.0), ws, up, True))


def test_deterministic_empty_view_and_small_scratch():
    scene = synth.room_scene(5_000, 2, 0.01, 0)
    scene.opacity[:] = np.float32(1e-3)  # below 1/255: no Gaussian reaches a tile
    cam = synth.fisheye_camera(64, 48, 180.0)
    pose = synth.identity_pose()
    print(f"case n={scene.n} empty view", flush=True)
    gs = to_gpu(scene)
    _, ws, K = gpu_forward(gs, pose, cam)
    assert K == 0
    up = torch.ones((3, cam.height, cam.width), dtype=torch.float32, device="cuda")
    d = _backward(gs, pose, cam, (0.0, 0.0, 0.0), ws, up, True)
    for k in _KEYS:
        assert not bool(d[k].any()), k

    scene = synth.room_scene(5_000, 2, 0.01, 0)
    gs = to_gpu(scene)
    _, ws, K = gpu_forward(gs, pose, cam)
    assert K > 0
    need = L.fgs_deterministic_workspace_bytes(scene.n, K)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = {k: torch.empty_like(gs[k]) for k in ("means", "scales", "quats", "opacities", "sh")}
    gr = L.fgs_grads(out["means"].data_ptr(), out["scales"].data_ptr(), out["quats"].data_ptr(),
                     out["opacities"].data_ptr(), out["sh"].data_ptr(), None, 0)
    g = R.gaussians_struct(*_params(gs))
    rc = L.fgs_render_backward_deterministic(g, R.pose_struct(pose), R.camera_struct(cam), (0.0, 0.0, 0.0), ws.ptr,
                                             ws.nbytes, up.data_ptr(), gr, buf.data_ptr(), need - 1,
                                             R._stream_handle(buf.device))
    assert rc == L.FGS_ERR_WORKSPACE
    rc = L.fgs_render_backward_deterministic(g, R.pose_struct(pose), R.camera_struct(cam), (0.0, 0.0, 0.0), ws.ptr,
                                             ws.nbytes, up.data_ptr(), gr, buf.data_ptr(), need,
                                             R._stream_handle(buf.device))
    assert rc == L.FGS_OK
    torch.cuda.synchronize()


def test_deterministic_autograd_workspace():
    scene = synth.room_scene(40_000, 11, 0.01, 3)
    cam = synth.fisheye_camera(200, 150, 190.0)
    pose = synth.identity_pose()
    gs = to_gpu(scene)
    target = torch.rand((3, cam.height, cam.width), device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    ws = R.Workspace(torch.device("cuda"), deterministic=True)

    def grads():
        leaves = [t.detach().clone().requires_grad_(True) for t in _params(gs)[:5]]
        img = R.rasterize(*leaves, 3, pose, cam, (0.0, 0.0, 0.0), ws)
        loss = R.l1_loss(img, target)
        return torch.autograd.grad(loss, leaves)

    a, b = grads(), grads()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert ws.det_buf is not None


def test_deterministic_benchmark_view():
    """The 3M-Gaussian room at 1752x1168, 180 deg, in Morton order, as the
    benchmark renders it: two deterministic backwards are bit-identical and
    within float reassociation of the atomic one."""
    scene = synth.room_scene(3_000_000, 0, 0.01, 3)
    cam = synth.fisheye_camera(1752, 1168, 180.0)
    pose = synth.identity_pose()
    print(f"case n={scene.n} cam={cam.width}x{cam.height} benchmark view", flush=True)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    *p, _ = R.spatially_ordered(f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacity), f(scene.sh))
    gs = dict(means=p[0], scales=p[1], quats=p[2], opacities=p[3], sh=p[4], sh_degree=3)
    del scene
    _, ws, K = gpu_forward(gs, pose, cam)
    print(f"  K={K}", flush=True)
    up = (torch.rand((3, cam.height, cam.width), device="cuda", generator=torch.Generator("cuda").manual_seed(1))
          - 0.5).contiguous()
    d1 = _backward(gs, pose, cam, (0.0, 0.0, 0.0), ws, up, True)
    d2 = _backward(gs, pose, cam, (0.0, 0.0, 0.0), ws, up, True)
    _identical(d1, d2)
    del d2
    a = _backward(gs, pose, cam, (0.0, 0.0, 0.0), ws, up, False)
    _close_to_atomic(d1, a)
