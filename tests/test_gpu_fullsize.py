"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (same library entry points, same workspace protocol).

  * 500k Gaussians, SH3, 1752x1168 fisheye at 180 deg: full forward + backward
    against the full oracle, per-pixel state included.
  * 3M Gaussians (1% large), SH3, 1752x1168 at 180 deg (the benchmark view,
    with the scene in the spatial order the benchmark stores it in): the tile
    lists of all ~23.2M intersections and the ranges of all 8030 tiles
    bit-exact (ties printed), image, per-pixel state, and the backward with
    transmittance recomputation against the full oracle.  The same view with
    the vanilla 3-sigma-rect lists (~49M pairs) bit-exact too.
  * 3M Gaussians, 2048x2048 at 200 deg, the four seeded poses of one training
    step through the multi-view autograd function: each view's lists and
    image, and the step's summed gradients, against the oracle; then a crop
    of 2,000 Gaussians visible in pose 0, rendered as their own scene through
    the same autograd path, with every gradient element checked.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2409_04751_amd import render as R  # noqa: E402
from paper_2409_04751_amd import synth  # noqa: E402

from parity import (check_blocks_elementwise, check_blocks_rel_l2, check_k, compare_pixel_state,  # noqa: E402
                    compare_preprocess, compare_tile_lists, gpu_forward, gradient_parity, image_tolerance_check,
                    masked_upstream, read_grad2d, read_state, check_2d, to_gpu, _stack2d_abs)

pytestmark = pytest.mark.gpu


def _params(gs):
    return gs["means"], gs["scales"], gs["quats"], gs["opacities"], gs["sh"], gs["sh_degree"]


def _forward_parity(scene, pose, cam, ws, K, ora, binning="tight"):
    print(f"K gpu {K} oracle {ora['bins']['K']}", flush=True)
    st = read_state(ws, scene.n, cam, K)
    check_k(K, ora["pre"], ora["bins"])
    compare_preprocess(st, ora["pre"])
    compare_tile_lists(st, ora["bins"], ora["pre"], cam)
    return st


def _fwd_bwd(scene, pose, cam, seed=0):
    print(f"case n={scene.n} cam={cam.width}x{cam.height}", flush=True)
    gs = to_gpu(scene)
    img, ws, K = gpu_forward(gs, pose, cam)
    ora = oracle.render(scene, pose, cam)
    _forward_parity(scene, pose, cam, ws, K, ora)
    print("image", image_tolerance_check(img.cpu().numpy(), ora), flush=True)
    # per-pixel state from a second forward that saves it
    _, ws_s, _ = gpu_forward(gs, pose, cam, save_pixel_state=True)
    st_s = read_state(ws_s, scene.n, cam, K)
    print("flagged pixels whose contributor count differs:", compare_pixel_state(st_s, ora), flush=True)
    del ws_s, st_s
    g = masked_upstream(ora, np.random.default_rng(seed), cam, scale=1.0 / (3 * cam.width * cam.height))
    grads = R.render_backward(*_params(gs), pose, cam, (0, 0, 0), ws, torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    stats, _ = gradient_parity(scene, pose, cam, ws, grads, ora, g)
    print(stats, flush=True)


def test_room500k_full_view():
    scene_fn, cam, poses = synth.workload("room500k")
    _fwd_bwd(scene_fn(), poses[0], cam)


@pytest.fixture(scope="module")
def scene3m():
    return synth.room_scene(3_000_000, 0, 0.01, 3)


def test_room3m_benchmark_view(scene3m):
    """The benchmark's resident scene: the 3M scene stored in the library's
    spatial (Morton) order, as bench.py times it."""
    cam = synth.fisheye_camera(1752, 1168, 180.0)
    order = R.spatial_order(torch.from_numpy(np.ascontiguousarray(scene3m.means)).cuda()).cpu().numpy()
    _fwd_bwd(scene3m.subset(order), synth.identity_pose(), cam, seed=1)


def test_room3m_benchmark_view_rect_lists(scene3m):
    """The vanilla lists (every tile of each 3-sigma rect) at the benchmark
    view: ~49M pairs bit-exact, ranges included, same image."""
    cam = synth.fisheye_camera(1752, 1168, 180.0)
    pose = synth.identity_pose()
    gs = to_gpu(scene3m)
    img, ws, K = gpu_forward(gs, pose, cam, binning="rect", k_hint=52_000_000)
    pre = oracle.preprocess(scene3m, pose, cam, "rect")
    bins = oracle.bin_and_sort(pre, cam)
    print(f"rect lists: K gpu {K} oracle {bins['K']}", flush=True)
    st = read_state(ws, scene3m.n, cam, K)
    check_k(K, pre, bins)
    compare_preprocess(st, pre)
    compare_tile_lists(st, bins, pre, cam)
    del st, bins
    img_t, _, _ = gpu_forward(gs, pose, cam)
    torch.testing.assert_close(img, img_t, rtol=0, atol=0)


def _linear_upstreams(oras, cams, seed):
    """Per view a seeded N(0, 1) / (3 H W) weight image, zero on the pixels the
    oracle flags: the loss sum_v <W_v, image_v> has dL/dimage_v = W_v."""
    rng = np.random.default_rng(seed)
    return [masked_upstream(o, rng, c, scale=1.0 / (3 * c.width * c.height)) for o, c in zip(oras, cams)]


def _views_autograd(scene, poses, cam, seed):
    """Four views through rasterize_views, then the linear loss's backward
    through autograd.  Returns (images, workspaces, grads, oracle forwards,
    upstreams)."""
    gs = to_gpu(scene)
    params = [gs[k].requires_grad_(True) for k in ("means", "scales", "quats", "opacities", "sh")]
    cams = [cam] * len(poses)
    wss = [R.Workspace(params[0].device) for _ in poses]
    imgs = R.rasterize_views(*params, scene.sh_degree, poses, cams, None, wss)
    torch.cuda.synchronize()
    oras = []
    for v, pose in enumerate(poses):
        print(f"view {v}: oracle forward", flush=True)
        ora = oracle.render(scene, pose, cam)
        K = int(ora["bins"]["K"])
        lay = wss[v].layout(scene.n, cam.width, cam.height)
        Kg = int(wss[v].view(lay.counters, 16, torch.int32)[0].item())
        _forward_parity(scene, pose, cam, wss[v], Kg, ora)
        print(f"view {v} image", image_tolerance_check(imgs[v].detach().cpu().numpy(), ora), flush=True)
        oras.append(ora)
        del ora
    ups = _linear_upstreams(oras, cams, seed)
    loss = sum((img * torch.from_numpy(u).cuda()).sum() for img, u in zip(imgs, ups))
    loss.backward()
    torch.cuda.synchronize()
    grads = dict(means=params[0].grad, scales=params[1].grad, quats=params[2].grad, opacities=params[3].grad,
                 sh=params[4].grad)
    return imgs, wss, grads, oras, ups


def _oracle_sum(scene, poses, cam, oras, ups, with_scale=False):
    """The oracle's gradients summed over the views, the views' 2D gradients,
    and (with_scale) the summed rounding-error scale of each element."""
    total, scale = None, None
    g2d = []
    for pose, ora, u in zip(poses, oras, ups):
        go = oracle.render_backward(scene, pose, cam, ora, u, abs_sums=True)
        g2d.append(go.pop("g2d"))
        total = go if total is None else {k: total[k] + go[k] for k in total}
        if with_scale:
            sc = oracle.chain_error_scale(scene, pose, cam, ora["pre"], _stack2d_abs(g2d[-1]))
            scale = sc if scale is None else {k: scale[k] + sc[k] for k in scale}
    return total, g2d, scale


def test_room3m_2048_200deg_four_views_autograd(scene3m):
    _, cam, poses = synth.workload("room3m_2k")
    assert len(poses) == 4
    print(f"case n={scene3m.n} cam={cam.width}x{cam.height} fov 200 views 4", flush=True)
    imgs, wss, grads, oras, ups = _views_autograd(scene3m, poses, cam, seed=5)
    total, _, _ = _oracle_sum(scene3m, poses, cam, oras, ups)
    print("summed over 4 views, rel_l2", check_blocks_rel_l2(grads, total), flush=True)


def test_room3m_2048_200deg_2k_crop_four_views_autograd(scene3m):
    _, cam, poses = synth.workload("room3m_2k")
    pre = oracle.preprocess(scene3m, poses[0], cam)
    rng = np.random.default_rng(2)
    vis = np.nonzero(pre["visible"])[0]
    crop = np.sort(rng.choice(vis, 2000, replace=False))
    sub = scene3m.subset(crop)
    print(f"case crop n={sub.n} cam={cam.width}x{cam.height} fov 200 views 4", flush=True)
    imgs, wss, grads, oras, ups = _views_autograd(sub, poses, cam, seed=6)
    total, g2d, scale = _oracle_sum(sub, poses, cam, oras, ups, with_scale=True)
    print("rel_l2", check_blocks_rel_l2(grads, total), flush=True)
    print("elementwise", check_blocks_elementwise(grads, total, err_scale=scale), flush=True)
    # each view's 2D gradients are still in its own workspace
    for v in range(len(poses)):
        print(f"view {v} blend 2D", check_2d(read_grad2d(wss[v], sub.n, cam), g2d[v]), flush=True)


def test_workspace_reuse_before_backward_raises():
    """Two forwards on one workspace before the first one's backward: the
    backward refuses instead of using the second view's lists."""
    scene_fn, cam, poses = synth.workload("shell1k")
    scene = scene_fn()
    gs = to_gpu(scene)
    params = [gs[k].requires_grad_(True) for k in ("means", "scales", "quats", "opacities", "sh")]
    ws = R.Workspace(params[0].device)
    a = R.rasterize(*params, scene.sh_degree, poses[0], cam, workspace=ws)
    pose2 = synth.random_poses(1, 9, (-0.5, -0.5, -0.5), (0.5, 0.5, 0.5))[0]
    b = R.rasterize(*params, scene.sh_degree, pose2, cam, workspace=ws)
    with pytest.raises(R.WorkspaceReused):
        a.sum().backward(retain_graph=True)
    b.sum().backward()  # the latest forward's backward still works
    with pytest.raises(ValueError):
        R.rasterize_views(*params, scene.sh_degree, [poses[0], pose2], [cam, cam], None, [ws, ws])
