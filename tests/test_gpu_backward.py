"""GPU backward parity against the CPU oracle, through the C ABI.

The upstream gradient is random with zeros on pixels whose alpha cut or
transmittance stop the oracle flags as within margin of the threshold (there
the two precisions may take different discrete decisions).  Bar:
  * per parameter block ||gpu - oracle|| / ||oracle|| <= 1e-4, and every
    element within 1e-4 max(|ref|, 1e-3 ||ref||_inf);
  * blend backward, every per-Gaussian 2D gradient element within
    1e-4 |ref| + 1e-5 sum_pixels |term| (the rounding scale of its float sum);
  * preprocess backward, every element within 1e-5 |ref| + 1e-6 |ref column|
    of the oracle's chain fed with the GPU's own 2D gradients.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2409_04751_amd import render as R  # noqa: E402
from paper_2409_04751_amd import synth  # noqa: E402

from parity import gpu_forward, gradient_parity, masked_upstream, to_gpu  # noqa: E402

pytestmark = pytest.mark.gpu


def _params(gs):
    return gs["means"], gs["scales"], gs["quats"], gs["opacities"], gs["sh"], gs["sh_degree"]


def _posed(seed):
    rng = np.random.default_rng(seed)
    R_ = synth._haar_rotation(rng)
    pos = rng.uniform(-1, 1, 3)
    return synth.Pose(R_.astype(np.float32), (-(R_ @ pos)).astype(np.float32))


def _check(scene, pose, cam, bg=(0.0, 0.0, 0.0), save=False, seed=0):
    print(f"case n={scene.n} deg={scene.sh_degree} cam={cam.width}x{cam.height} save={save}", flush=True)
    gs = to_gpu(scene)
    img, ws, K = gpu_forward(gs, pose, cam, bg, save_pixel_state=save)
    ora = oracle.render(scene, pose, cam, bg)
    g = masked_upstream(ora, np.random.default_rng(seed), cam)
    grads = R.render_backward(*_params(gs), pose, cam, bg, ws, torch.from_numpy(g).cuda(), want_means2d=True)
    torch.cuda.synchronize()
    stats, go = gradient_parity(scene, pose, cam, ws, grads, ora, g, bg)
    m2 = grads["means2d"].cpu().numpy().T.astype(np.float64)
    ref2 = go["g2d"]["mu_p"]
    assert np.linalg.norm(m2 - ref2) <= 1e-4 * np.linalg.norm(ref2)
    print(stats, flush=True)
    return grads, go


def test_backward_room_sh3_posed():
    scene = synth.room_scene(20_000, 4, 0.01, 3)
    cam = synth.fisheye_camera(160, 128, 200.0)
    _check(scene, _posed(1), cam, bg=(0.1, 0.2, 0.3))


def test_backward_shell_sh0():
    scene_fn, cam, poses = synth.workload("shell1k")
    _check(scene_fn(), poses[0], cam)


def test_backward_unnormalised_quaternions_ragged():
    scene = synth.room_scene(8_000, 6, 0.02, 2)
    rng = np.random.default_rng(3)
    scene.quats *= rng.uniform(0.3, 3.0, scene.n).astype(np.float32)
    cam = synth.fisheye_camera(150, 90, 185.0)
    _check(scene, _posed(2), cam)


def test_backward_long_unsaturated_lists():
    """Faint splats: pixels stay above the transmittance floor for hundreds
    of entries, so the backward's re-sweep and reverse pass both span many
    staged chunks of the tile lists (the opaque scenes finish in the first)."""
    scene = synth.room_scene(30_000, 9, 0.01, 1)
    scene.opacity = np.random.default_rng(5).uniform(0.01, 0.04, scene.n).astype(np.float32)
    cam = synth.fisheye_camera(96, 64, 190.0)
    pose = synth.identity_pose()
    assert oracle.render(scene, pose, cam)["last"].max() > 4 * 128
    _check(scene, pose, cam, bg=(0.2, 0.1, 0.0))


def test_saved_state_matches_recompute():
    """The backward that reads the forward's saved per-pixel T and last
    contributor equals the one that recomputes them."""
    scene = synth.room_scene(20_000, 8, 0.01, 3)
    cam = synth.fisheye_camera(160, 128, 200.0)
    pose = _posed(4)
    gs = to_gpu(scene)
    g = torch.from_numpy(np.random.default_rng(1).normal(size=(3, cam.height, cam.width)).astype(np.float32)).cuda()
    out = []
    for save in (False, True):
        img, ws, K = gpu_forward(gs, pose, cam, save_pixel_state=save)
        out.append(R.render_backward(*_params(gs), pose, cam, (0, 0, 0), ws, g))
    for k in out[0]:
        a, b = out[0][k].cpu().numpy(), out[1][k].cpu().numpy()
        # identical transmittance; only the order of float atomics differs
        assert np.allclose(a, b, rtol=1e-5, atol=1e-6 * np.abs(a).max()), k


def test_autograd_function_recomputes_and_matches_direct_backward():
    scene = synth.room_scene(20_000, 2, 0.01, 3)
    cam = synth.fisheye_camera(128, 128, 200.0)
    pose = _posed(5)
    gs = to_gpu(scene)
    target = torch.from_numpy(synth.target_image(cam.width, cam.height, 1)).cuda()
    leaves = [gs[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacities", "sh")]
    img = R.rasterize(*leaves, gs["sh_degree"], pose, cam)
    loss = (img - target).abs().mean()
    loss.backward()
    # direct C-ABI backward with the same upstream gradient
    img2, ws, K = gpu_forward(gs, pose, cam)
    assert torch.equal(img.detach(), img2)
    dL = (torch.sign(img2 - target) / img2.numel()).contiguous()
    ref = R.render_backward(*_params(gs), pose, cam, (0, 0, 0), ws, dL)
    for leaf, k in zip(leaves, ("means", "scales", "quats", "opacities", "sh")):
        a, b = leaf.grad.cpu().numpy(), ref[k].cpu().numpy()
        assert np.allclose(a, b, rtol=1e-5, atol=1e-6 * max(np.abs(b).max(), 1e-30)), k


def test_accumulate_mode_adds_a_second_view():
    """fgs_grads.accumulate = 1 adds a view's gradient to the buffers: view A
    written then view B accumulated equals A + B computed from two written
    backwards, to fp32 accuracy (the blend's float atomics vary the last bits
    of each run), and Gaussians culled in view B keep A's values."""
    scene = synth.room_scene(20_000, 12, 0.01, 3)
    cam = synth.fisheye_camera(160, 128, 200.0)
    poses = [_posed(6), _posed(7)]
    gs = to_gpu(scene)
    rng = np.random.default_rng(4)
    sep, wss = [], []
    ups = [torch.from_numpy(rng.normal(size=(3, cam.height, cam.width)).astype(np.float32)).cuda() for _ in poses]
    for pose, g in zip(poses, ups):
        _, ws, _ = gpu_forward(gs, pose, cam)
        wss.append(ws)
        sep.append(R.render_backward(*_params(gs), pose, cam, (0, 0, 0), ws, g, want_means2d=True))
    acc = R.render_backward(*_params(gs), poses[0], cam, (0, 0, 0), wss[0], ups[0], want_means2d=True)
    acc = R.render_backward(*_params(gs), poses[1], cam, (0, 0, 0), wss[1], ups[1], want_means2d=True,
                            accumulate_into=acc)
    torch.cuda.synchronize()
    for k in ("scales", "quats", "opacities", "sh", "means2d"):
        # the blend's float atomics make each view's own 2D gradients vary in
        # their last bits from run to run, so compare to fp32 accuracy
        torch.testing.assert_close(acc[k], sep[0][k] + sep[1][k], rtol=1e-5, atol=1e-6 * float(acc[k].abs().max()))
    torch.testing.assert_close(acc["means"], sep[0]["means"] + sep[1]["means"], rtol=1e-5,
                               atol=1e-6 * float(acc["means"].abs().max()))


def test_rasterize_views_autograd_matches_oracle():
    """Three views of different size and field of view through the multi-view
    autograd function; a linear loss whose per-view weights are zero on the
    pixels the oracle flags.  The summed parameter gradients against the
    oracle's, every element."""
    from parity import _stack2d_abs, check_blocks_elementwise, check_blocks_rel_l2

    scene = synth.room_scene(20_000, 13, 0.01, 3)
    cams = [synth.fisheye_camera(160, 128, 200.0), synth.fisheye_camera(96, 96, 150.0),
            synth.fisheye_camera(130, 70, 185.0)]
    poses = [_posed(8), _posed(9), _posed(10)]
    gs = to_gpu(scene)
    leaves = [gs[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacities", "sh")]
    imgs = R.rasterize_views(*leaves, scene.sh_degree, poses, cams)
    rng = np.random.default_rng(7)
    total, scale = None, None
    loss = 0.0
    for img, pose, cam in zip(imgs, poses, cams):
        ora = oracle.render(scene, pose, cam)
        w = masked_upstream(ora, rng, cam)
        loss = loss + (img * torch.from_numpy(w).cuda()).sum()
        go = oracle.render_backward(scene, pose, cam, ora, w, abs_sums=True)
        sc = oracle.chain_error_scale(scene, pose, cam, ora["pre"], _stack2d_abs(go.pop("g2d")))
        total = go if total is None else {k: total[k] + go[k] for k in total}
        scale = sc if scale is None else {k: scale[k] + sc[k] for k in scale}
    loss.backward()
    torch.cuda.synchronize()
    grads = dict(means=leaves[0].grad, scales=leaves[1].grad, quats=leaves[2].grad, opacities=leaves[3].grad,
                 sh=leaves[4].grad)
    print(check_blocks_rel_l2(grads, total), check_blocks_elementwise(grads, total, err_scale=scale), flush=True)
