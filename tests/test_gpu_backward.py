"""GPU backward parity against the CPU oracle, through the C ABI.

The upstream gradient is random with zeros on pixels whose alpha cut or
transmittance stop the oracle flags as within margin of the threshold (there
the two precisions may take different discrete decisions).  Bar:
  * per parameter block ||gpu - oracle|| / ||oracle|| <= 1e-4;
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
