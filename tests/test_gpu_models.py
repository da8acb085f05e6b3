"""GPU parity for the other camera models (pinhole, panorama, equisolid,
orthographic, stereographic) against the CPU oracle, through the C ABI.

Same bar as the equidistant tests: preprocess decisions, tile lists and
ranges bit-exact (oracle-flagged ties as sets), images within 1e-4, and the
three gradient checks.  A batch that mixes models must equal its views
rendered one at a time, bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2409_04751_amd import _lib as L  # noqa: E402
from paper_2409_04751_amd import render as R  # noqa: E402
from paper_2409_04751_amd import synth  # noqa: E402

from parity import (check_k, compare_preprocess, compare_tile_lists, gpu_forward, gradient_parity,  # noqa: E402
                    image_tolerance_check, masked_upstream, read_state, to_gpu)

pytestmark = pytest.mark.gpu

MODELS = [synth.MODEL_PINHOLE, synth.MODEL_PANORAMA, synth.MODEL_EQUISOLID, synth.MODEL_ORTHOGRAPHIC,
          synth.MODEL_STEREOGRAPHIC]


def _camera(model, w=200, h=136):
    if model == synth.MODEL_PANORAMA:
        return synth.panorama_camera(2 * w, w)
    fov = {synth.MODEL_PINHOLE: 100.0, synth.MODEL_ORTHOGRAPHIC: 170.0}.get(model, 195.0)
    return synth.fisheye_camera(w, h, fov, model=model)


def _posed(seed):
    rng = np.random.default_rng(seed)
    R_ = synth._haar_rotation(rng)
    pos = rng.uniform(-1, 1, 3)
    return synth.Pose(R_.astype(np.float32), (-(R_ @ pos)).astype(np.float32))


@pytest.mark.parametrize("model", MODELS)
def test_forward_matches_oracle(model):
    scene = synth.room_scene(30_000, 40 + model, 0.01, 3)
    cam = _camera(model)
    pose = _posed(model)
    bg = (0.1, 0.2, 0.3)
    print(f"case model={model} n={scene.n} cam={cam.width}x{cam.height}", flush=True)
    gs = to_gpu(scene)
    img, ws, K = gpu_forward(gs, pose, cam, bg)
    ora = oracle.render(scene, pose, cam, bg)
    assert ora["pre"]["visible"].sum() > 1000
    check_k(K, ora["pre"], ora["bins"])
    st = read_state(ws, scene.n, cam, K)
    compare_preprocess(st, ora["pre"])
    compare_tile_lists(st, ora["bins"], ora["pre"], cam)
    print(image_tolerance_check(img.cpu().numpy(), ora), flush=True)


@pytest.mark.parametrize("model", MODELS)
def test_backward_matches_oracle(model):
    scene = synth.room_scene(15_000, 50 + model, 0.01, 3)
    cam = _camera(model, 160, 112)
    pose = _posed(10 + model)
    bg = (0.2, 0.1, 0.0)
    print(f"case model={model} n={scene.n} cam={cam.width}x{cam.height}", flush=True)
    gs = to_gpu(scene)
    img, ws, K = gpu_forward(gs, pose, cam, bg)
    ora = oracle.render(scene, pose, cam, bg)
    g = masked_upstream(ora, np.random.default_rng(model), cam)
    grads = R.render_backward(gs["means"], gs["scales"], gs["quats"], gs["opacities"], gs["sh"], gs["sh_degree"],
                              pose, cam, bg, ws, torch.from_numpy(g).cuda(), want_means2d=True)
    torch.cuda.synchronize()
    stats, _ = gradient_parity(scene, pose, cam, ws, grads, ora, g, bg)
    print(stats, flush=True)


def test_batch_mixing_models_equals_single_views():
    scene = synth.room_scene(30_000, 60, 0.01, 3)
    gs = to_gpu(scene)
    views = [(_posed(20 + k), _camera(m, 96 + 16 * k, 80), (0.05 * k, 0.1, 0.2))
             for k, m in enumerate([synth.MODEL_EQUIDISTANT] + MODELS)]
    g = R.gaussians_struct(gs["means"], gs["scales"], gs["quats"], gs["opacities"], gs["sh"], gs["sh_degree"])
    cams = [R.camera_struct(c) for _, c, _ in views]
    outs = [torch.empty((3, c.height, c.width), device="cuda") for _, c, _ in views]
    refs = [gpu_forward(gs, p, c, b) for p, c, b in views]
    ws = R.Workspace()
    ws.ensure(L.fgs_batch_workspace_bytes(g.n, cams, sum(k for _, _, k in refs) + 4096))
    rc, kv, kt = L.fgs_render_forward_batch(g, [R.pose_struct(p) for p, _, _ in views], cams,
                                            [b for _, _, b in views], ws.ptr, ws.nbytes, [o.data_ptr() for o in outs],
                                            R._stream_handle(outs[0].device))
    L.check(rc)
    torch.cuda.synchronize()
    for (img, _, K), out, k in zip(refs, outs, kv):
        assert K == k
        assert torch.equal(out, img)


def test_camera_validation():
    scene = synth.room_scene(100, 1, 0.0, 0)
    gs = to_gpu(scene)
    for cam in (synth.Camera(64, 64, 50.0, 50.0, 32.0, 32.0, 7, 0.2, 1.0),      # unknown model
                synth.Camera(64, 64, 50.0, 50.0, 32.0, 32.0, 1, 0.2, 1.6),      # pinhole beyond pi/2
                synth.Camera(64, 64, 50.0, 50.0, 32.0, 32.0, 2, 0.2, 1.6)):     # panorama latitude beyond pi/2
        with pytest.raises(L.FgsError):
            gpu_forward(gs, synth.identity_pose(), cam)
