"""GPU forward parity against the CPU oracle, through the C ABI.

Bar: visibility, radius, rectangle, tiles touched, depth key bits, the sorted
(tile, id) lists and tile ranges bit-exact (ties the oracle marks within 1e-9
of a rounding boundary are compared as sets instead); 2D records to fp32
accuracy; image max error <= 1e-4 * max(1, |ref|_inf) on every pixel whose
alpha cut / transmittance stop the oracle does not find within its margin.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2409_04751_amd import _lib as L  # noqa: E402
from paper_2409_04751_amd import synth  # noqa: E402

from parity import (check_k, compare_preprocess, compare_tile_lists, gpu_forward, image_tolerance_check,  # noqa: E402
                    read_state, to_gpu)

pytestmark = pytest.mark.gpu


def _full_check(scene, pose, cam, bg=(0.0, 0.0, 0.0), save=False, binning="tight"):
    print(f"case n={scene.n} cam={cam.width}x{cam.height} bg={bg} binning={binning}", flush=True)
    gs = to_gpu(scene)
    img, ws, K = gpu_forward(gs, pose, cam, bg, save_pixel_state=save, binning=binning)
    ora = oracle.render(scene, pose, cam, bg, binning=binning)
    check_k(K, ora["pre"], ora["bins"])
    st = read_state(ws, scene.n, cam, K)
    compare_preprocess(st, ora["pre"])
    compare_tile_lists(st, ora["bins"], ora["pre"], cam)
    stats = image_tolerance_check(img.cpu().numpy(), ora)
    print(stats, flush=True)
    return img, ws, K, st, ora


def test_shell_1k_256_180deg():
    scene_fn, cam, poses = synth.workload("shell1k")
    _full_check(scene_fn(), poses[0], cam)


def test_shell_1k_nonzero_background_and_saved_state():
    scene_fn, cam, poses = synth.workload("shell1k")
    img, ws, K, st, ora = _full_check(scene_fn(), poses[0], cam, bg=(0.3, 0.6, 0.9), save=True)
    ok = ora["flags"] == 0
    np.testing.assert_array_equal(st["pixel_last"][ok], ora["last"][ok])
    np.testing.assert_allclose(st["pixel_T"][ok], ora["T_final"][ok], rtol=1e-4, atol=1e-7)


def test_ragged_image_posed_camera():
    """Image size not a multiple of 16 (ragged last tile row and column), a
    rotated and translated camera, larger splats spanning several tiles."""
    rng = np.random.default_rng(7)
    scene = synth.shell_scene(4000, 3)
    scene.scales[:] = np.exp(rng.normal(-2.6, 0.6, size=scene.scales.shape)).astype(np.float32)
    cam = synth.fisheye_camera(200, 117, 195.0)
    R = synth._haar_rotation(rng)
    pose = synth.Pose(R.astype(np.float32), (-(R @ np.array([0.2, -0.1, 0.3]))).astype(np.float32))
    _full_check(scene, pose, cam, bg=(0.2, 0.1, 0.0))


def test_room_sh3_many_tiles():
    scene = synth.room_scene(60_000, 5, 0.01, 3)
    cam = synth.fisheye_camera(320, 240, 200.0)
    _full_check(scene, synth.identity_pose(), cam)


def test_empty_scene_is_background():
    scene = synth.shell_scene(0, 0)
    cam = synth.fisheye_camera(64, 40, 180.0)
    gs = to_gpu(scene)
    img, ws, K = gpu_forward(gs, synth.identity_pose(), cam, (0.25, 0.5, 0.75))
    assert K == 0
    np.testing.assert_array_equal(img.cpu().numpy(), np.broadcast_to(np.array([0.25, 0.5, 0.75], np.float32)[:, None, None], img.shape))


def test_all_culled_is_background():
    scene = synth.shell_scene(500, 1)
    scene.means[2] = -np.abs(scene.means[2]) - 0.5   # all behind the camera
    scene.means[0] *= 0.01
    scene.means[1] *= 0.01                           # close to the rear axis: theta > theta_max
    cam = synth.fisheye_camera(64, 64, 180.0)
    gs = to_gpu(scene)
    img, ws, K = gpu_forward(gs, synth.identity_pose(), cam, (0.5, 0.5, 0.5))
    ora = oracle.render(scene, synth.identity_pose(), cam, (0.5, 0.5, 0.5))
    assert ora["pre"]["visible"].sum() == 0 and K == 0
    assert np.all(img.cpu().numpy() == 0.5)


def test_non_finite_parameters_are_culled():
    scene = synth.shell_scene(300, 2)
    scene.means[0, 3] = np.nan
    scene.scales[1, 5] = np.inf
    scene.quats[:, 7] = 0.0
    scene.opacity[9] = np.nan
    cam = synth.fisheye_camera(128, 128, 180.0)
    img, ws, K, st, ora = _full_check(scene, synth.identity_pose(), cam)
    for i in (3, 5, 7, 9):
        assert st["tiles"][i] == 0 and st["depth_bits"][i] == 0xFFFFFFFF


def test_single_huge_gaussian_covers_image():
    scene = synth.shell_scene(1, 0)
    scene.means[:, 0] = [0.0, 0.0, 1.0]
    scene.scales[:, 0] = [2.0, 2.0, 2.0]
    cam = synth.fisheye_camera(100, 60, 180.0)
    img, ws, K, st, ora = _full_check(scene, synth.identity_pose(), cam, bg=(0.0, 0.0, 1.0))
    assert K == cam.tiles_x * cam.tiles_y


def test_workspace_too_small_then_grown():
    scene_fn, cam, poses = synth.workload("shell1k")
    scene = scene_fn()
    gs = to_gpu(scene)
    from paper_2409_04751_amd import render as R
    ws = R.Workspace()
    ws.ensure(L.fgs_workspace_bytes(scene.n, cam.width, cam.height, 10))
    g = R.gaussians_struct(gs["means"], gs["scales"], gs["quats"], gs["opacities"], gs["sh"], 0)
    out = torch.empty((3, cam.height, cam.width), device="cuda")
    rc, K = L.fgs_render_forward(g, R.pose_struct(poses[0]), R.camera_struct(cam), (0, 0, 0), 0, ws.ptr, ws.nbytes,
                                 out.data_ptr(), R._stream_handle(out.device))
    ora = oracle.render(scene, poses[0], cam)
    assert rc == L.FGS_ERR_WORKSPACE
    check_k(K, ora["pre"], ora["bins"])
    ws.ensure(L.fgs_workspace_bytes(scene.n, cam.width, cam.height, K))
    rc, K2 = L.fgs_render_forward(g, R.pose_struct(poses[0]), R.camera_struct(cam), (0, 0, 0), 0, ws.ptr, ws.nbytes,
                                  out.data_ptr(), R._stream_handle(out.device))
    assert rc == L.FGS_OK and K2 == K


def test_forward_is_bit_deterministic():
    scene = synth.room_scene(40_000, 9, 0.01, 3)
    cam = synth.fisheye_camera(256, 192, 190.0)
    gs = to_gpu(scene)
    a, wa, Ka = gpu_forward(gs, synth.identity_pose(), cam)
    a = a.clone()
    sa = read_state(wa, scene.n, cam, Ka)
    b, wb, Kb = gpu_forward(gs, synth.identity_pose(), cam)
    sb = read_state(wb, scene.n, cam, Kb)
    assert Ka == Kb
    assert torch.equal(a, b)
    np.testing.assert_array_equal(sa["tile_ids"], sb["tile_ids"])
    np.testing.assert_array_equal(sa["ranges"], sb["ranges"])


def test_rect_binning_matches_oracle_and_tight_image():
    """Vanilla 3-sigma-rect lists (FGS_RECT_BINNING) against the oracle's rect
    binning, and the tight lists' image equal to it bit for bit: binning only
    drops pairs that are never blended."""
    scene = synth.room_scene(60_000, 3, 0.02, 3)
    _, cam, poses = synth.workload("room3m_2k")
    cam = synth.fisheye_camera(320, 256, 200.0)
    img_r, ws_r, K_r, st_r, ora_r = _full_check(scene, poses[1], cam, binning="rect")
    gs = to_gpu(scene)
    img_t, ws_t, K_t = gpu_forward(gs, poses[1], cam, binning="tight")
    assert K_t < K_r
    assert torch.equal(img_t, img_r)
