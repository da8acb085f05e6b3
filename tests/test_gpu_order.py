"""Spatial order of a resident scene (fgs_spatial_order, fgs_gather_planes).

  * The permutation equals a numpy stable sort by the 30-bit Morton code of
    each mean on a 1024^3 grid over the finite means' bounding box, computed
    here in float32 by the same definition (u = (x - lo) / (hi - lo), cell =
    min(max(1024 u, 0), 1023) truncated; x in bit 2, y bit 1, z bit 0 of each
    triple; non-finite means last), index for index.
  * The gather applies it to every parameter plane exactly.
  * A reordered scene renders the same image as the original and its
    gradients are the original's, permuted (up to float atomics).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2409_04751_amd import render as R  # noqa: E402
from paper_2409_04751_amd import synth  # noqa: E402

from parity import gpu_forward, to_gpu  # noqa: E402

pytestmark = pytest.mark.gpu


def _spread(v):
    out = np.zeros_like(v, dtype=np.uint64)
    for b in range(10):
        out |= ((v.astype(np.uint64) >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def morton_order_reference(means: np.ndarray) -> np.ndarray:
    m = means.astype(np.float32)
    fin = np.all(np.isfinite(m), axis=0)
    lo = m[:, fin].min(axis=1)
    hi = m[:, fin].max(axis=1)
    code = np.zeros(m.shape[1], np.uint64)
    with np.errstate(invalid="ignore"):
        for a in range(3):
            ext = np.float32(hi[a] - lo[a])
            u = (m[a] - lo[a]) / ext if ext > 0 else np.zeros_like(m[a])
            q = np.minimum(np.maximum(u * np.float32(1024.0), np.float32(0.0)), np.float32(1023.0))
            q = np.where(fin, q, 0).astype(np.uint32)
            code |= _spread(q) << np.uint64(2 - a)
    code[~fin] = (1 << 30) - 1
    return np.lexsort((np.arange(m.shape[1]), code))


@pytest.mark.parametrize("n", [1, 1000, 70_001, 3_000_000])
def test_order_equals_reference(n):
    scene = synth.room_scene(n, 31, 0.01, 0)
    if n >= 1000:
        scene.means[:, 5] = np.nan  # one non-finite mean sorts last
    m = torch.from_numpy(np.ascontiguousarray(scene.means)).cuda()
    order = R.spatial_order(m).cpu().numpy()
    ref = morton_order_reference(scene.means)
    np.testing.assert_array_equal(order, ref)
    if n >= 1000:
        assert order[-1] == 5
    g = R.gather_planes(m, torch.from_numpy(order).cuda())
    torch.testing.assert_close(g, m[:, torch.from_numpy(order).cuda()], rtol=0, atol=0, equal_nan=True)


def test_reordered_scene_renders_the_same():
    scene = synth.room_scene(200_000, 32, 0.01, 3)
    cam = synth.fisheye_camera(320, 240, 190.0)
    pose = synth.identity_pose()
    gs = to_gpu(scene)
    p = (gs["means"], gs["scales"], gs["quats"], gs["opacities"], gs["sh"])
    *q, order = R.spatially_ordered(*p)
    img_a, ws_a, K_a = gpu_forward(gs, pose, cam)
    gq = dict(means=q[0], scales=q[1], quats=q[2], opacities=q[3], sh=q[4], sh_degree=3)
    img_b, ws_b, K_b = gpu_forward(gq, pose, cam)
    assert K_a == K_b
    # the same splats blended in the same depth order: equal up to depth ties
    # between Gaussians (broken by the new ids)
    torch.testing.assert_close(img_a, img_b, rtol=0, atol=1e-6)
    up = torch.from_numpy(np.random.default_rng(3).normal(size=(3, cam.height, cam.width)).astype(np.float32)).cuda()
    ga = R.render_backward(*p, 3, pose, cam, (0, 0, 0), ws_a, up)
    gb = R.render_backward(*q, 3, pose, cam, (0, 0, 0), ws_b, up)
    for k in ga:
        a = ga[k][..., order]
        torch.testing.assert_close(a, gb[k], rtol=1e-4, atol=1e-6 * float(a.abs().max()))
