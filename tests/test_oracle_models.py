"""Pins for the oracle's other camera models.

Sec. 3.2 lists the equisolid-angle, orthographic and stereographic fisheye
projections besides the equidistant one; Sec. 5.3 extends the method to a
panorama and prints its projection and J.  The oracle takes J and dJ/dmu_c
of these models as the first and second derivatives of the projection (by
forward-mode differentiation), so they are pinned here against:
  * central finite differences of the projection and of J;
  * the textbook pinhole Jacobian [[f/z, 0, -f x/z^2], [0, f/z, -f y/z^2]];
  * the panorama J the paper prints (Sec. 5.3);
  * landmark points of each lens law (where a 90 or 45 degree ray lands) and
    of the equirectangular map (straight ahead, sideways, behind);
  * the small-angle limit, where every radial model is the equidistant one
    to third order.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2409_04751_amd import synth

FX, FY, CX, CY = 357.7, 331.3, 400.0, 300.0
RADIAL = [synth.MODEL_PINHOLE, synth.MODEL_EQUISOLID, synth.MODEL_ORTHOGRAPHIC, synth.MODEL_STEREOGRAPHIC]
ALL_OTHER = RADIAL + [synth.MODEL_PANORAMA]


def _points(model, rng, count):
    """Random camera-space points inside the model's domain (incidence below
    0.4 pi for the pinhole and orthographic models, 0.9 pi otherwise;
    panorama latitude within 0.4 pi and longitude off the rear seam),
    distances 0.3-30."""
    pts = []
    for _ in range(count):
        r = math.exp(rng.uniform(math.log(0.3), math.log(30)))
        if model == synth.MODEL_PANORAMA:
            lon = rng.uniform(-0.95 * math.pi, 0.95 * math.pi)
            lat = rng.uniform(-0.4 * math.pi, 0.4 * math.pi)
            pts.append([r * math.cos(lat) * math.sin(lon), r * math.sin(lat), r * math.cos(lat) * math.cos(lon)])
        else:
            top = 0.4 * math.pi if model in (synth.MODEL_PINHOLE, synth.MODEL_ORTHOGRAPHIC) else 0.9 * math.pi
            theta = rng.uniform(0.01, top)
            psi = rng.uniform(0, 2 * math.pi)
            pts.append([r * math.sin(theta) * math.cos(psi), r * math.sin(theta) * math.sin(psi), r * math.cos(theta)])
    return np.array(pts)


def _fd(f, p, h):
    cols = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        cols.append((f(p + e) - f(p - e)) / (2 * h))
    return np.stack(cols, axis=-1)


@pytest.mark.parametrize("model", ALL_OTHER)
def test_jacobian_matches_finite_differences(model):
    rng = np.random.default_rng(10 + model)
    for p in _points(model, rng, 200):
        J = oracle.jacobian_model(model, p, FX, FY)
        Jfd = _fd(lambda q: oracle.project_model(model, q, FX, FY, CX, CY), p, 1e-6 * np.linalg.norm(p))
        assert np.abs(J - Jfd).max() <= 1e-7 * np.abs(Jfd).max(), (p, J, Jfd)


@pytest.mark.parametrize("model", ALL_OTHER)
def test_jacobian_grad_matches_finite_differences(model):
    rng = np.random.default_rng(20 + model)
    for p in _points(model, rng, 200):
        dJ = oracle.jacobian_grad_model(model, p, FX, FY)
        h = 1e-6 * np.linalg.norm(p)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fd = (oracle.jacobian_model(model, p + e, FX, FY) - oracle.jacobian_model(model, p - e, FX, FY)) / (2 * h)
            scale = max(np.abs(fd).max(), np.abs(dJ).max())
            assert np.abs(dJ[c] - fd).max() <= 2e-6 * scale, (p, c, dJ[c], fd)


def test_equidistant_dispatch_is_the_paper_form():
    """Model 0 through the dispatcher is the paper's closed form."""
    rng = np.random.default_rng(3)
    for p in _points(synth.MODEL_EQUISOLID, rng, 50):
        np.testing.assert_array_equal(oracle.project_model(0, p, FX, FY, CX, CY), oracle.project(p, FX, FY, CX, CY))
        np.testing.assert_array_equal(oracle.jacobian_model(0, p, FX, FY), oracle.jacobian(p, FX, FY))
        np.testing.assert_array_equal(oracle.jacobian_grad_model(0, p, FX, FY), oracle.jacobian_grad(p, FX, FY))


def test_pinhole_is_textbook():
    """mu_p = c + f (x/z, y/z) and the EWA-splatting Jacobian of 3DGS."""
    rng = np.random.default_rng(4)
    for p in _points(synth.MODEL_PINHOLE, rng, 100):
        x, y, z = p
        np.testing.assert_allclose(oracle.project_model(1, p, FX, FY, CX, CY), [CX + FX * x / z, CY + FY * y / z],
                                   rtol=1e-13)
        np.testing.assert_allclose(oracle.jacobian_model(1, p, FX, FY),
                                   [[FX / z, 0.0, -FX * x / z ** 2], [0.0, FY / z, -FY * y / z ** 2]],
                                   rtol=1e-12, atol=1e-12 * FX / z)


@pytest.mark.parametrize("model,theta_deg,radius", [
    (synth.MODEL_PINHOLE, 45.0, 1.0),                       # tan 45 = 1
    (synth.MODEL_EQUISOLID, 90.0, math.sqrt(2.0)),          # 2 sin 45
    (synth.MODEL_EQUISOLID, 180.0 * 0.9, 2.0 * math.sin(0.45 * math.pi)),
    (synth.MODEL_ORTHOGRAPHIC, 90.0 * 0.999, math.sin(0.4995 * math.pi)),
    (synth.MODEL_ORTHOGRAPHIC, 30.0, 0.5),                  # sin 30
    (synth.MODEL_STEREOGRAPHIC, 90.0, 2.0),                 # 2 tan 45
    (synth.MODEL_STEREOGRAPHIC, 60.0, 2.0 / math.sqrt(3.0)),
])
def test_radial_lens_landmarks(model, theta_deg, radius):
    """Where a ray at a given incidence lands, for f = 100, on four azimuths."""
    f = 100.0
    th = math.radians(theta_deg)
    for psi in (0.0, 0.7, 2.0, -2.5):
        p = 3.0 * np.array([math.sin(th) * math.cos(psi), math.sin(th) * math.sin(psi), math.cos(th)])
        mp = oracle.project_model(model, p, f, f, 0.0, 0.0)
        np.testing.assert_allclose(mp, f * radius * np.array([math.cos(psi), math.sin(psi)]), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("model", RADIAL)
def test_radial_models_are_equidistant_near_the_axis(model):
    """r(theta) = theta + O(theta^3) for every listed lens: near the axis the
    image point and J approach the equidistant model's."""
    for th in (1e-3, 1e-2):
        p = 2.0 * np.array([math.sin(th) * 0.6, math.sin(th) * 0.8, math.cos(th)])
        a = oracle.project_model(model, p, FX, FX, 0.0, 0.0)
        b = oracle.project(p, FX, FX, 0.0, 0.0)
        assert np.abs(a - b).max() <= FX * th ** 3
        Ja, Jb = oracle.jacobian_model(model, p, FX, FX), oracle.jacobian(p, FX, FX)
        assert np.abs(Ja - Jb).max() <= 2.0 * th ** 2 * np.abs(Jb).max()


def _paper_panorama_jacobian(p, W, H):
    """The J of the panorama as printed in Sec. 5.3 (image width W, height H)."""
    x, y, z = p
    r2 = x * x + z * z
    l2 = x * x + y * y + z * z
    return np.array([[W * z / (2 * math.pi * r2), 0.0, -W * x / (2 * math.pi * r2)],
                     [-H * x * y / (math.pi * math.sqrt(r2) * l2), H * math.sqrt(r2) / (math.pi * l2),
                      -H * y * z / (math.pi * math.sqrt(r2) * l2)]])


def test_panorama_jacobian_is_the_printed_one():
    W, H = 2048, 1024
    cam = synth.panorama_camera(W, H)
    rng = np.random.default_rng(5)
    for p in _points(synth.MODEL_PANORAMA, rng, 200):
        J = oracle.jacobian_model(2, p, cam.fx, cam.fy)
        np.testing.assert_allclose(J, _paper_panorama_jacobian(p, W, H), rtol=1e-12,
                                   atol=1e-12 * np.abs(J).max())


def test_panorama_landmarks():
    """Equirectangular map of a W x H image: straight ahead is the centre,
    90 degrees right / left are at 3W/4 and W/4, straight behind is the
    left/right edge, 45 degrees down (+y) is at 3H/4; equal angles give
    equal pixel steps."""
    W, H = 2048, 1024
    cam = synth.panorama_camera(W, H)
    pr = lambda p: oracle.project_model(2, np.asarray(p, float), cam.fx, cam.fy, cam.cx, cam.cy)
    np.testing.assert_allclose(pr([0, 0, 5]), [W / 2, H / 2], atol=1e-12)
    np.testing.assert_allclose(pr([2, 0, 0]), [3 * W / 4, H / 2], atol=1e-9)
    np.testing.assert_allclose(pr([-2, 0, 0]), [W / 4, H / 2], atol=1e-9)
    np.testing.assert_allclose(pr([1e-12, 0, -1]), [W, H / 2], atol=1e-6)
    np.testing.assert_allclose(pr([-1e-12, 0, -1]), [0, H / 2], atol=1e-6)
    np.testing.assert_allclose(pr([0, 1, 1]), [W / 2, 3 * H / 4], atol=1e-9)
    steps = [pr([math.sin(a), 0.3, math.cos(a)])[0] for a in (0.1, 0.3, 0.5)]
    assert steps[1] - steps[0] == pytest.approx(steps[2] - steps[1], rel=1e-12)
    assert oracle.cull_angle(2, [0.0, -3.0, 3.0]) == pytest.approx(math.pi / 4, rel=1e-15)


@pytest.mark.parametrize("model", ALL_OTHER)
def test_tiled_equals_bruteforce(model):
    """Tile lists, sort and ranges under every camera model: the tiled blend
    equals the untiled per-pixel blend over all survivors."""
    rng = np.random.default_rng(30 + model)
    n = 48
    sc = synth.shell_scene(n, model)
    sc.scales[:] = np.exp(rng.normal(-2.5, 0.6, size=(3, n))).astype(np.float32)
    if model == synth.MODEL_PANORAMA:
        cam = synth.panorama_camera(96, 48)
    else:
        fov = 100.0 if model == synth.MODEL_PINHOLE else (170.0 if model == synth.MODEL_ORTHOGRAPHIC else 190.0)
        cam = synth.fisheye_camera(64, 48, fov, model=model)
    out = oracle.render(sc, synth.identity_pose(), cam, (0.1, 0.2, 0.3))
    brute = oracle.blend_bruteforce(out["pre"], cam, (0.1, 0.2, 0.3))
    assert out["pre"]["visible"].sum() > 5
    np.testing.assert_array_equal(out["image"], brute)
