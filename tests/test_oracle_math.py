"""Pins for the oracle's projection, Jacobian, Jacobian derivative and SH basis.

Each check ties the oracle to something other than itself: the equidistant
closed form r = f theta (Sec. 3.2), central finite differences of the
projection and of J, the pinhole limit on the optical axis, and scipy's
spherical harmonics.  The paper's two printed typos (Sec. 4.2 J_phi theta
terms without f; Sec. 4.3 dJ/dy_c entry [0][2] with f_y) are kept as negative
controls: the printed forms must fail the same finite-difference test.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle

FX, FY, CX, CY = 557.7, 431.3, 876.0, 584.0


def _points(rng, count):
    """Random camera-space points spanning on-axis to far off-axis, both
    hemispheres (theta up to 0.9 pi), distances 0.3-30."""
    pts = []
    for _ in range(count):
        theta = rng.uniform(0.0, 0.9 * math.pi)
        psi = rng.uniform(0, 2 * math.pi)
        r = math.exp(rng.uniform(math.log(0.3), math.log(30)))
        pts.append([r * math.sin(theta) * math.cos(psi), r * math.sin(theta) * math.sin(psi), r * math.cos(theta)])
    # near-axis points on both sides of the series switch (u = l_z / z = 1e-2)
    for u in (1e-7, 1e-4, 3e-3, 9.99e-3, 1.001e-2, 3e-2):
        z = rng.uniform(0.5, 5)
        psi = rng.uniform(0, 2 * math.pi)
        pts.append([u * z * math.cos(psi), u * z * math.sin(psi), z])
    return np.array(pts)


def _fd_jacobian(f, p, h):
    cols = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        cols.append((f(p + e) - f(p - e)) / (2 * h))
    return np.stack(cols, axis=-1)


def test_equidistant_radius_is_f_theta():
    """Sec. 3.2: the image point lies at distance f theta from the principal
    point, in the azimuth of (x_c, y_c).  theta here is the angle between
    p and the optical axis by Kahan's formula 2 atan(|a - b| / |a + b|) on
    unit vectors, not the oracle's atan2(l_z, z_c)."""
    rng = np.random.default_rng(1)
    for p in _points(rng, 200):
        mp = oracle.project(p, FX, FY, CX, CY)
        a = p / np.linalg.norm(p)
        b = np.array([0.0, 0.0, 1.0])
        theta = 2 * math.atan(np.linalg.norm(a - b) / np.linalg.norm(a + b))
        lz = math.hypot(p[0], p[1])
        if lz == 0:
            continue
        assert (mp[0] - CX) / FX == pytest.approx(theta * p[0] / lz, rel=1e-12, abs=1e-12)
        assert (mp[1] - CY) / FY == pytest.approx(theta * p[1] / lz, rel=1e-12, abs=1e-12)


def test_equidistant_worked_example_256():
    """256x256 at 180 deg: f = 256/pi, so a point at 90 deg incidence lands
    128 px from the centre (the image edge), one at 45 deg at 64 px."""
    f = 256 / math.pi
    assert oracle.project([1.0, 0.0, 0.0], f, f, 128, 128) == pytest.approx([256.0, 128.0], abs=1e-12)
    assert oracle.project([0.0, -2.0, 2.0], f, f, 128, 128) == pytest.approx([128.0, 64.0], abs=1e-12)
    assert oracle.project([0.0, 0.0, 3.0], f, f, 128, 128) == pytest.approx([128.0, 128.0], abs=0)


def test_jacobian_matches_finite_differences():
    rng = np.random.default_rng(2)
    for p in _points(rng, 300):
        J = oracle.jacobian(p, FX, FY)
        Jfd = _fd_jacobian(lambda q: oracle.project(q, FX, FY, CX, CY), p, 1e-6 * np.linalg.norm(p))
        scale = np.abs(Jfd).max()
        assert np.abs(J - Jfd).max() <= 1e-7 * scale, (p, J, Jfd)


def test_jacobian_on_axis_is_pinhole():
    for z in (0.25, 1.0, 7.5):
        J = oracle.jacobian([0.0, 0.0, z], FX, FY)
        np.testing.assert_allclose(J, [[FX / z, 0, 0], [0, FY / z, 0]], rtol=1e-15, atol=0)


def test_jacobian_grad_matches_finite_differences():
    rng = np.random.default_rng(3)
    for p in _points(rng, 300):
        dJ = oracle.jacobian_grad(p, FX, FY)  # [coord, 2, 3]
        h = 1e-6 * np.linalg.norm(p)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fd = (oracle.jacobian(p + e, FX, FY) - oracle.jacobian(p - e, FX, FY)) / (2 * h)
            scale = max(np.abs(fd).max(), np.abs(dJ).max())
            assert np.abs(dJ[c] - fd).max() <= 2e-6 * scale, (p, c, dJ[c], fd)


def test_series_branch_is_continuous():
    """J and dJ just below and above the near-axis switch agree."""
    z = 2.0
    a = np.array([1e-2 * z * (1 - 1e-12) / math.sqrt(2), 1e-2 * z * (1 - 1e-12) / math.sqrt(2), z])
    b = np.array([1e-2 * z * (1 + 1e-12) / math.sqrt(2), 1e-2 * z * (1 + 1e-12) / math.sqrt(2), z])
    np.testing.assert_allclose(oracle.jacobian(a, FX, FY), oracle.jacobian(b, FX, FY), rtol=1e-9, atol=1e-9)
    ga, gb = oracle.jacobian_grad(a, FX, FY), oracle.jacobian_grad(b, FX, FY)
    assert np.abs(ga - gb).max() <= 1e-8 * np.abs(ga).max()


# ---- negative controls: the formulas exactly as printed -------------------

def _printed_jacobian(p, fx, fy):
    """Sec. 4.2 as printed: the theta terms carry no focal length."""
    x, y, z = p
    lz2 = x * x + y * y
    l2 = lz2 + z * z
    lz = math.sqrt(lz2)
    th = math.atan2(lz, z)
    return np.array([
        [fx * x * x * z / (lz2 * l2) + y * y * th / lz ** 3, x * y * (fx * z / (lz2 * l2) - th / lz ** 3), -fx * x / l2],
        [x * y * (fy * z / (lz2 * l2) - th / lz ** 3), fy * y * y * z / (lz2 * l2) + x * x * th / lz ** 3, -fy * y / l2],
    ])


def test_printed_jacobian_fails_fd():
    p = np.array([0.7, -0.4, 1.3])
    Jfd = _fd_jacobian(lambda q: oracle.project(q, FX, FY, CX, CY), p, 1e-6)
    assert np.abs(_printed_jacobian(p, FX, FY) - Jfd).max() > 1.0
    assert np.abs(oracle.jacobian(p, FX, FY) - Jfd).max() < 1e-5


def test_printed_dJdy_entry_fails_fd():
    """dJ[0][2]/dy_c printed as 2 f_y x y / l_2^2; finite differences say f_x."""
    p = np.array([0.7, -0.4, 1.3])
    h = 1e-6
    e = np.array([0, h, 0])
    fd = (oracle.jacobian(p + e, FX, FY) - oracle.jacobian(p - e, FX, FY)) / (2 * h)
    l2 = float(p @ p)
    printed = 2 * FY * p[0] * p[1] / l2 ** 2
    corrected = 2 * FX * p[0] * p[1] / l2 ** 2
    assert abs(fd[0, 2] - corrected) < 1e-6 * abs(corrected)
    assert abs(fd[0, 2] - printed) > 0.1 * abs(corrected)


# ---- spherical harmonics --------------------------------------------------

def _real_sh_scipy(l, m, d):
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0])
    if hasattr(sp, "sph_harm_y"):
        Y = complex(sp.sph_harm_y(l, abs(m), theta, phi))
    else:  # older scipy: (m, n, azimuth, polar)
        Y = complex(sp.sph_harm(abs(m), l, phi, theta))
    if m == 0:
        return Y.real
    if m > 0:
        return math.sqrt(2) * Y.real
    return math.sqrt(2) * Y.imag


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(4)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                assert Y[l * (l + 1) + m] == pytest.approx(_real_sh_scipy(l, m, d), abs=1e-12), (l, m)


def test_sh_basis_orthonormal():
    """Gauss-Legendre in cos(polar) x uniform azimuth integrates degree <= 6
    products exactly."""
    xs, ws = np.polynomial.legendre.leggauss(12)
    nphi = 16
    G = np.zeros((16, 16))
    for z, w in zip(xs, ws):
        s = math.sqrt(1 - z * z)
        for j in range(nphi):
            phi = 2 * math.pi * j / nphi
            Y = oracle.sh_basis(3, [s * math.cos(phi), s * math.sin(phi), z])
            G += np.outer(Y, Y) * w * (2 * math.pi / nphi)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_dc_constant():
    """Y_00 = 1 / (2 sqrt(pi)) everywhere."""
    assert oracle.sh_basis(0, [0.0, 0.6, 0.8])[0] == pytest.approx(0.5 / math.sqrt(math.pi), rel=1e-15)
