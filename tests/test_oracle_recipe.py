"""Pins for the oracle's binary32 key recipe of the tight binning.

The tight binning keeps a tile of a Gaussian's 3-sigma rect only if the
Gaussian's alpha >= 1/255 ellipse (Eq. 3 weights with the 3DGS cut-off),
grown by 1% in radius and padded by 1/8 px, reaches the tile's pixel centres.
The oracle decides this rule two ways: in fp64 (its definition, "tight64")
and by a fixed sequence of binary32 operations on the float record of the
splat ("tight", the key recipe the renderer's decisions are compared with).
Pinned here:

  * a circular splat (B = 0, A = C): the kept tiles are those whose pixel-
    centre box, padded by 1/8 px, meets the disk of the grown radius -- a
    closed form in fp64, independent of both implementations;
  * the recipe keeps the same tiles as the fp64 rule for every Gaussian
    whose decisions the rule does not find within its margin band, on the
    shell and room workloads;
  * the recipe never drops a tile in which some pixel blends the Gaussian
    (brute force over pixels in fp64), and a planted error in the recipe's
    inputs (a transposed conic) is caught by that check.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2409_04751_amd import synth


def _pre(mu, conic, cov, opac, rect):
    n = len(opac)
    return dict(visible=np.ones(n, np.uint8), mu_p=np.ascontiguousarray(mu, np.float64),
                conic=np.ascontiguousarray(conic, np.float64), cov2d=np.ascontiguousarray(cov, np.float64),
                opacity=np.ascontiguousarray(opac, np.float64), rect=np.ascontiguousarray(rect, np.int32),
                tiles=np.zeros(n, np.uint32), tie=np.zeros(n, np.uint8))


def _kept(pre, i):
    """Kept (tile column, tile row) set of Gaussian i under the recipe."""
    alts = oracle.tight_alternatives(pre, i)
    r = pre["rect"][i]
    out = set()
    for row, (c0, c1) in enumerate(alts[0]):
        out |= {(tx, r[1] + row) for tx in range(c0, c1)}
    return out, len(alts)


def test_circle_closed_form():
    """B = 0, A = C = 1 / v: the reach is the disk |p - mu| <= rho with
    rho^2 = 2 ln(255 o) 1.0201 v, and a tile is kept iff the disk meets its
    pixel-centre box [16 tx, 16 tx + 15] x [16 ty, 16 ty + 15] padded by 1/8."""
    rng = np.random.default_rng(11)
    n = 400
    mu = rng.uniform(-40.0, 296.0, size=(n, 2))
    v = np.exp(rng.uniform(np.log(0.5), np.log(2000.0), n))
    o = rng.uniform(0.01, 0.99, n).astype(np.float32).astype(np.float64)
    conic = np.stack([1 / v, np.zeros(n), 1 / v], axis=1)
    cov = np.stack([v, np.zeros(n), v], axis=1)
    gx = gy = 16
    r = np.ceil(3 * np.sqrt(v + np.sqrt(0.1)))
    rect = np.stack([np.clip(np.floor((mu[:, 0] - r) / 16), 0, gx), np.clip(np.floor((mu[:, 1] - r) / 16), 0, gy),
                     np.clip(np.floor((mu[:, 0] + r + 15) / 16), 0, gx),
                     np.clip(np.floor((mu[:, 1] + r + 15) / 16), 0, gy)], axis=1).astype(np.int32)
    pre = _pre(mu, conic, cov, o, rect)
    checked = 0
    for i in range(n):
        x0, y0, x1, y1 = rect[i]
        if x1 <= x0 or y1 <= y0:
            continue
        p32 = float(np.float32(255.0) * np.float32(o[i]))
        rho2 = 2.0 * math.log(p32) * 1.0201 * v[i]
        got, _ = _kept(pre, i)
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                bx0, bx1 = 16 * tx - 0.125, 16 * tx + 15 + 0.125
                by0, by1 = 16 * ty - 0.125, 16 * ty + 15 + 0.125
                ddx = max(bx0 - mu[i, 0], 0.0, mu[i, 0] - bx1)
                ddy = max(by0 - mu[i, 1], 0.0, mu[i, 1] - by1)
                d2 = ddx * ddx + ddy * ddy
                if rho2 < 0:
                    want = False
                elif abs(math.sqrt(d2) - math.sqrt(rho2)) < 1e-3 * (1 + math.sqrt(rho2)):
                    continue  # within float rounding of the edge
                else:
                    want = d2 <= rho2
                assert ((tx, ty) in got) == want, (i, tx, ty, d2, rho2)
                checked += 1
    assert checked > 2000


def _agree_outside_band(scene, pose, cam):
    p32 = oracle.preprocess(scene, pose, cam, "tight")
    p64 = oracle.preprocess(scene, pose, cam, "tight64")
    band = (p64["tie"] & oracle.TIE_RULE) > 0
    rec_tie = (p32["tie"] & oracle.TIE_RECORD) > 0
    ok = ~band & ~rec_tie
    np.testing.assert_array_equal(p32["visible"][ok], p64["visible"][ok])
    np.testing.assert_array_equal(p32["tiles"][ok], p64["tiles"][ok])
    b32 = oracle.bin_and_sort(p32, cam)
    b64 = oracle.bin_and_sort(p64, cam)
    keep32 = ok[b32["vals"]]
    keep64 = ok[b64["vals"]]
    np.testing.assert_array_equal(b32["keys"][keep32], b64["keys"][keep64])
    np.testing.assert_array_equal(b32["vals"][keep32], b64["vals"][keep64])
    return int(band.sum()), int(rec_tie.sum()), int((p64["visible"] > 0).sum())


def test_recipe_equals_fp64_rule_shell():
    scene_fn, cam, poses = synth.workload("shell1k")
    band, rec, vis = _agree_outside_band(scene_fn(), poses[0], cam)
    assert vis > 500 and band < vis // 20


@pytest.mark.slow
def test_recipe_equals_fp64_rule_room():
    scene = synth.room_scene(60_000, 4, 0.01, 0)
    cam = synth.fisheye_camera(1752, 1168, 180.0)
    band, rec, vis = _agree_outside_band(scene, synth.identity_pose(), cam)
    assert vis > 20_000 and band < vis // 20
    print(f"visible {vis}, rule band {band}, record ties {rec}")


def _reaches_any(mu, con, o, tx, ty, cam):
    xs = np.arange(tx * 16, min(tx * 16 + 16, cam.width), dtype=np.float64)
    ys = np.arange(ty * 16, min(ty * 16 + 16, cam.height), dtype=np.float64)
    u = xs[None, :] - mu[0]
    w = ys[:, None] - mu[1]
    A, B, C = con
    q = -0.5 * (A * u * u + C * w * w) - B * u * w
    return bool(np.any(o * np.exp(q) >= 1.0 / 255.0))


def _dropped_but_reached(pre, cam, conic_override=None):
    """(Gaussian, tile) pairs of the rect the recipe drops although a pixel
    of the tile blends the Gaussian (in fp64)."""
    bad = []
    for i in np.nonzero(pre["visible"])[0]:
        x0, y0, x1, y1 = pre["rect"][i]
        alts = oracle.tight_alternatives(pre, i)
        con = pre["conic"][i] if conic_override is None else conic_override[i]
        for row, (c0, c1) in enumerate(alts[0]):
            ty = y0 + row
            for tx in range(x0, x1):
                if c0 <= tx < c1:
                    continue
                if _reaches_any(pre["mu_p"][i], con, pre["opacity"][i], tx, ty, cam):
                    bad.append((i, tx, ty))
    return bad


def test_recipe_is_conservative_and_catches_a_planted_error():
    cam = synth.fisheye_camera(96, 80, 190.0)
    rng = np.random.default_rng(5)
    n = 60
    means = np.stack([rng.uniform(-2, 2, n), rng.uniform(-2, 2, n), rng.uniform(0.5, 3, n)])
    scene = synth.Scene(means.astype(np.float32), np.exp(rng.normal(-2.5, 0.8, (3, n))).astype(np.float32),
                        rng.normal(size=(4, n)).astype(np.float32),
                        (1 / (1 + np.exp(-rng.normal(size=n)))).astype(np.float32),
                        rng.uniform(0, 1, (3, n)).astype(np.float32), 0)
    pre = oracle.preprocess(scene, synth.identity_pose(), cam, "rect")
    pre["binning"] = "tight"
    assert pre["visible"].sum() > 30
    assert _dropped_but_reached(pre, cam) == []
    # the same check with the conic's B term sign-flipped (a plausible
    # mistake in a record) finds reached pixels in dropped tiles
    flipped = pre["conic"].copy()
    flipped[:, 1] *= -1
    assert len(_dropped_but_reached(pre, cam, conic_override=flipped)) > 0
