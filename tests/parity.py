"""Helpers for GPU-vs-oracle parity tests (test infrastructure).

Runs the HIP path through the C ABI (via the package's ctypes binding), reads
the forward state back from the workspace at the offsets fgs_workspace_layout
reports, and compares it with the CPU oracle on the same seeded inputs.
"""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle
from paper_2409_04751_amd import render as R

LOG2E = 1.4426950408889634


def to_gpu(scene, device="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    return dict(means=t(scene.means), scales=t(scene.scales), quats=t(scene.quats), opacities=t(scene.opacity),
                sh=t(scene.sh), sh_degree=scene.sh_degree)


def _params(gs):
    return gs["means"], gs["scales"], gs["quats"], gs["opacities"], gs["sh"], gs["sh_degree"]


def gpu_forward(gs, pose, cam, bg=(0.0, 0.0, 0.0), save_pixel_state=False, workspace=None, k_hint=None):
    img, ws, K = R.render_forward(*_params(gs), pose, cam, bg, workspace=workspace,
                                  save_pixel_state=save_pixel_state, k_hint=k_hint)
    torch.cuda.synchronize()
    return img, ws, K


def read_state(ws, n, cam, K):
    """Forward state as numpy arrays."""
    lay = ws.layout(n, cam.width, cam.height)
    u32 = lambda off, cnt: ws.view(off, cnt, torch.int32).cpu().numpy().view(np.uint32)
    ntiles = lay.tiles_x * lay.tiles_y
    splats = ws.view(lay.splats, 12 * n, torch.float32).cpu().numpy().reshape(n, 3, 4).astype(np.float64)
    mu = splats[:, 0, 0:2] + splats[:, 0, 2:4]
    Ap, beta, Dp, q2min = splats[:, 1, 0], splats[:, 1, 1], splats[:, 1, 2], splats[:, 1, 3]
    A = Ap / (-0.5 * LOG2E)
    D = Dp / (-0.5 * LOG2E)
    B = beta * A
    C = D + B * beta
    rects = u32(lay.rects, 2 * n).reshape(n, 2)
    rect = np.stack([rects[:, 0] & 0xFFFF, rects[:, 0] >> 16, rects[:, 1] & 0xFFFF, rects[:, 1] >> 16], axis=1)
    return dict(
        mu_p=mu, conic=np.stack([A, B, C], axis=1), opacity=splats[:, 2, 0], rgb=splats[:, 2, 1:4], q2min=q2min,
        depth_bits=u32(lay.depth_keys, n), tiles=u32(lay.tiles, n), rect=rect.astype(np.int32),
        radius=ws.view(lay.radii, n, torch.int32).cpu().numpy(), depth_order=u32(lay.depth_order, n),
        tile_keys=u32(lay.tile_keys, K) if K else np.zeros(0, np.uint32),
        tile_ids=u32(lay.tile_ids, K) if K else np.zeros(0, np.uint32),
        ranges=u32(lay.ranges, 2 * ntiles).reshape(ntiles, 2), counters=u32(lay.counters, 16),
        pixel_T=ws.view(lay.pixel_T, cam.width * cam.height, torch.float32).cpu().numpy().reshape(cam.height, cam.width),
        pixel_last=u32(lay.pixel_last, cam.width * cam.height).reshape(cam.height, cam.width), layout=lay)


def compare_preprocess(st, pre, report=None):
    """Integer decisions bit-exact (except Gaussians the oracle marks as a tie),
    records to fp32 accuracy."""
    vis_o = pre["visible"] > 0
    vis_g = st["tiles"] > 0
    tie = pre["tie"] > 0
    bad = (vis_o != vis_g) & ~tie
    assert not bad.any(), f"visibility differs for {np.nonzero(bad)[0][:10]}"
    both = vis_o & vis_g & ~tie
    np.testing.assert_array_equal(st["radius"][both], pre["radius"][both])
    np.testing.assert_array_equal(st["rect"][both], pre["rect"][both])
    np.testing.assert_array_equal(st["tiles"][both], pre["tiles"][both])
    np.testing.assert_array_equal(st["depth_bits"][both], pre["depth"][both].view(np.uint32))
    assert np.all(st["depth_bits"][~vis_g] == 0xFFFFFFFF)
    # fp64 geometry rounded to float hi + lo: ~1e-12 px
    np.testing.assert_allclose(st["mu_p"][both], pre["mu_p"][both], rtol=0, atol=1e-6)
    # conic through the float record (A, B/A, D): relative ~1e-7 of the matrix scale
    scale = np.abs(pre["conic"][both]).max(axis=1, keepdims=True)
    assert np.all(np.abs(st["conic"][both] - pre["conic"][both]) <= 2e-6 * scale)
    np.testing.assert_allclose(st["rgb"][both], pre["rgb"][both], rtol=0, atol=2e-6)
    if report is not None:
        report["ties"] = int(tie.sum())
        report["visible"] = int(vis_o.sum())
    return both


def compare_tile_lists(st, bins, pre):
    """Sorted (tile, id) lists and ranges bit-exact; Gaussians the oracle
    marks as ties are removed from both lists first."""
    tie = pre["tie"] > 0
    keys_o = (bins["keys"] >> np.uint64(32)).astype(np.uint32)
    ids_o = bins["vals"]
    keys_g, ids_g = st["tile_keys"], st["tile_ids"]
    if tie.any():
        ko = ~tie[ids_o]
        kg = ~tie[ids_g]
        np.testing.assert_array_equal(keys_g[kg], keys_o[ko])
        np.testing.assert_array_equal(ids_g[kg], ids_o[ko])
    else:
        np.testing.assert_array_equal(keys_g, keys_o)
        np.testing.assert_array_equal(ids_g, ids_o)
        np.testing.assert_array_equal(st["ranges"], bins["ranges"])


def image_tolerance_check(img_gpu, ora, tol=1e-4):
    """max |gpu - oracle| <= tol * max(1, |ref|_inf) over pixels the oracle
    does not flag as within margin of a discrete threshold.  Returns stats."""
    ref = ora["image"]
    diff = np.abs(img_gpu.astype(np.float64) - ref)
    ok = ora["flags"] == 0
    bound = tol * max(1.0, float(np.abs(ref).max()))
    worst = float(diff[:, ok].max()) if ok.any() else 0.0
    assert worst <= bound, f"max image error {worst:.3e} > {bound:.3e}"
    return dict(max_err=worst, flagged=int((~ok).sum()), pixels=int(ok.size))


def gradient_check(g_gpu: dict, g_ora: dict, rel_l2=1e-4, elem=1e-4, floor=1e-2):
    """Per parameter block: ||d||/||ref|| <= rel_l2 and
    |d| <= elem * max(|ref|, floor * |ref|_inf) elementwise."""
    stats = {}
    for name in ("means", "scales", "quats", "opacity", "sh"):
        gk = "opacities" if name == "opacity" else name
        a = g_gpu[gk].detach().cpu().numpy().astype(np.float64)
        b = g_ora[name]
        nb = np.linalg.norm(b)
        rel = float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))
        m = float(np.abs(b).max()) if b.size else 0.0
        bad = np.abs(a - b) > elem * np.maximum(np.abs(b), floor * m)
        stats[name] = dict(rel_l2=rel, n_bad=int(bad.sum()), max_abs=float(np.abs(a - b).max()) if b.size else 0.0)
        assert rel <= rel_l2, (name, stats[name])
        assert not bad.any(), (name, stats[name], np.argwhere(bad)[:5])
    return stats


def masked_upstream(ora, rng, cam, scale=1.0):
    """Random dL/dimage with zeros on pixels whose decisions the oracle flags."""
    g = rng.normal(size=(3, cam.height, cam.width)) * scale
    g[:, ora["flags"] > 0] = 0.0
    return g.astype(np.float32)
