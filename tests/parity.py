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


def gpu_forward(gs, pose, cam, bg=(0.0, 0.0, 0.0), save_pixel_state=False, workspace=None, k_hint=None,
                binning="tight"):
    img, ws, K = R.render_forward(*_params(gs), pose, cam, bg, workspace=workspace,
                                  save_pixel_state=save_pixel_state, k_hint=k_hint, binning=binning)
    torch.cuda.synchronize()
    return img, ws, K


TIE_ANY = oracle.TIE_RECT | oracle.TIE_RECORD


def tie_mask(pre):
    """Gaussians whose tile decisions the oracle cannot fix uniquely: a
    radius or rect decision within 1e-9 of a boundary (fp64), or a float
    record whose other possible rounding keeps other tiles."""
    return (pre["tie"] & TIE_ANY) > 0


def check_k(K, pre, bins):
    """The intersection count equals the oracle's, except for tied Gaussians,
    whose kept tiles may differ -- by at most their rects.  Returns the
    number of tied Gaussians."""
    tie = tie_mask(pre)
    if not tie.any():
        assert K == bins["K"], (K, bins["K"])
        return 0
    r = pre["rect"][tie].astype(np.int64)
    slack = int(((r[:, 2] - r[:, 0]) * (r[:, 3] - r[:, 1])).sum())
    assert abs(K - bins["K"]) <= slack, (K, bins["K"], slack)
    return int(tie.sum())


def read_state(ws, n, cam, K):
    """Forward state as numpy arrays."""
    lay = ws.layout(n, cam.width, cam.height)
    u32 = lambda off, cnt: ws.view(off, cnt, torch.int32).cpu().numpy().view(np.uint32)
    ntiles = lay.tiles_x * lay.tiles_y
    splats = ws.view(lay.splats, 8 * n, torch.float32).cpu().numpy().reshape(n, 2, 4).astype(np.float64)
    colors = ws.view(lay.colors, 4 * n, torch.float32).cpu().numpy().reshape(n, 4).astype(np.float64)
    mu = splats[:, 0, 0:2] + splats[:, 0, 2:4]
    Ap, beta, Dp, q2min = splats[:, 1, 0], splats[:, 1, 1], splats[:, 1, 2], splats[:, 1, 3]
    A = Ap / (-0.5 * LOG2E)
    D = Dp / (-0.5 * LOG2E)
    B = beta * A
    C = D + B * beta
    rects = u32(lay.rects, 2 * n).reshape(n, 2)
    rect = np.stack([rects[:, 0] & 0xFFFF, rects[:, 0] >> 16, rects[:, 1] & 0xFFFF, rects[:, 1] >> 16], axis=1)
    return dict(
        mu_p=mu, conic=np.stack([A, B, C], axis=1), opacity=colors[:, 0], rgb=colors[:, 1:4], q2min=q2min,
        depth_bits=u32(lay.depth_keys, n), tiles=u32(lay.tiles, n), rect=rect.astype(np.int32),
        radius=ws.view(lay.radii, n, torch.int32).cpu().numpy(), depth_order=u32(lay.depth_order, n),
        tile_keys=u32(lay.tile_keys, K) if K else np.zeros(0, np.uint32),
        tile_ids=u32(lay.tile_ids, K) if K else np.zeros(0, np.uint32),
        ranges=u32(lay.ranges, 2 * ntiles).reshape(ntiles, 2), counters=u32(lay.counters, 16),
        pixel_T=ws.view(lay.pixel_T, cam.width * cam.height, torch.float32).cpu().numpy().reshape(cam.height, cam.width),
        pixel_last=u32(lay.pixel_last, cam.width * cam.height).reshape(cam.height, cam.width), layout=lay)


def compare_preprocess(st, pre, report=None):
    """Integer decisions bit-exact, records to fp32 accuracy.  A Gaussian
    whose radius or rect decision is an fp64 tie is compared for validity
    only; one whose tile count depends on the rounding of its float record
    has its count and visibility compared against the oracle's alternatives
    by compare_tile_lists."""
    vis_o = pre["visible"] > 0
    vis_g = st["tiles"] > 0
    rect_tie = (pre["tie"] & oracle.TIE_RECT) > 0
    tie = tie_mask(pre)
    bad = (vis_o != vis_g) & ~tie
    assert not bad.any(), f"visibility differs for {np.nonzero(bad)[0][:10]}"
    both = vis_o & vis_g & ~rect_tie
    np.testing.assert_array_equal(st["radius"][both], pre["radius"][both])
    np.testing.assert_array_equal(st["rect"][both], pre["rect"][both])
    np.testing.assert_array_equal(st["depth_bits"][both], pre["depth"][both].view(np.uint32))
    counted = both & ~tie
    np.testing.assert_array_equal(st["tiles"][counted], pre["tiles"][counted])
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


def _rows_of(keys, ids, g, gx, rect):
    """Kept column interval per rect row of Gaussian g from a sorted list."""
    sel = ids == g
    tiles = keys[sel].astype(np.int64)
    rows = np.zeros((int(rect[3] - rect[1]), 2), np.int64)
    for r in range(rows.shape[0]):
        cols = np.sort(tiles[tiles // gx == rect[1] + r] % gx)
        if cols.size:
            assert np.array_equal(cols, np.arange(cols[0], cols[0] + cols.size)), "kept columns not one interval"
            rows[r] = (cols[0], cols[-1] + 1)
    return rows


def _same_rows(a, b):
    a, b = np.asarray(a, np.int64), np.asarray(b, np.int64)
    ea, eb = a[:, 0] == a[:, 1], b[:, 0] == b[:, 1]
    return bool(np.all(ea == eb) and np.all((a == b)[~ea]))


def compare_tile_lists(st, bins, pre, cam, report=None):
    """Sorted (tile, id) lists and ranges bit-exact.  A tied Gaussian's pairs
    are checked on their own -- its kept intervals must be one of the
    oracle's alternatives (record ties) or lie in its rect (rect ties) -- and
    then left out of both lists; ranges are compared on every tile, with the
    tied pairs taken out of both lengths.  Returns the counts."""
    tie = tie_mask(pre)
    keys_o = (bins["keys"] >> np.uint64(32)).astype(np.uint32)
    ids_o = bins["vals"]
    keys_g, ids_g = st["tile_keys"], st["tile_ids"]
    gx = cam.tiles_x
    ntiles = cam.tiles_x * cam.tiles_y
    ko = ~tie[ids_o]
    kg = ~tie[ids_g]
    keys_t, ids_t = keys_g[~kg], ids_g[~kg]
    for g in np.nonzero(tie)[0]:
        if not (pre["tie"][g] & oracle.TIE_RECT):
            rows_g = _rows_of(keys_t, ids_t, g, gx, pre["rect"][g])
            alts = oracle.tight_alternatives(pre, int(g))
            assert any(_same_rows(rows_g, a) for a in alts), f"Gaussian {g}: kept tiles match no rounding"
        else:
            r = st["rect"][g]
            t = keys_t[ids_t == g].astype(np.int64)
            assert np.all((t % gx >= r[0]) & (t % gx < r[2]) & (t // gx >= r[1]) & (t // gx < r[3]))
    np.testing.assert_array_equal(keys_g[kg], keys_o[ko])
    np.testing.assert_array_equal(ids_g[kg], ids_o[ko])
    # ranges: lengths on every tile (tied pairs removed), starts wherever the
    # tile has entries (an empty tile's start is arbitrary: the oracle writes
    # 0, the GPU its insertion point)
    rg, ro = st["ranges"].astype(np.int64), bins["ranges"].astype(np.int64)
    tg = np.bincount(keys_g[~kg].astype(np.int64), minlength=ntiles)
    to = np.bincount(keys_o[~ko].astype(np.int64), minlength=ntiles)
    np.testing.assert_array_equal(rg[:, 1] - rg[:, 0] - tg, ro[:, 1] - ro[:, 0] - to)
    nz = rg[:, 1] > rg[:, 0]
    starts = np.concatenate([[0], np.cumsum(rg[:, 1] - rg[:, 0])[:-1]])
    np.testing.assert_array_equal(rg[nz, 0], starts[nz])
    if not tie.any():
        nzo = ro[:, 1] > ro[:, 0]
        np.testing.assert_array_equal(rg[nzo], ro[nzo])
    out = dict(K=int(keys_g.size), ties=int(tie.size and tie.sum()), excluded_pairs_gpu=int((~kg).sum()),
               excluded_pairs_oracle=int((~ko).sum()))
    print("tile lists:", out, flush=True)
    if report is not None:
        report.update(out)
    return out


def image_tolerance_check(img_gpu, ora, tol=1e-4):
    """max |gpu - oracle| <= tol * max(1, |ref|_inf) over pixels the oracle
    does not flag as within the binary32 error bound of a discrete threshold.
    Returns stats, with the error over every pixel (flagged ones included)
    for the record."""
    ref = ora["image"]
    diff = np.abs(img_gpu.astype(np.float64) - ref)
    ok = ora["flags"] == 0
    bound = tol * max(1.0, float(np.abs(ref).max()))
    worst = float(diff[:, ok].max()) if ok.any() else 0.0
    assert worst <= bound, f"max image error {worst:.3e} > {bound:.3e}"
    over = (diff > bound).any(axis=0)
    return dict(max_err=worst, max_err_all_pixels=float(diff.max()) if diff.size else 0.0,
                flagged=int((~ok).sum()), pixels=int(ok.size), flagged_frac=float((~ok).mean()),
                flagged_over_bound=int((over & ~ok).sum()))


def compare_pixel_state(st, ora):
    """With the forward's per-pixel state saved: the number of blended
    entries (last) equal on every unflagged pixel, T_final to fp32 accuracy."""
    ok = ora["flags"] == 0
    np.testing.assert_array_equal(st["pixel_last"][ok], ora["last"][ok])
    np.testing.assert_allclose(st["pixel_T"][ok], ora["T_final"][ok], rtol=2e-4, atol=1e-7)
    return int((st["pixel_last"][~ok] != ora["last"][~ok]).sum())


BLOCKS = ("means", "scales", "quats", "opacity", "sh")


def _gpu_block(g_gpu, name):
    return g_gpu["opacities" if name == "opacity" else name].detach().cpu().numpy().astype(np.float64)


def check_blocks_rel_l2(g_gpu: dict, g_ora: dict, tol=1e-4):
    """End to end, per parameter block: ||gpu - oracle|| / ||oracle|| <= tol."""
    stats = {}
    for name in BLOCKS:
        a, b = _gpu_block(g_gpu, name), g_ora[name]
        nb = np.linalg.norm(b)
        rel = float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))
        stats[name] = rel
        assert rel <= tol, (name, rel)
    return stats


ABS_SCALE = 1e-5  # the rounding scale of a float32 evaluation of a sum, per unit of its summed magnitudes


def check_blocks_elementwise(g_gpu: dict, g_ora: dict, rel=1e-4, floor=1e-3, err_scale: dict | None = None):
    """End to end, per element of each parameter block:
    |gpu - oracle| <= rel * max(|oracle|, floor * ||oracle||_inf)
                      + 1e-5 * (the element's rounding-error scale, if given).
    The error scale (oracle.chain_error_scale) is the sum of the magnitudes
    of the per-pixel terms behind the element, carried through the chain:
    with a random-signed upstream gradient an element can be a small
    difference of large float32 sums, and only there does it matter.  Reports
    how many elements exceed the first part alone ("over_plain")."""
    stats = {}
    for name in BLOCKS:
        a, b = _gpu_block(g_gpu, name), g_ora[name]
        inf = float(np.abs(b).max()) if b.size else 0.0
        plain = rel * np.maximum(np.abs(b), floor * inf)
        err = np.abs(a - b)
        bound = plain + (ABS_SCALE * err_scale[name] if err_scale is not None else 0.0)
        ratio = err / np.maximum(bound, 1e-300)
        bad = int((ratio > 1.0).sum())
        ratio_plain = err / np.maximum(plain, 1e-300)
        stats[name] = dict(worst=float(ratio.max()) if ratio.size else 0.0, over=bad,
                           worst_plain=float(ratio_plain.max()) if ratio.size else 0.0,
                           over_plain=int((ratio_plain > 1.0).sum()), elements=int(b.size))
        assert bad == 0, (name, stats[name], np.unravel_index(int(np.argmax(ratio)), ratio.shape))
    return stats


def read_grad2d(ws, n, cam):
    """The blend backward's per-Gaussian accumulators [n][9]: mu_p x y,
    conic A B C, opacity, rgb."""
    lay = ws.layout(n, cam.width, cam.height)
    groups = (n + 63) // 64
    buf = ws.view(lay.grad2d, 9 * 64 * groups, torch.float32).cpu().numpy().reshape(64 * groups, 9)
    ids = np.arange(n, dtype=np.int64)
    slot = (ids & ~63) | ((ids * 9) & 63)  # the layout's permutation inside each group of 64
    g = buf[slot].T.astype(np.float64)
    return dict(mu_p=np.ascontiguousarray(g[0:2].T), conic=np.ascontiguousarray(g[2:5].T),
                opacity=np.ascontiguousarray(g[5]), rgb=np.ascontiguousarray(g[6:9].T))


def _stack2d(g):
    return np.concatenate([g["mu_p"], g["conic"], g["opacity"][:, None], g["rgb"]], axis=1)


def _stack2d_abs(g):
    """Operand magnitudes of the 2D gradients plus their pixel-offset
    sensitivity times the float32 offset rounding, [n, 9]."""
    return g["abs"] + (POS_ROUNDING_PX / ABS_SCALE) * g["pos"]


POS_ROUNDING_PX = 2e-6  # float32 tile-relative pixel offsets up to 32 px


def check_2d(g2d_gpu: dict, g2d_ora: dict, rel=1e-4, abs_scale=1e-5):
    """Blend backward, elementwise: |gpu - oracle| <= rel |oracle| +
    abs_scale * (operand magnitudes summed over pixels) + 2e-6 px * (summed
    sensitivity to the pixel offset).  The second part is the rounding scale
    of a float32 evaluation of the per-pixel terms and their sum (random-signed
    upstream gradients make these sums cancel); the third covers the float32
    position of the splat, which matters for terms that vanish at its
    centre (d/dA ~ dx^2)."""
    a, b = _stack2d(g2d_gpu), _stack2d(g2d_ora)
    bound = rel * np.abs(b) + abs_scale * g2d_ora["abs"] + POS_ROUNDING_PX * g2d_ora["pos"]
    bad = np.abs(a - b) > bound
    assert not bad.any(), (int(bad.sum()), np.argwhere(bad)[:5], a[bad][:5], b[bad][:5])
    return dict(max_rel_to_abs=float(np.max(np.abs(a - b) / np.maximum(g2d_ora["abs"], 1e-300))))


def check_chain(g_gpu: dict, chain_ref: dict, rel=1e-5, col=1e-6):
    """Preprocess backward, elementwise, against the oracle's chain fed with
    the GPU's own 2D gradients: |gpu - ref| <= rel |ref| + col ||ref[:, i]||."""
    out = {}
    for name in BLOCKS:
        a, b = _gpu_block(g_gpu, name), chain_ref[name]
        colnorm = np.linalg.norm(b.reshape(-1, b.shape[-1]), axis=0)
        bad = np.abs(a - b) > rel * np.abs(b) + col * colnorm
        assert not bad.any(), (name, int(bad.sum()), np.argwhere(bad)[:5])
        out[name] = float(np.abs(a - b).max()) if b.size else 0.0
    return out


def gradient_parity(scene, pose, cam, ws, g_gpu, ora, dL, bg=(0.0, 0.0, 0.0)):
    """All three gradient checks; returns their statistics."""
    go = oracle.render_backward(scene, pose, cam, ora, dL, bg, abs_sums=True)
    stats = dict(rel_l2=check_blocks_rel_l2(g_gpu, go))
    print("rel_l2", stats["rel_l2"], flush=True)
    scale = oracle.chain_error_scale(scene, pose, cam, ora["pre"], _stack2d_abs(go["g2d"]))
    stats["elementwise"] = check_blocks_elementwise(g_gpu, go, err_scale=scale)
    g2d = read_grad2d(ws, scene.n, cam)
    stats["blend_2d"] = check_2d(g2d, go["g2d"])
    chain = oracle.preprocess_backward(scene, pose, cam, ora["pre"], g2d)
    stats["chain_max_abs"] = check_chain(g_gpu, chain)
    return stats, go


def masked_upstream(ora, rng, cam, scale=1.0):
    """Random dL/dimage with zeros on pixels whose decisions the oracle flags."""
    g = rng.normal(size=(3, cam.height, cam.width)) * scale
    g[:, ora["flags"] > 0] = 0.0
    return g.astype(np.float32)
