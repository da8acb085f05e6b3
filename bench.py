#!/usr/bin/env python3
"""Fisheye Gaussian-splatting fwd+bwd benchmark on one MI355X.

Workload (the headline configuration): 3,000,000 Gaussians, SH degree 3,
fp32 parameters, means uniform in a 10 x 4 x 10 m room, log-scales
N(-4, 0.7) with 1% large N(-1, 0.5), one 1752x1168 equidistant-fisheye view
at 180 deg from the room centre, L1 loss against a seeded random target.

One step = one view through the differentiable rasterizer: preprocess, depth
sort, tile duplication, tile sort, ranges, blend, then the backward with
transmittance recomputation (blend backward, preprocess backward), driven by
torch autograd with the L1 loss.  Inputs are resident in HBM before timing.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ms/view @3M Gaussians 1752×1168; served views/s + p99 vs plain"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(name: str, N: int, V: int, K: int, P: int, S: int) -> float | None:
    """Algorithmic HBM bytes of ONE launch of `name` (byte model)."""
    if name == "preprocess":  # one view: geometry and colour fused, plus the colour's direction gradient
        return 52.0 * N + (4.0 * S + 124.0) * V
    if name == "color":
        return 4.0 * N + (4.0 * S + 32.0) * V
    if name == "depth_sort_scatter":
        return 16.0 * N
    if name == "depth_sort_hist":
        return 4.0 * N
    if name == "duplicate":  # K pairs out, in the tile sort's first-pass order, with 16-bit keys (the rows'
        # offsets, ids and columns are read once per row)
        return 6.0 * K
    if name == "tile_sort_hist":  # the second pass's histogram over the 16-bit keys
        return 2.0 * K
    if name == "tile_sort_scatter":  # the second pass: 16-bit keys and ids in, 32-bit keys and ids out
        return 14.0 * K
    if name == "ranges":
        return 4.0 * K
    if name == "preprocess_backward":  # colour and geometry parts in one launch: tile count and mean of
        # every Gaussian, the colour's direction gradient, scale, quaternion, opacity and 2D gradient slot
        # of the visible ones in; dL/dSH and dL/d(mu, s, q, o) of every Gaussian out
        return 16.0 * N + 116.0 * V + (4.0 * S + 44.0) * N
    return None


def path_bytes(N: int, V: int, K: int, P: int, S: int) -> float:
    """Algorithmic HBM bytes of one whole fwd+bwd view: every array the tile
    method needs, read or written the fewest times it must be (the sort as one
    read + write of the K pairs; extra radix passes are overhead):
    52 N + (12 S + 316) V + 124 K + 44 P."""
    return 52.0 * N + (12.0 * S + 316.0) * V + 124.0 * K + 44.0 * P


def path_bytes_staged(N: int, V: int, K: int, P: int, S: int, staged: int) -> float:
    """The same view's bytes with the two blends counted for the entries they
    actually stage: both stop at saturation, so each reads, per tile, the
    records of its list only up to the tile's last blended entry (`staged`
    = the sum over tiles of that count) instead of all K."""
    return path_bytes(N, V, K, P, S) - 80.0 * K + 80.0 * staged


def forward_bytes(N: int, V: int, K: int, P: int, S: int) -> float:
    """Algorithmic bytes of a forward-only view (preprocess, scan,
    duplication, sort, ranges, blend): 52 N + (4 S + 72) V + 84 K + 16 P."""
    return 52.0 * N + (4.0 * S + 72.0) * V + 84.0 * K + 16.0 * P


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_room3m_1752x1168.json")


def traffic_for(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if there is
    none or it was taken on other sources than the current ones."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha") != source_sha():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


# Floating-point operations of the blend backward (an FMA counts 2, exp2 and
# rcp count 1 each).  The autograd path keeps no per-pixel state, so the
# backward first re-sweeps front to back: every (pixel, entry) pair up to the
# pixel's last blended entry evaluates the exponent (9) and tests it (1); a
# pair that blends adds alpha 3 (exp2, scale, clamp), 1 - alpha, the new
# transmittance and the stop test (3).  The reverse pass then evaluates and
# tests the exponent again (10); a pair that blends adds alpha 3,
# transmittance in front 3, colour gradient 7, colour difference 3,
# dL/dalpha 6, colour behind 6, opacity term 2, dL/dq 1 and the mean and
# conic terms 16.
BLEND_BWD_FLOPS_TESTED = 10.0 + 10.0
BLEND_BWD_FLOPS_BLENDED = 6.0 + 47.0


def staged_entries(ws, lay) -> int:
    """Sum over tiles of the tile's largest per-pixel count of blended
    entries (the saved per-pixel state): the entries a blend that stops at
    saturation reads of each list."""
    import torch

    W, H, tx, ty = lay.width, lay.height, lay.tiles_x, lay.tiles_y
    last = ws.view(lay.pixel_last, W * H, torch.int32).view(H, W)
    pad = torch.zeros((ty * 16, tx * 16), dtype=torch.int32, device=last.device)
    pad[:H, :W] = last
    return int(pad.view(ty, 16, tx, 16).amax(dim=(1, 3)).sum().item())


def contributing_pairs(ws, lay, n: int, K: int) -> tuple[int, int]:
    """(E_b, C) of the blend backward: E_b = (pixel, entry) pairs up to each
    pixel's last blended entry (the sum of the saved counts); C = those whose
    alpha is at least 1/255 at the pixel, evaluated from the library's own
    state in fp64."""
    import torch

    tx, ty = lay.tiles_x, lay.tiles_y
    W, H = lay.width, lay.height
    rng = ws.view(lay.ranges, 2 * tx * ty, torch.int32).view(-1, 2).long()
    ids = ws.view(lay.tile_ids, K, torch.int32).long()
    sp = ws.view(lay.splats, 8 * n, torch.float32).view(n, 8).double()
    last = ws.view(lay.pixel_last, W * H, torch.int32).long()
    counts = (rng[:, 1] - rng[:, 0]).clamp_min(0)
    tile = torch.repeat_interleave(torch.arange(tx * ty, device=ids.device), counts)
    assert tile.numel() == K
    rel = torch.arange(K, device=ids.device) - rng[tile, 0]
    u = torch.arange(16, device=ids.device)
    total = 0
    step = 1 << 19
    for s in range(0, K, step):
        e = min(K, s + step)
        g = ids[s:e]
        t = tile[s:e]
        px = (t % tx)[:, None, None] * 16 + u[None, None, :]
        py = (t // tx)[:, None, None] * 16 + u[None, :, None]
        inside = (px < W) & (py < H)
        rec = sp[g]
        dx = (rec[:, 0] + rec[:, 2])[:, None, None] - px
        dy = (rec[:, 1] + rec[:, 3])[:, None, None] - py
        q = dx + rec[:, 5][:, None, None] * dy
        q2 = rec[:, 4][:, None, None] * q * q + rec[:, 6][:, None, None] * dy * dy
        lp = last[(py.clamp(max=H - 1) * W + px.clamp(max=W - 1))]
        ok = inside & (q2 >= rec[:, 7][:, None, None]) & (rel[s:e][:, None, None] < lp)
        total += int(ok.sum().item())
    return int(last.sum().item()), total


def source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2409_04751_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_view(scene, pose, cam, target) -> float:
    import numpy as np

    import oracle

    t0 = time.perf_counter()
    ora = oracle.render(scene, pose, cam)
    g = (np.sign(ora["image"] - target) / ora["image"].size).astype(np.float32)
    oracle.render_backward(scene, pose, cam, ora, g)
    return (time.perf_counter() - t0) * 1000.0


def cpu_baseline(scene, pose, cam, target, small):
    """The oracle (plain fp64 C, OpenMP) timed on the host: the benchmark view
    (fwd + bwd) three times on every host thread, median; and once on one
    thread for a bounded sample, the 500k-Gaussian view `small` = (scene,
    pose, cam, target), so the single-thread rate is measured rather than
    extrapolated."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.lib().orc_set_threads(threads)
    runs = sorted(_oracle_view(scene, pose, cam, target) for _ in range(3))
    oracle.lib().orc_set_threads(1)
    one = _oracle_view(*small)
    oracle.lib().orc_set_threads(threads)
    return dict(value=round(runs[1], 1), unit="ms/view", cores=threads, kind="oracle",
                sample="the benchmark view (3M Gaussians, 1752x1168, fwd + bwd, fp64), median of 3 runs on "
                       "every host thread",
                runs_ms=[round(r, 1) for r in runs], cpu_model=cpu_model(),
                single_thread=dict(value=round(one, 1), unit="ms/view",
                                   sample="the 500k-Gaussian SH3 1752x1168 view, fwd + bwd, one run on 1 thread"))


SERVE_P99_BOUND_MS = 20.0


def serving_bench(params, deg, rates, count):
    """Resident scene; open-loop Poisson requests, each a random pose in the
    room, resolution from {512^2, 1024^2, 1752x1168, 2048^2}, FOV U(150, 200)
    deg.  Batched server vs serial rendering on the same trace."""
    from paper_2409_04751_amd import server as S

    srv = S.RenderServer(*params, deg, workspace_bytes=16 << 30)
    warm = S.poisson_trace(2000.0, 24, seed=99)
    srv.serve(warm, "batched")
    srv.serve(warm, "serial")
    out = dict(scene="room3m resident (3M Gaussians, SH3)", requests_per_rate=count,
               resolutions=["512x512", "1024x1024", "1752x1168", "2048x2048"], fov_deg=[150, 200], rates={})
    for rate in rates:
        trace = S.poisson_trace(rate, count, seed=3)
        res = {}
        for mode in ("serial", "batched"):
            srv.batches = srv.splits = 0
            r = srv.serve(trace, mode)
            res[mode] = {k: round(v, 3) if isinstance(v, float) else v for k, v in r.items()}
            log(f"serve rate={rate:g}/s {mode}: p50 {r['p50_ms']:.2f} ms p99 {r['p99_ms']:.2f} ms "
                f"{r['views_per_s']:.0f} views/s")
        res["batched_over_serial_views_per_s"] = round(res["batched"]["views_per_s"] / res["serial"]["views_per_s"], 3)
        out["rates"][f"{rate:g}"] = res
    # the highest offered rate each mode keeps up with (views/s within 3% of
    # the offered rate) at a p99 latency within the bound
    out["sustained_p99_bound_ms"] = SERVE_P99_BOUND_MS
    for mode in ("serial", "batched"):
        ok = [float(k) for k, v in out["rates"].items()
              if v[mode]["views_per_s"] >= 0.97 * v[mode]["offered_rate"] and v[mode]["p99_ms"] <= SERVE_P99_BOUND_MS]
        out[f"max_sustained_rate_{mode}"] = max(ok) if ok else None
    log(f"highest rate sustained at p99 <= {SERVE_P99_BOUND_MS} ms: serial {out['max_sustained_rate_serial']}, "
        f"batched {out['max_sustained_rate_batched']}")
    return out


def serving_train_bench(n: int, rate: float, count: int, train_seconds: float):
    """Serving while training (resident n-Gaussian SH-3 room scene, Adam):
    mixed-resolution Poisson requests at `rate` served batched, with fwd+bwd
    training views of 1752x1168 at 180 deg (4 per step, random poses) in the
    gaps; beside it, the same trace served without training and training
    alone for `train_seconds`."""
    import numpy as np
    import torch

    from paper_2409_04751_amd import render as R
    from paper_2409_04751_amd import server as S
    from paper_2409_04751_amd import synth

    dev = torch.device("cuda", 0)
    scene = synth.room_scene(n, 5, 0.01, 3)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    *ordered, _ = R.spatially_ordered(*[f(a) for a in (scene.means, scene.scales, scene.quats, scene.opacity,
                                                       scene.sh)])
    leaves = [t.requires_grad_(True) for t in ordered]
    del ordered
    # one Adam per parameter tensor (Adam is elementwise, so this is the same
    # update as one optimizer over all of them), stepped one tensor per phase
    opts = [torch.optim.Adam([p], lr=1e-4) for p in leaves]
    cam = synth.fisheye_camera(1752, 1168, 180.0)
    poses = synth.random_poses(64, 7, tuple(x + 1.0 for x in synth.ROOM_LO), tuple(x - 1.0 for x in synth.ROOM_HI))
    targets = [f(synth.target_image(cam.width, cam.height, 100 + k)) for k in range(4)]
    ws = R.Workspace(dev)

    def train_view(k):  # two phases: forward and loss, then backward
        img = R.rasterize(*leaves, 3, poses[k % len(poses)], cam, (0.0, 0.0, 0.0), ws)
        loss = R.l1_loss(img, targets[k % 4])
        yield
        loss.backward()

    def optimizer_step():  # one phase per parameter tensor
        for o in opts:
            o.step()
            o.zero_grad(set_to_none=False)
            yield

    srv = S.RenderServer(*[x.detach() for x in leaves], 3, workspace_bytes=16 << 30)
    warm = S.poisson_trace(rate, 16, seed=98)
    srv.serve(warm, "batched")
    for k in range(4):
        S.run_phases(train_view(k))
    S.run_phases(optimizer_step())
    torch.cuda.synchronize()
    trace = S.poisson_trace(rate, count, seed=11)
    srv.batches = srv.splits = 0
    alone = srv.serve(trace, "batched")
    srv.batches = srv.splits = 0
    mixed = srv.serve_with_training(trace, train_view, optimizer_step, 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < train_seconds:
        for k in range(4):
            S.run_phases(train_view(k))
        S.run_phases(optimizer_step())
        torch.cuda.synchronize()
        steps += 1
    train_only = steps / (time.perf_counter() - t0)
    r = lambda d: {k: round(v, 3) if isinstance(v, float) else v for k, v in d.items()}
    log(f"serve+train: p99 {mixed['p99_ms']:.2f} ms (serve only {alone['p99_ms']:.2f}), "
        f"{mixed['train_steps_per_s']:.1f} train steps/s (train only {train_only:.1f})")
    return dict(scene=f"room {n} Gaussians, SH3, resident, Adam lr 1e-4", rate=rate, requests=count,
                train_view="1752x1168 fisheye 180 deg, 4 views per step", serve_only=r(alone), serve_and_train=r(mixed),
                train_only_steps_per_s=round(train_only, 3))


def _counts(ws, n, cam):
    """(V, K) of the forward left in a workspace (its counters)."""
    import numpy as np
    import torch

    lay = ws.layout(n, cam.width, cam.height)
    c = ws.view(lay.counters, 18, torch.int32).cpu().numpy().view(np.uint32).astype(np.int64)
    return int(c[1]), int(c[14] + (c[15] << 32))


def config_bench(label, scene, poses, cams, steps, warmup, train=True):
    """Times `steps` steps of one configuration after `warmup` untimed ones.
    A training step renders every view of `poses` through the multi-view
    autograd function, adds the views' L1 losses against seeded U(0, 1)
    targets and runs the backward; a forward-only step renders each view.
    Returns ms per step and per view, the workload's counts and its path
    roofline fraction (the byte model per view, summed over the views)."""
    import numpy as np
    import torch

    from paper_2409_04751_amd import render as R
    from paper_2409_04751_amd import synth

    dev = torch.device("cuda", 0)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    *ordered, _ = R.spatially_ordered(*[f(a) for a in (scene.means, scene.scales, scene.quats, scene.opacity,
                                                       scene.sh)])
    leaves = [t.requires_grad_(train) for t in ordered]
    del ordered
    deg = scene.sh_degree
    wss = [R.Workspace(dev) for _ in poses]
    targets = [f(synth.target_image(c.width, c.height, 1 + v)) for v, c in enumerate(cams)]
    one = torch.ones((), dtype=torch.float32, device=dev)

    def step():
        if train:
            imgs = R.rasterize_views(*leaves, deg, poses, cams, None, wss)
            loss = sum(R.l1_loss(img, t) for img, t in zip(imgs, targets))
            torch.autograd.grad(loss, leaves, grad_outputs=one)
        else:
            with torch.no_grad():
                for pose, cam, ws in zip(poses, cams, wss):
                    R.render_forward(*leaves, deg, pose, cam, (0.0, 0.0, 0.0), ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    N, S = scene.n, scene.sh.shape[0]
    total_bytes = 0.0
    views = []
    for ws, cam in zip(wss, cams):
        V, K = _counts(ws, N, cam)
        P = cam.width * cam.height
        total_bytes += path_bytes(N, V, K, P, S) if train else forward_bytes(N, V, K, P, S)
        views.append(dict(width=cam.width, height=cam.height, visible=V, intersections=K))
    gbs = total_bytes / (ms * 1e-3) / 1e9
    out = dict(ms_per_step=round(ms, 4), ms_per_view=round(ms / len(poses), 4), views_per_step=len(poses),
               gaussians=N, sh_degree=deg, views=views, steps=steps, warmup=warmup,
               step="fwd+bwd (multi-view autograd, L1)" if train else "forward only",
               path=dict(bytes_per_step=total_bytes, achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=round(gbs / HBM_PEAK_GBS, 4)))
    log(f"{label}: {ms:.3f} ms/step ({out['ms_per_view']:.3f} ms/view), path {gbs:.0f} GB/s")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=3_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-rates", type=float, nargs="+",
                    default=[50.0, 100.0, 200.0, 500.0, 1000.0, 1500.0, 2000.0],
                    help="Poisson arrival rates (requests/s) for the serving measurement")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per rate")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (1k 256^2 forward, 500k fwd+bwd, 3M 2048^2 four views)")
    ap.add_argument("--no-serve-train", action="store_true",
                    help="skip the measurement of serving while training a 6M-Gaussian scene")
    ap.add_argument("--serve-train-n", type=int, default=6_000_000)
    ap.add_argument("--serve-train-rate", type=float, default=200.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device once (rocprofv3 counter calibration) and exit")
    ap.add_argument("--source-sha", action="store_true", help="print the hash of the kernel sources and exit")
    args = ap.parse_args()
    if args.source_sha:
        print(source_sha())
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the fisheye rasterizer has no "
              "multi-GPU path in this build", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2409_04751_amd import _lib as L
    from paper_2409_04751_amd import render as R
    from paper_2409_04751_amd import synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        a = torch.ones(args.copy_calibration << 18, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB")
        return 0
    t = time.perf_counter()
    scene = synth.room_scene(args.n, 0, 0.01, 3)
    cam = synth.fisheye_camera(1752, 1168, 180.0)
    pose = synth.identity_pose()
    target_np = synth.target_image(cam.width, cam.height, 1)
    log(f"scene generated in {time.perf_counter() - t:.1f}s")
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    # the resident scene is stored in Morton order of its means (a permutation)
    *ordered, _ = R.spatially_ordered(*[f(a) for a in (scene.means, scene.scales, scene.quats, scene.opacity,
                                                       scene.sh)])
    leaves = [t.requires_grad_(True) for t in ordered]
    del ordered
    target = f(target_np)
    deg = scene.sh_degree
    ws = R.Workspace(dev)
    bg = (0.0, 0.0, 0.0)
    stats = {}

    one = torch.ones((), dtype=torch.float32, device=dev)  # dL/dL, made once

    def step():
        img = R.rasterize(*leaves, deg, pose, cam, bg, ws)
        loss = R.l1_loss(img, target)
        grads = torch.autograd.grad(loss, leaves, grad_outputs=one)
        return loss, grads

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms:.3f} ms/step")
    # the same K steps again with a HIP event pair around every library
    # kernel (on the stream it runs on): per-kernel times for the roofline
    prof = {}
    ms_profiled = None
    if not args.no_profile:
        L.fgs_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms_profiled = (time.perf_counter() - t0) * 1000.0 / args.steps
        prof = L.fgs_profile_read()
        L.fgs_profile_enable(False)
        log(f"profiled {args.steps} steps: {ms_profiled:.3f} ms/step")

    # counts of the workload (from the library's own state)
    _, ws2, K = R.render_forward(*[x.detach() for x in leaves], deg, pose, cam, bg)
    lay = ws2.layout(scene.n, cam.width, cam.height)
    tiles = ws2.view(lay.tiles, scene.n, torch.int32)
    V = int((tiles > 0).sum().item())
    cnt = ws2.view(lay.counters, 18, torch.int32).cpu().numpy().view(np.uint32).astype(np.int64)
    rows_binned = int(cnt[16] + (cnt[17] << 32))
    N, P, S = scene.n, cam.width * cam.height, scene.sh.shape[0]

    pairs = None
    staged = None
    if not args.no_profile:
        _, ws3, _ = R.render_forward(*[x.detach() for x in leaves], deg, pose, cam, bg, save_pixel_state=True)
        lay3 = ws3.layout(scene.n, cam.width, cam.height)
        pairs = contributing_pairs(ws3, lay3, scene.n, K)
        staged = staged_entries(ws3, lay3)
        del ws3
        log(f"blend backward pairs: tested {pairs[0]}, blended {pairs[1]}; entries staged per blend {staged}")

    kernels = {k: dict(launches=v[0] // args.steps if args.steps else 0, ms=v[1] / args.steps,
                       avg_ms=v[1] / max(v[0], 1)) for k, v in prof.items()}
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms"])
        d = kernels[dom]
        b = kernel_bytes(dom, N, V, K, P, S)
        if b is not None:
            ach = b / (d["avg_ms"] * 1e-3) / 1e9
            roofline = dict(kernel=dom, bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                            frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic_for(dom),
                            bytes_per_launch=b, avg_launch_ms=round(d["avg_ms"], 5))
        elif dom == "blend_backward" and pairs:
            fl = BLEND_BWD_FLOPS_TESTED * pairs[0] + BLEND_BWD_FLOPS_BLENDED * pairs[1]
            ach = fl / (d["avg_ms"] * 1e-3) / 1e12
            roofline = dict(kernel=dom, bound="alu", achieved=round(ach, 2), peak=FP32_VALU_PEAK_TFLOPS,
                            unit="TFLOP/s", frac=round(ach / FP32_VALU_PEAK_TFLOPS, 4), traffic=traffic_for(dom),
                            flops_per_launch=fl, pairs_tested=pairs[0], pairs_blended=pairs[1],
                            avg_launch_ms=round(d["avg_ms"], 5))
        else:
            roofline = dict(kernel=dom, bound="alu", achieved=None, peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                            frac=None, traffic=traffic_for(dom), avg_launch_ms=round(d["avg_ms"], 5))
        pb = path_bytes(N, V, K, P, S)
        roofline["path"] = dict(bytes_per_view=pb, achieved=round(pb / (ms * 1e-3) / 1e9, 1), peak=HBM_PEAK_GBS,
                                unit="GB/s", frac=round(pb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
        if staged is not None:
            ps = path_bytes_staged(N, V, K, P, S, staged)
            roofline["path_staged"] = dict(
                bytes_per_view=ps, entries_staged=staged, achieved=round(ps / (ms * 1e-3) / 1e9, 1),
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                note="blends counted for the entries they stage (up to each tile's last blended entry), not all K")
        for k, v in kernels.items():
            bb = kernel_bytes(k, N, V, K, P, S)
            if bb is not None:
                v["GBs"] = round(bb * v["launches"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None
            v["ms"] = round(v["ms"], 5)
            v["avg_ms"] = round(v["avg_ms"], 5)

    del ws2
    configs = None
    if not args.no_configs:
        ws = None
        torch.cuda.empty_cache()
        configs = {}
        s1, cam1, poses1 = synth.workload("shell1k")
        configs["c1_shell1k_256x256_180deg_forward"] = config_bench("1k 256^2 forward", s1(), poses1, [cam1],
                                                                    args.steps, args.warmup, train=False)
        s2, cam2, poses2 = synth.workload("room500k")
        configs["c2_room500k_1752x1168_180deg_fwdbwd"] = config_bench("500k 1752x1168 fwd+bwd", s2(), poses2, [cam2],
                                                                      args.steps, args.warmup)
        _, cam3, poses3 = synth.workload("room3m_2k")
        configs["c3_room3m_2048x2048_200deg_4views_fwdbwd"] = config_bench(
            "3M 2048^2 200deg 4 views fwd+bwd", scene, poses3, [cam3] * len(poses3), max(5, args.steps // 4),
            min(args.warmup, 3))
        torch.cuda.empty_cache()

    serving = None
    if not args.no_serve:
        serving = serving_bench([x.detach() for x in leaves], deg, args.serve_rates, args.serve_requests)

    serve_train = None
    if not args.no_serve and not args.no_serve_train:
        serve_train = serving_train_bench(args.serve_train_n, args.serve_train_rate, args.serve_requests, 3.0)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        s2, cam2, poses2 = synth.workload("room500k")
        small = (s2(), poses2[0], cam2, synth.target_image(cam2.width, cam2.height, 1))
        cpu = cpu_baseline(scene, pose, cam, target_np, small)
        log(f"oracle: {cpu['value']:.0f} ms/view on {cpu['cores']} threads (runs {cpu['runs_ms']}), "
            f"500k view on 1 thread {cpu['single_thread']['value']:.0f} ms, {cpu['cpu_model']}")

    out = dict(metric=METRIC, value=round(ms, 4), unit="ms/view", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=round(ms, 4), higher_is_better=False, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload="room3m_fisheye1752x1168_180deg", scene_order="morton (fgs_spatial_order)",
                           gaussians=N, sh_degree=3, width=cam.width,
                           height=cam.height, fov_deg=180.0, views_per_step=1, visible=V, intersections=K,
                           rows_binned=rows_binned,
                           geometry_dtype="f64"),
               roofline=roofline, cpu_baseline=cpu, kernels=kernels,
               ms_per_step_event_profiled=round(ms_profiled, 4) if ms_profiled else None, configs=configs,
               serving=serving, serving_with_training=serve_train)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
