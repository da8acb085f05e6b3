"""Batched render server over a resident scene.

The scene's parameters stay in HBM.  Requests (a pose and a fisheye camera of
any resolution and field of view) queue in arrival order; the server takes
as many as fit into one batch (at most FGS_MAX_BATCH views and a workspace
byte budget, estimated from the intersections per pixel seen so far for that
field of view) and renders them with one fgs_render_forward_batch call: one
preprocess launch reads every Gaussian once for the whole batch, one tile
sort and one blend launch cover all views.  If the estimate was low and the
batch does not fit, it is split and the rest deferred.

`serve()` replays an open-loop arrival trace on the wall clock and reports
per-request latency (completion - arrival), p50 / p99 and views/s, for the
batched server or for serial one-request-at-a-time rendering.
`serve_with_training()` does the same while training the resident scene in
the gaps: whenever no request is queued, one training view (forward +
backward) runs, and every few views an optimizer step ends a training step;
it reports the served latency together with training steps/s.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np
import torch

from . import _lib as L
from . import render as R
from . import synth


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds from the start of the trace
    pose: object
    cam: object
    bg: tuple = (0.0, 0.0, 0.0)


def poisson_trace(rate: float, count: int, seed: int = 3, resolutions=((512, 512), (1024, 1024), (1752, 1168),
                                                                       (2048, 2048)),
                  fov_range=(150.0, 200.0)) -> list[Request]:
    """Open-loop Poisson arrivals; each request a random pose inside the room
    (shrunk by 1 m), a resolution drawn uniformly from `resolutions` and an
    equidistant fisheye with FOV ~ U(fov_range)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(synth.ROOM_LO) + 1.0
    hi = np.asarray(synth.ROOM_HI) - 1.0
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        pos = lo + (hi - lo) * rng.random(3)
        Rm = synth._haar_rotation(rng).astype(np.float32)
        pose = synth.Pose(Rm, (-(Rm.astype(np.float64) @ pos)).astype(np.float32))
        w, h = resolutions[int(rng.integers(len(resolutions)))]
        fov = float(rng.uniform(*fov_range))
        out.append(Request(k, t, pose, synth.fisheye_camera(w, h, fov)))
    return out


def _phases(result):
    """The phases of a training callable's result, one per next(), each
    yielding whether it finished the callable's work: a generator runs up to
    each of its yields and then to its end; anything else has already run
    when the callable returned."""
    if hasattr(result, "__next__"):
        while True:
            try:
                next(result)
            except StopIteration:
                break
            yield False
    yield True


def run_phases(result) -> None:
    """Runs every phase of a training callable's result."""
    for _ in _phases(result):
        pass


class RenderServer:
    def __init__(self, means, scales, quats, opacities, sh, sh_degree: int, max_batch: int = L.FGS_MAX_BATCH,
                 workspace_bytes: int = 12 << 30, kpp_prior: float = 8.0):
        self.params = (means, scales, quats, opacities, sh)
        self.sh_degree = sh_degree
        self.g = R.gaussians_struct(means, scales, quats, opacities, sh, sh_degree)
        self.n = self.g.n
        self.max_batch = max(1, min(max_batch, L.FGS_MAX_BATCH))
        self.device = means.device
        self.ws = R.Workspace(self.device)
        self.ws.ensure(workspace_bytes)
        self.single_ws = R.Workspace(self.device)
        # intersections per pixel, by FOV in 10-degree buckets (EMA)
        self.kpp = collections.defaultdict(lambda: kpp_prior)
        self.k_seen: dict[int, int] = {}
        self.batches = 0
        self.splits = 0

    # -- estimates -----------------------------------------------------------
    def _bucket(self, cam) -> int:
        return int(math.degrees(cam.width / cam.fx) // 10)

    def _k_est(self, cam) -> int:
        return int(self.kpp[self._bucket(cam)] * cam.width * cam.height * 1.3) + 4096

    def _observe(self, cam, k: int) -> None:
        b = self._bucket(cam)
        self.kpp[b] = 0.7 * self.kpp[b] + 0.3 * (k / (cam.width * cam.height))

    def _bytes(self, cams, k_total: int) -> int:
        return L.fgs_batch_workspace_bytes(self.n, [R.camera_struct(c) for c in cams], k_total)

    # -- admission -----------------------------------------------------------
    def admit(self, pending: collections.deque) -> list[Request]:
        """Oldest first, while the batch's estimated workspace fits."""
        batch: list[Request] = []
        k = 0
        while pending and len(batch) < self.max_batch:
            r = pending[0]
            k2 = k + self._k_est(r.cam)
            if batch and self._bytes([x.cam for x in batch] + [r.cam], k2) > self.ws.nbytes:
                break
            batch.append(pending.popleft())
            k = k2
        return batch

    # -- rendering -----------------------------------------------------------
    def render_batch(self, batch: list[Request]) -> tuple[list[torch.Tensor], list[Request]]:
        """Renders as much of `batch` as fits; returns (images, deferred)."""
        outs = [torch.empty((3, r.cam.height, r.cam.width), dtype=torch.float32, device=self.device) for r in batch]
        rc, kv, kt = L.fgs_render_forward_batch(self.g, [R.pose_struct(r.pose) for r in batch],
                                                [R.camera_struct(r.cam) for r in batch], [r.bg for r in batch],
                                                self.ws.ptr, self.ws.nbytes, [o.data_ptr() for o in outs],
                                                R._stream_handle(self.device))
        if rc == L.FGS_ERR_WORKSPACE and kt >= 0:
            for r, k in zip(batch, kv):
                self._observe(r.cam, k)
            if len(batch) == 1:
                raise L.FgsError(rc, "one view does not fit the server workspace: " + L.fgs_last_error())
            self.splits += 1
            half = len(batch) // 2
            imgs, deferred = self.render_batch(batch[:half])
            return imgs, deferred + batch[half:]
        L.check(rc)
        for r, k in zip(batch, kv):
            self._observe(r.cam, k)
            self.k_seen[r.rid] = k
        self.batches += 1
        return outs, []

    def render_one(self, r: Request) -> torch.Tensor:
        img, self.single_ws, k = R.render_forward(*self.params, self.sh_degree, r.pose, r.cam, r.bg,
                                                  workspace=self.single_ws)
        self.k_seen[r.rid] = k
        return img

    # -- open-loop replay ----------------------------------------------------
    def serve_with_training(self, trace: list[Request], train_view, optimizer_step, views_per_step: int = 4) -> dict:
        """Batched serving of `trace` with training in the gaps.  Requests
        have priority: whenever the queue is empty, one phase of training
        work runs, and the queue is checked again.  `train_view(k)` runs the
        k-th training view (forward + backward); after every `views_per_step`
        views `optimizer_step()` updates the parameters in place (the server
        renders the same tensors, so requests see the scene as trained so
        far).  Either may be a generator function, whose yields split its
        work into phases (say the forward, then the backward; or one
        parameter tensor's update at a time): a request then waits for at
        most one phase rather than a whole view or step."""
        pending: collections.deque = collections.deque()
        lat = np.zeros(len(trace))
        nxt = done = 0
        count = dict(views=0, steps=0)
        stream = torch.cuda.current_stream(self.device)

        def training():  # one training phase per next()
            while True:
                for last in _phases(train_view(count["views"])):
                    count["views"] += last
                    yield
                if count["views"] % views_per_step == 0:
                    for last in _phases(optimizer_step()):
                        count["steps"] += last
                        yield

        work = training()
        t0 = time.perf_counter()
        while done < len(trace):
            now = time.perf_counter() - t0
            while nxt < len(trace) and trace[nxt].arrival <= now:
                pending.append(trace[nxt])
                nxt += 1
            if not pending:
                next(work)
                stream.synchronize()
                continue
            batch = self.admit(pending)
            imgs, deferred = self.render_batch(batch)
            for r in reversed(deferred):
                pending.appendleft(r)
            batch = batch[:len(imgs)]
            stream.synchronize()
            t_done = time.perf_counter() - t0
            for r in batch:
                lat[r.rid] = t_done - r.arrival
            done += len(batch)
        span = time.perf_counter() - t0
        views, steps = count["views"], count["steps"]
        return dict(mode="batched+training", requests=len(trace), p50_ms=float(np.percentile(lat, 50) * 1e3),
                    p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                    views_per_s=len(trace) / span, span_s=span, offered_rate=len(trace) / trace[-1].arrival,
                    train_views=views, train_steps=steps, train_steps_per_s=steps / span, batches=self.batches,
                    splits=self.splits)

    def serve(self, trace: list[Request], mode: str = "batched", keep_images: bool = False) -> dict:
        assert mode in ("batched", "serial")
        pending: collections.deque = collections.deque()
        lat = np.zeros(len(trace))
        images = {} if keep_images else None
        nxt = 0
        done = 0
        stream = torch.cuda.current_stream(self.device)
        t0 = time.perf_counter()
        while done < len(trace):
            now = time.perf_counter() - t0
            while nxt < len(trace) and trace[nxt].arrival <= now:
                pending.append(trace[nxt])
                nxt += 1
            if not pending:
                wait = trace[nxt].arrival - now
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
                continue
            if mode == "serial":
                batch = [pending.popleft()]
                imgs = [self.render_one(batch[0])]
            else:
                batch = self.admit(pending)
                imgs, deferred = self.render_batch(batch)
                for r in reversed(deferred):
                    pending.appendleft(r)
                batch = batch[:len(imgs)]
            stream.synchronize()
            t_done = time.perf_counter() - t0
            for r, img in zip(batch, imgs):
                lat[r.rid] = t_done - r.arrival
                if images is not None:
                    images[r.rid] = img
            done += len(batch)
        span = time.perf_counter() - t0
        out = dict(mode=mode, requests=len(trace), p50_ms=float(np.percentile(lat, 50) * 1e3),
                   p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                   views_per_s=len(trace) / span, span_s=span, offered_rate=len(trace) / trace[-1].arrival)
        if mode == "batched":
            out.update(batches=self.batches, splits=self.splits)
        if images is not None:
            out["images"] = images
        return out
