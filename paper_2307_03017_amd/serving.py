"""Continuous-batching serving of HSGD refinements over the library's batch core.

A workload of persistent streams (scenes); each request is one frame of a stream: the
stream's views (its targets) and an initial MPI at the coarsest level, refined coarse to
fine in BF16 storage. Requests arrive open-loop (Poisson). The loop admits queued
requests first-come first-served whenever the core has a free slot and HBM budget,
evicting idle streams (least recently used) when a new stream does not fit, runs one
batched iteration (hsgd_batch_step: every request in flight advances one level-iteration,
all in one captured HIP graph) and collects completions. Latency is arrival (host clock)
to the completion of the request's last iteration on the device (its step event, mapped
onto the host clock through the batch's reference event).

The mix: 8 scenes, three at 256x192 with 16 planes (k = 2), three at 512x384 with 32
planes (k = 4), two at 1008x756 with 32 planes (k = 4), 3 to 5 views each (focal length
0.78125 W, translations within +-0.1), 3 levels with one iteration each.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import hsgd, scenes

MIX = [("s256", 100), ("s256", 101), ("s256", 102), ("s512", 103), ("s512", 104), ("s512", 105),
       ("s1008", 106), ("s1008", 107)]


@dataclass
class SceneInputs:
    name: str
    sc: scenes.Scene
    targets: torch.Tensor                    # [N][H][W][3] FP32 (device)
    inits: list                              # per frame variant: [D][h0][w0][4] (device, storage dtype)
    inits32: list                            # the same initial MPIs in FP32 (device)


def make_mix(mix_seed: int = 7, variants: int = 4, device="cuda", dtype=torch.bfloat16, mix=None):
    """Scenes of the serving mix with their targets (rendered from the ground truth by the
    library) and a few initial-MPI variants per scene (the per-frame stand-in for the
    initial MPI network: the scene's ground truth at the coarsest level with fresh noise)."""
    rng = np.random.default_rng(mix_seed)
    mix = MIX if mix is None else mix
    out = []
    for cfg, seed, *over in mix:                # (name, seed[, scene overrides])
        N = int(rng.integers(3, 6))
        sc = scenes.make_scene(cfg, seed=seed, N=N, **(over[0] if over else {}))
        table = hsgd.level_warps(sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths,
                                 sc.W, sc.H, sc.W, sc.H, device)
        gt = torch.from_numpy(sc.gt_mpi(np.float32)).to(device)
        targets, _ = hsgd.hsgd_render(gt, table, sc.N)
        del gt
        w0, h0 = sc.shapes()[0]
        inits, inits32 = [], []
        for v in range(variants):
            m32 = torch.from_numpy(sc.noisy_mpi(w0, h0, seed=1000 * seed + v)).to(device)
            inits32.append(m32)
            inits.append(m32 if dtype == torch.float32 else hsgd.hsgd_convert(m32, dtype))
        out.append(SceneInputs(cfg, sc, targets, inits, inits32))
    return out


def new_stream(i: int, si: SceneInputs, dtype=torch.bfloat16, device="cuda") -> hsgd.ServingStream:
    sc = si.sc
    st = hsgd.ServingStream(i, sc.K_ref(), sc.K_views(), sc.R_views(), sc.t_views(), sc.depths,
                            sc.W, sc.H, sc.iters, sc.k, dtype=dtype, device=device)
    st.images[-1].copy_(si.targets)
    return st


@dataclass
class Served:
    scene: int
    variant: int
    arrival: float
    ticket: int = -1
    admitted: float = 0.0
    done: float = -1.0                       # host seconds
    loss: list = field(default_factory=list)


class Server:
    """The request loop around one hsgd.Batch."""

    def __init__(self, inputs, max_slots: int = 8, hbm_budget: int = 64 << 30, dtype=torch.bfloat16,
                 device="cuda", snapshot=None, batch=None, make_stream=None):
        self.inputs = inputs
        self.dtype = dtype
        self.device = device
        if batch is None:
            D = max(si.sc.D for si in inputs)
            N = max(si.sc.N for si in inputs)
            H = max(si.sc.H for si in inputs)
            W = max(si.sc.W for si in inputs)
            k = max(si.sc.k for si in inputs)
            batch = hsgd.Batch(max_slots, D, N, H, W, k, dtype=dtype, hbm_budget=hbm_budget, device=device)
        self.batch = batch
        self.make_stream = make_stream or (lambda i, si: new_stream(i, si, self.dtype, self.device))
        self.streams = {}                    # scene index -> ServingStream (resident buffers)
        self.last_used = {}
        self.snapshot = snapshot             # callable(request, stream) after a request's last step
        self.inflight = {}                   # ticket -> Served
        self.stream_busy = set()

    def _stream(self, i: int) -> hsgd.ServingStream:
        if i not in self.streams:
            self.streams[i] = self.make_stream(i, self.inputs[i])
        return self.streams[i]

    def try_admit(self, req: Served, now: float) -> bool:
        if req.scene in self.stream_busy:
            return False
        st = self._stream(req.scene)
        t = self.batch.admit(st)
        while t is None and self.batch.last_refusal == hsgd.HSGD_E_BUDGET:
            idle = [s for s in sorted(self.last_used, key=self.last_used.get)
                    if s != req.scene and s not in self.stream_busy and s in self.streams]
            if not idle:
                return False
            victim = idle[0]
            self.batch.release_stream(victim)
            del self.streams[victim]
            del self.last_used[victim]
            t = self.batch.admit(st)
        if t is None:
            return False
        # the frame's input: its initial MPI into the stream's coarsest level, enqueued after
        # every step so far and before the step that starts the frame
        st.levels[0].copy_(self.inputs[req.scene].inits[req.variant])
        req.ticket, req.admitted = t, now
        self.inflight[t] = req
        self.stream_busy.add(req.scene)
        self.last_used[req.scene] = now
        return True

    def step(self):
        n, finished = self.batch.step()
        for t in finished:
            req = self.inflight[t]
            self.stream_busy.discard(req.scene)
            if self.snapshot is not None:
                self.snapshot(req, self.streams[req.scene])
        return n

    def collect(self, origin: float):
        """Requests completed on the device; their done time is origin + milliseconds after
        the batch's reference event (seconds)."""
        done = []
        for t, req in list(self.inflight.items()):
            ok, ms = self.batch.poll(t)
            if ok:
                req.done = origin + ms * 1e-3
                done.append(req)
                del self.inflight[t]
        return done


def poisson_requests(n: int, rate: float, n_scenes: int, variants: int, seed: int = 7):
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1.0 / rate, size=n)
    scene = rng.integers(0, n_scenes, size=n)
    var = rng.integers(0, variants, size=n)
    t = np.cumsum(gaps)
    return [Served(int(s), int(v), float(a)) for s, v, a in zip(scene, var, t)]


def run(server: Server, reqs, warmup: int = 0, progress=None, clock=time.perf_counter, sleep=time.sleep):
    """Open-loop run: requests become visible at their arrival times (seconds after the
    start). Returns the completed requests in completion order."""
    if torch.cuda.is_available():
        torch.cuda.synchronize()
    server.batch.reference()
    t0 = clock()
    pending = list(reqs)
    queue = []
    done = []
    nxt = 0
    last_print = t0
    while len(done) < len(reqs):
        now = clock() - t0
        while nxt < len(pending) and pending[nxt].arrival <= now:
            queue.append(pending[nxt])
            nxt += 1
        # FIFO admission, skipping requests whose stream has a frame in flight
        kept = []
        for r in queue:
            if not server.try_admit(r, now):
                kept.append(r)
        queue = kept
        active = server.step()
        done += server.collect(0.0)           # completion times on the same origin as arrivals
        if progress and clock() - last_print > 5.0:
            last_print = clock()
            progress(f"serving: {len(done)}/{len(reqs)} done, {len(queue)} queued")
        if active == 0 and server.inflight:
            sleep(0.0002)                     # every admitted step is enqueued: wait for events
        elif active == 0:
            if nxt < len(pending):
                wait = pending[nxt].arrival - (clock() - t0)
                if wait > 0:
                    sleep(min(wait, 0.002))
            elif queue:
                sleep(0.0005)
    if torch.cuda.is_available():
        torch.cuda.synchronize()
    return done


def summary(done, warmup: int, inputs):
    meas = sorted(done, key=lambda r: r.arrival)[warmup:]
    lat = np.array([(r.done - r.arrival) * 1e3 for r in meas])
    span = max(r.done for r in meas) - min(r.arrival for r in meas)
    dense = sum(sum(n * inputs[r.scene].sc.D * w * h
                    for (w, h), n in zip(inputs[r.scene].sc.shapes(), inputs[r.scene].sc.iters)) for r in meas)
    return {
        "requests": len(meas),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "frames_per_s": len(meas) / span,
        "voxel_updates_per_s": dense / span,
    }
