"""Serving loop: many independent quantized MLS-MPM scenes on one GPU.

Scenes arrive over time (a Poisson stream in the benchmark).  The server
admits a scene when its device memory (packed state, two grid buffers,
scratch, ids, encode staging; sizes from mpmq_query_sizes) fits in the HBM
budget, creates a context for it on one of a pool of HIP streams, encodes its
initial state, and then advances every active scene by `steps_per_tick`
substeps per tick until it has run its steps; a finished scene releases its
memory.  Every scene keeps its own packed state resident on the device, its
own Philox key (scheme seed) and slot numbering, so its result does not
depend on which other scenes share the GPU.

Two ways to issue the substeps of a tick:
  - batched (default): scenes are spread over a few streams at admission,
    and the scenes of one stream, dimension and material advance together
    through mpmq_step_batch, one grid-update launch and one fused-substep
    launch per substep for the whole set (continuous batching: a scene
    admitted between ticks joins the next tick's batch of its stream, a
    finished one leaves it; the streams let one batch's tail overlap
    another's work and admissions run beside the batches);
  - per scene (batched=False): one context per scene on a pool of streams,
    each with its own launches.
Either way a scene computes the same words bit for bit.

Latency of a scene = time from its submission (its arrival) to the GPU
completing its last substep, measured with HIP events on its stream against
an event recorded when the server starts.

Host logic only; all simulation work runs in libmpmq.so through Context.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from . import Context, mpmq_query_sizes, step_batch


def scene_bytes(scene: dict) -> int:
    """Device bytes one scene holds while active."""
    sz = mpmq_query_sizes(scene["scheme"], scene["params"], scene["n"])
    dim = scene["params"]["dim"]
    staging = 4 * scene["n"] * (2 * dim + 2 * dim * dim)  # float32 x, v, C, F for the encode
    return sz["packed_bytes"] + 2 * sz["grid_bytes"] + sz["scratch_bytes"] + sz["ids_bytes"] + staging


@dataclass
class _Active:
    scene: dict
    ctx: Context
    stream: object
    nbytes: int
    submitted: float
    done_steps: int = 0
    last_event: object = None
    start_event: object = None
    inflight: object = field(default_factory=collections.deque)


@dataclass
class ServeResult:
    latencies_s: dict = field(default_factory=dict)      # scene name -> seconds
    queue_wait_s: dict = field(default_factory=dict)     # scene name -> seconds before admission
    particle_substeps: int = 0
    makespan_s: float = 0.0
    peak_bytes: int = 0
    max_active: int = 0
    words: dict = field(default_factory=dict)            # scene name -> final packed words (if kept)

    def percentile(self, q):
        import numpy as np
        v = list(self.latencies_s.values())
        return float(np.percentile(v, q)) if v else 0.0

    def throughput(self):
        return self.particle_substeps / self.makespan_s if self.makespan_s > 0 else 0.0


class Server:
    """Admits scenes under an HBM budget and steps them in ticks."""

    def __init__(self, hbm_budget_bytes=200e9, streams=4, steps_per_tick=10, keep_words=False, device=None,
                 batched=True):
        import torch
        self.budget = float(hbm_budget_bytes)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.batched = bool(batched)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(int(streams))]
        self.steps_per_tick = int(steps_per_tick)
        self.keep_words = keep_words
        self._next_stream = 0

    def _admit(self, scene, submitted, used):
        import torch
        st = self.streams[self._next_stream % len(self.streams)]
        self._next_stream += 1
        nbytes = scene_bytes(scene)
        with torch.cuda.stream(st):
            ctx = Context(scene["scheme"], scene["params"], scene["n"], stream=st, device=self.device)
            dim = scene["params"]["dim"]
            n = scene["n"]
            if scene.get("state") is not None:
                x, v, C, F = (torch.from_numpy(a).to(self.device, non_blocking=False) for a in scene["state"])
            else:
                x = torch.from_numpy(scene["x"]).to(self.device)
                v = torch.from_numpy(scene["vel"]).to(self.device)[:, None].expand(dim, n).contiguous()
                C = torch.zeros((dim * dim, n), dtype=torch.float32, device=self.device)
                F = torch.zeros((dim * dim, n), dtype=torch.float32, device=self.device)
                for a in range(dim):
                    F[a * dim + a].fill_(1.0)
            ctx.encode(x, v, C, F)
        return _Active(scene, ctx, st, nbytes, submitted)

    def run(self, scenes, arrivals=None):
        """scenes: list of scene dicts (workloads.c4_scene); arrivals: seconds
        after start at which each scene is submitted (None: all at 0)."""
        import torch
        arrivals = list(arrivals) if arrivals is not None else [0.0] * len(scenes)
        order = sorted(range(len(scenes)), key=lambda i: arrivals[i])
        pending = collections.deque(order)
        waiting = collections.deque()          # submitted, not yet admitted
        active = []
        res = ServeResult()
        used = 0
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev0.record(torch.cuda.current_stream(self.device))
        finished = []
        while pending or waiting or active:
            now = time.perf_counter() - t0
            while pending and arrivals[pending[0]] <= now:
                i = pending.popleft()
                waiting.append((i, arrivals[i]))
            # admission in arrival order under the memory budget
            while waiting:
                i, sub = waiting[0]
                need = scene_bytes(scenes[i])
                if used + need > self.budget and active:
                    break
                waiting.popleft()
                a = self._admit(scenes[i], sub, used)
                a.start_event = torch.cuda.Event(enable_timing=True)
                a.start_event.record(a.stream)
                res.queue_wait_s[scenes[i]["name"]] = max(0.0, (time.perf_counter() - t0) - sub)
                used += a.nbytes
                active.append(a)
            res.peak_bytes = max(res.peak_bytes, used)
            res.max_active = max(res.max_active, len(active))
            # one tick: every active scene with fewer than two ticks in flight
            # gets `steps_per_tick` more substeps
            progressed = False
            due = []
            for a in active:
                while a.inflight and a.inflight[0].query():
                    a.inflight.popleft()
                if a.done_steps >= a.scene["steps"] or len(a.inflight) >= 2:
                    continue
                due.append(a)
            if self.batched:
                # scenes of one dimension, material and substep count go out together
                groups = collections.defaultdict(list)
                for a in due:
                    k = min(self.steps_per_tick, a.scene["steps"] - a.done_steps)
                    groups[(id(a.stream), a.ctx.dim, a.ctx.f3, k)].append(a)
                for (_, _, _, k), grp in groups.items():
                    step_batch([a.ctx for a in grp], k)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(grp[0].stream)
                    for a in grp:
                        a.done_steps += k
                        a.last_event = ev
                        a.inflight.append(ev)
                    progressed = True
            else:
                for a in due:
                    k = min(self.steps_per_tick, a.scene["steps"] - a.done_steps)
                    a.ctx.step(k)
                    a.done_steps += k
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(a.stream)
                    a.last_event = ev
                    a.inflight.append(ev)
                    progressed = True
            # retire finished scenes
            still = []
            for a in active:
                if a.done_steps >= a.scene["steps"] and a.last_event.query():
                    name = a.scene["name"]
                    done_ms = ev0.elapsed_time(a.last_event)
                    res.latencies_s[name] = done_ms / 1e3 - a.submitted
                    res.particle_substeps += a.scene["n"] * a.scene["steps"]
                    if self.keep_words:
                        res.words[name] = a.ctx.words()
                    finished.append(done_ms / 1e3)
                    a.ctx.close()
                    used -= a.nbytes
                else:
                    still.append(a)
            active = still
            if not progressed and not waiting:
                if active:
                    time.sleep(0.0002)
                elif pending:
                    time.sleep(max(0.0, min(0.01, arrivals[pending[0]] - (time.perf_counter() - t0))))
        torch.cuda.synchronize(self.device)
        res.makespan_s = max(finished) if finished else 0.0
        return res
