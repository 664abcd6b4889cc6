"""Shared helpers of the GPU parity tests: run a scene through the C-ABI
library and through the oracle from the same seeded float32 inputs."""
import sys

import numpy as np


def note(msg):
    """Names the GPU case before it runs (flushed, so a crash still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_context(mq, scene, capacity=None, track_ids=True):
    import torch
    x, v, C, F = scene["state"]
    n = x.shape[1]
    ctx = mq.Context(scene["scheme"], scene["params"], capacity or max(n, 1), track_ids=track_ids)
    dev = ctx.device
    ctx.encode(*(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (x, v, C, F)))
    return ctx


def gpu_decode_np(ctx):
    return tuple(t.cpu().numpy().astype(np.float64) for t in ctx.decode())


def oracle_sim(orc, scene):
    x, v, C, F = scene["state"]
    words, st = orc.encode(scene["scheme"], x, v, C, F, 0, 2)
    return orc.Sim(scene["scheme"], scene["params"], words), words, st


def by_id(arr, ids):
    """Reorders the particle axis so that column i holds original particle i."""
    out = np.empty_like(arr)
    out[..., ids] = arr
    return out
