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


def _bits(words, off, nbits):
    """Bits [off, off + nbits) of every record (words: uint32 [W, n])."""
    w = np.asarray(words).astype(np.uint64)
    lo = w[off // 32]
    hi = w[off // 32 + 1] if off // 32 + 1 < w.shape[0] else np.zeros_like(lo)
    return (((lo | (hi << np.uint64(32))) >> np.uint64(off % 32)) & np.uint64((1 << nbits) - 1)).astype(np.int64)


def field_steps_per_particle(orc, scheme, words):
    """Quantization step of each particle's stored value, per field (slot
    order x, v, C, F/J): Delta for a fixed-point field, 2^(E - m + 1) from the
    stored exponent for a shared-exponent field, the float32 spacing at the
    stored value for a raw field (None: taken from the values)."""
    import math
    _, fo, _, _ = orc.layout(scheme)
    names = ["x", "v", "C", "J" if any(f["field"] == "J" for f in scheme["fields"]) else "F"]
    out = {}
    for f in scheme["fields"]:
        slot = names.index(f["field"])
        if f["kind"] == "fixed":
            out[f["field"]] = np.full(words.shape[1], (f["hi"] - f["lo"]) * 2.0 ** -f["bits"])
        elif f["kind"] == "shared_exp":
            emax = math.ceil(math.log2(f["hi"]))
            emin = emax - (2 ** f["exp_bits"] - 1)
            e = _bits(words, int(fo[slot]), f["exp_bits"]) + emin
            out[f["field"]] = np.ldexp(1.0, (e - (f["bits"] - 1)).astype(np.int32))
        else:
            out[f["field"]] = None
    return out


def lsb_differences(orc, scheme, gw, gids, ow, oids):
    """Decoded GPU and oracle states (ordered by original particle) and, per
    field, |gpu - oracle| in units of the larger of the two quantization
    steps of each particle's stored value.  Returns (x difference in domain
    units [dim, n], {field: LSB differences [ncomp, n]})."""
    g = [by_id(a, gids) for a in orc.decode(scheme, gw)]
    o = [by_id(a, oids) for a in orc.decode(scheme, ow)]
    sg = field_steps_per_particle(orc, scheme, gw)
    so = field_steps_per_particle(orc, scheme, ow)
    names = ["x", "v", "C", "J" if any(f["field"] == "J" for f in scheme["fields"]) else "F"]
    lsb = {}
    for i, f in enumerate(names):
        if sg[f] is None:
            step = np.maximum(np.spacing(np.abs(o[i]).astype(np.float32)).astype(np.float64), 2.0 ** -149)
        else:
            step = np.maximum(by_id(sg[f], gids), by_id(so[f], oids))[None, :]
        lsb[f] = np.abs(g[i] - o[i]) / step
    return np.abs(g[0] - o[0]), lsb
