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


def comparison_units(params, dim, v_step, v_max, steps=1):
    """Per-field units (absolute, per particle) in which GPU and oracle
    states are compared, beyond each stored value's own quantization step.

    A store whose unquantized value lies within FP32 error of a rounding
    boundary may round the other way on the GPU: one code of v.  Such a flip
    changes the node velocities around the particle by up to one v step
    Delta_v, and C' = (4 / dx^2) sum_i w_i v_i (x_i - x_p)^T of every particle
    that gathers from those nodes by up to (4 / dx) Delta_v (the weights sum
    to 1 and |x_i - x_p| <= 1.5 dx); F' = (I + dt C') F then moves by dt |F|
    times that (J' = J (1 + dt tr C') by dt d |J| times it).  C is the
    most sensitive field: at the c1 scheme on a 128^3 grid one code of v is
    about 200 codes of C.  Besides, the GPU's own FP32 arithmetic bounds the
    noise of v' and of the first moments S_b by (3 + 27) 2^-24 * 2 v_max <=
    2^-18 v_max (float32 quotients of exact fixed-point node sums, 27-term
    float32 sums whose terms add up to at most 2 v_max); C' of a uniformly
    moving particle is that noise on the GPU and ~1e-13 in the oracle.
    F (and J) integrate C' over the substeps: differences of C' of either
    sign accumulate like a random walk, so their unit after `steps`
    substeps is sqrt(steps) times that of one substep.
    Returns {field: unit}, each broadcastable against [ncomp, n]."""
    inv_dx = float(params["grid_res"])
    noise_v = 2.0 ** -18 * v_max
    u_c = 4.0 * inv_dx * np.maximum(v_step, noise_v)
    walk = float(np.sqrt(max(steps, 1)))
    return {"x": 0.0, "v": noise_v, "C": u_c, "F": params["dt"] * u_c * 2.0 * walk,
            "J": params["dt"] * dim * u_c * 2.0 * walk}


def lsb_differences(orc, scheme, gw, gids, ow, oids, params=None, steps=1):
    """Decoded GPU and oracle states (ordered by original particle) and, per
    field, |gpu - oracle| in units of the larger of the two quantization
    steps of each particle's stored value, or of the unit that
    comparison_units derives (when params are given, for a comparison after
    `steps` substeps) if that is larger.  Returns (x difference in domain
    units [dim, n], {field: unit differences [ncomp, n]})."""
    g = [by_id(a, gids) for a in orc.decode(scheme, gw)]
    o = [by_id(a, oids) for a in orc.decode(scheme, ow)]
    sg = field_steps_per_particle(orc, scheme, gw)
    so = field_steps_per_particle(orc, scheme, ow)
    names = ["x", "v", "C", "J" if any(f["field"] == "J" for f in scheme["fields"]) else "F"]
    unit = {}
    for i, f in enumerate(names):
        if sg[f] is None:
            unit[f] = np.maximum(np.spacing(np.abs(o[i]).astype(np.float32)).astype(np.float64), 2.0 ** -149)
        else:
            unit[f] = np.maximum(by_id(sg[f], gids), by_id(so[f], oids))[None, :]
    if params is not None:
        dim = o[0].shape[0]
        v_step = np.max(np.broadcast_to(unit["v"], o[1].shape), axis=0)[None, :]
        units = comparison_units(params, dim, v_step, float(np.max(np.abs(o[1]))), steps)
        for f in names:
            unit[f] = np.maximum(unit[f], units[f])
    lsb = {f: np.abs(g[i] - o[i]) / unit[f] for i, f in enumerate(names)}
    return np.abs(g[0] - o[0]), lsb
