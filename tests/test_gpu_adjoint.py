"""GPU adjoint (mpmq_adjoint, Sec. 6, Eqs. 8, 12-13) against the FP64
oracle adjoint on the same seeded inputs.

The oracle runs its own quantized trajectory (FP64 substeps, same codec and
Philox draws) and back-propagates through it with orc_step_vjp; the GPU runs
its FP32 substeps and its adjoint kernels.  The two trajectories can differ by
one code where a dithered rounding falls within FP32 error of a lattice
boundary, so quantities that depend on later states are compared with
tolerances scaled by each field's magnitude; after one substep from a
bit-identical encoded state (centre-of-mass objective, whose lambda_T is a
constant) lambda_0 is compared element by element.
"""
import math

import numpy as np
import pytest

import workloads as WL
from gpu_common import by_id, gpu_context, note

pytestmark = pytest.mark.gpu

FIELDS = ["x", "v", "C", "F"]


def oracle_trajectory(orc, scene, T):
    """Stored states s_0..s_T of the oracle's quantized run, in encode order."""
    sc, pr = scene["scheme"], scene["params"]
    x, v, C, F = scene["state"]
    w0, _ = orc.encode(sc, x, v, C, F, 0, 2)
    sim = orc.Sim(sc, pr, w0)
    states = [orc.pack_state(*orc.decode(sc, w0))]
    for _ in range(T):
        sim.step(1)
        st = orc.pack_state(*orc.decode(sc, sim.words()))
        states.append(by_id(st, sim.ids()))
    sim.close()
    return states


def field_slices(dim):
    d2 = dim * dim
    return {"x": slice(0, dim), "v": slice(dim, 2 * dim), "C": slice(2 * dim, 2 * dim + d2),
            "F": slice(2 * dim + d2, 2 * dim + 2 * d2)}


def field_steps(scheme):
    """Quantization step of each field (the Delta_h of Eq. 8)."""
    out = {}
    for f in scheme["fields"]:
        if f["kind"] == "fixed":
            out[f["field"]] = (f["hi"] - f["lo"]) * 2.0 ** -f["bits"]
        elif f["kind"] == "shared_exp":
            out[f["field"]] = 2.0 ** math.ceil(math.log2(f["hi"])) * 2.0 ** -(f["bits"] - 1)
        else:
            out[f["field"]] = 2.0 ** -23
    return out


def assert_weighted_close(got, ref, steps, rtol, what, power=1):
    """Per field f, got[f] and ref[f] (arrays or numbers) compared in units of
    the objective: each is weighted by Delta_f^power (the size of the error
    it multiplies).  Fields whose weighted magnitude is at least 1e-3 of the
    largest must agree to rtol of their own magnitude; all fields to rtol of
    the largest (fields that vanish analytically, e.g. C and F under the
    centre-of-mass objective, hold FP32 round-off only)."""
    w = {f: steps[f] ** power for f in FIELDS}
    mag = {f: float(np.max(np.abs(np.asarray(ref[f], dtype=np.float64)))) * w[f] for f in FIELDS}
    top = max(mag.values())
    for f in FIELDS:
        err = float(np.max(np.abs(np.asarray(got[f], dtype=np.float64) - np.asarray(ref[f], dtype=np.float64)))) * w[f]
        assert err <= rtol * top + 1e-300, f"{what}: {f} err {err:.3e} vs top {top:.3e}"
        if mag[f] >= 1e-3 * top:
            assert err <= rtol * mag[f], f"{what}: {f} err {err:.3e} vs own {mag[f]:.3e}"


def split_lambda(lam, dim):
    return {f: lam[sl] for f, sl in field_slices(dim).items()}


def small_scene(dim):
    if dim == 2:
        sc = WL.c1(seed=3, n=4096)
        sc["params"]["sort_every"] = 0
        return sc
    return WL.c5(seed=1, grid_res=16)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", ["com", "ke"])
def test_adjoint_one_step_lambda0(gpu_lib, orc, dim, kind):
    note(f"adjoint one step dim={dim} objective={kind}")
    scene = small_scene(dim)
    ctx = gpu_context(gpu_lib, scene)
    res = ctx.adjoint(1, objective=kind, axis=1, checkpoint_every=1, want_lambda0=True)
    lg = res["lambda0"].cpu().numpy().astype(np.float64)
    states = oracle_trajectory(orc, scene, 1)
    z, G, g, A, lo = orc.adjoint_full(scene["params"], states, kind, 1)
    steps = field_steps(scene["scheme"])
    # COM: lambda_1 is exact and s_0 is bit-identical, so only FP32 arithmetic differs
    assert_weighted_close(split_lambda(lg, dim), split_lambda(lo, dim), steps, 2e-3 if kind == "com" else 1e-2,
                          "lambda_0")
    assert math.isclose(res["z"], z, rel_tol=1e-5 if kind == "com" else 1e-3)
    assert_weighted_close(res["g"], g, steps, 2e-2, "g", power=2)
    assert_weighted_close(res["G"], G, steps, 1e-2, "G")
    ctx.close()


@pytest.mark.parametrize("dim,T", [(2, 6), (3, 8)])
@pytest.mark.parametrize("kind", ["com", "ke"])
@pytest.mark.parametrize("K", [3, 0])
def test_adjoint_trajectory_vs_oracle(gpu_lib, orc, dim, T, kind, K):
    note(f"adjoint trajectory dim={dim} T={T} objective={kind} K={K}")
    scene = small_scene(dim)
    ctx = gpu_context(gpu_lib, scene)
    res = ctx.adjoint(T, objective=kind, axis=1, checkpoint_every=K, want_lambda0=True)
    lg = res["lambda0"].cpu().numpy().astype(np.float64)
    states = oracle_trajectory(orc, scene, T)
    z, G, g, A, lo = orc.adjoint_full(scene["params"], states, kind, 1)
    assert math.isclose(res["z"], z, rel_tol=1e-5 if kind == "com" else 2e-3), (res["z"], z)
    steps = field_steps(scene["scheme"])
    assert_weighted_close(split_lambda(lg, dim), split_lambda(lo, dim), steps, 2e-2, "lambda_0")
    assert_weighted_close(res["g"], g, steps, 3e-2, "g", power=2)
    assert_weighted_close(res["G"], G, steps, 2e-2, "G")
    # Alg. 1 ranges: min / max of the stored values over s_0..s_T
    stack = np.stack(states)
    rel_f = any(fs["field"] == "F" and fs.get("rel_identity") for fs in scene["scheme"]["fields"])
    for f, sl in field_slices(dim).items():
        vals = stack[:, sl, :].copy()
        if f == "F" and rel_f:
            for a in range(dim):
                vals[:, a * (dim + 1), :] -= 1.0
        span = float(vals.max() - vals.min()) + 1e-12
        assert abs(res["lo"][f] - float(vals.min())) <= 1e-3 * span, f
        assert abs(res["hi"][f] - float(vals.max())) <= 1e-3 * span, f
    ctx.close()


def bisect_recomputed(T):
    """Substeps re-run by the bisection schedule (forward keeps the
    midpoints on the path to the last step)."""
    right = set()
    lo, hi = 0, T
    while hi - lo > 1:
        mid = (lo + hi) // 2
        right.add(mid)
        lo = mid

    def rev(lo, hi):
        if hi - lo == 1:
            return 0
        mid = (lo + hi) // 2
        cost = 0 if mid in right else mid - lo
        right.discard(mid)
        return cost + rev(mid, hi) + rev(lo, mid)

    return rev(0, T) if T > 0 else 0


def test_adjoint_checkpoint_modes_agree(gpu_lib):
    note("adjoint checkpoint modes K=1,4,13,0 T=13")
    scene = WL.c5(seed=2, grid_res=16)
    T = 13
    out = {}
    for K in [1, 4, 13, 0]:
        ctx = gpu_context(gpu_lib, scene)
        out[K] = ctx.adjoint(T, objective="ke", checkpoint_every=K, want_lambda0=True)
        out[K]["lambda0"] = out[K]["lambda0"].cpu().numpy().astype(np.float64)
        ctx.close()
    ref = out[1]
    steps = field_steps(scene["scheme"])
    for K, r in out.items():
        assert math.isclose(r["z"], ref["z"], rel_tol=1e-12), K  # identical forward
        assert_weighted_close(r["g"], ref["g"], steps, 1e-4, f"g K={K}", power=2)
        assert_weighted_close(split_lambda(r["lambda0"], 3), split_lambda(ref["lambda0"], 3), steps, 1e-4,
                              f"lambda_0 K={K}")
        if K >= 1:
            nseg = -(-T // K)
            assert r["recomputed"] == T - nseg, (K, r["recomputed"])
            assert r["states"] <= nseg + K, (K, r["states"])
        else:
            assert r["recomputed"] == bisect_recomputed(T), r["recomputed"]
            assert r["states"] <= math.ceil(math.log2(T)) + 2, r["states"]


def test_adjoint_leaves_forward_state(gpu_lib):
    note("adjoint leaves s_T like mpmq_step")
    scene = WL.c5(seed=4, grid_res=16)
    a = gpu_context(gpu_lib, scene)
    b = gpu_context(gpu_lib, scene)
    a.adjoint(7, objective="com", checkpoint_every=0)
    b.step(7)
    assert a.step_count() == b.step_count() == 7
    assert np.array_equal(a.words(), b.words())
    assert np.array_equal(a.ids(), b.ids())
    sa, sb = a.stats(), b.stats()
    for f in FIELDS:
        assert sa[f]["sat"] == sb[f]["sat"] and sa[f]["nan"] == sb[f]["nan"], f
    a.step(3)
    b.step(3)
    assert np.array_equal(a.words(), b.words())
    a.close()
    b.close()


def test_rollout_autograd(gpu_lib):
    import torch
    note("rollout autograd")
    scene = WL.c5(seed=5, grid_res=16)
    dev = torch.device("cuda", 0)
    ts = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).requires_grad_(True) for a in scene["state"]]
    ctx = gpu_lib.Context(scene["scheme"], scene["params"], scene["n"])
    z = gpu_lib.rollout(ctx, *ts, steps=5, objective="ke", checkpoint_every=2)
    z.backward()
    ref_ctx = gpu_context(gpu_lib, scene)
    ref = ref_ctx.adjoint(5, objective="ke", checkpoint_every=2, want_lambda0=True)
    lam = ref["lambda0"].cpu().numpy().astype(np.float64)
    grads = np.concatenate([t.grad.cpu().numpy().astype(np.float64) for t in ts], axis=0)
    assert math.isclose(float(z.detach()), ref["z"], rel_tol=1e-12)
    steps = field_steps(scene["scheme"])
    assert_weighted_close(split_lambda(grads, 3), split_lambda(lam, 3), steps, 1e-4, "autograd")
    ctx.close()
    ref_ctx.close()


def test_adjoint_empty_and_zero_steps(gpu_lib, orc):
    note("adjoint n=0 and T=0")
    scene = WL.c5(seed=6, grid_res=16)
    ctx = gpu_context(gpu_lib, scene)
    res = ctx.adjoint(0, objective="com", axis=2, want_lambda0=True)
    lg = res["lambda0"].cpu().numpy()
    n = scene["n"]
    assert np.all(lg[2] == np.float32(1.0 / n)) and np.count_nonzero(lg) == n
    assert math.isclose(res["G"]["x"], 1.0, rel_tol=1e-9)
    assert ctx.step_count() == 0
    ctx.close()
    empty = dict(scene)
    empty["state"] = tuple(a[:, :0] for a in scene["state"])
    ctx = gpu_context(gpu_lib, empty, capacity=64)
    res = ctx.adjoint(4, objective="ke")
    assert res["z"] == 0.0 and ctx.step_count() == 4
    ctx.close()


def test_adjoint_rejects_bad_spec(gpu_lib):
    note("adjoint spec errors")
    scene = WL.c5(seed=7, grid_res=16)
    ctx = gpu_context(gpu_lib, scene)
    for kw in [dict(axis=3), dict(checkpoint_every=-1), dict(objective="ke", steps=-1)]:
        args = dict(steps=2, objective="com", axis=1, checkpoint_every=2)
        args.update(kw)
        with pytest.raises(gpu_lib.MpmqError):
            ctx.adjoint(args.pop("steps"), **args)
    ctx.close()


@pytest.mark.timeout(600)
def test_adjoint_c5_full(gpu_lib, orc):
    """Adjoint scene at its full size: 262144 particles, 64^3, 64 substeps,
    checkpoint every 8 (and bisection)."""
    import time
    note("adjoint c5 full: T=1 lambda_0 vs oracle")
    scene = WL.c5(seed=0)
    ctx = gpu_context(gpu_lib, scene)
    res = ctx.adjoint(1, objective="com", axis=1, checkpoint_every=1, want_lambda0=True)
    lg = res["lambda0"].cpu().numpy().astype(np.float64)
    states = oracle_trajectory(orc, scene, 1)
    z, G, g, A, lo = orc.adjoint_full(scene["params"], states, "com", 1)
    steps = field_steps(scene["scheme"])
    assert_weighted_close(split_lambda(lg, 3), split_lambda(lo, 3), steps, 2e-3, "c5 lambda_0")
    # the per-field sums over 262,144 particles (reductions that share
    # accumulator copies across work-groups) and the recorded ranges
    assert math.isclose(res["z"], z, rel_tol=1e-5)
    assert_weighted_close(res["G"], G, steps, 1e-2, "c5 G")
    assert_weighted_close(res["g"], g, steps, 2e-2, "c5 g", power=2)
    stack = np.stack(states)
    for f, sl in field_slices(3).items():
        vals = stack[:, sl, :].copy()
        if f == "F":
            for a_ in range(3):
                vals[:, 4 * a_, :] -= 1.0
        span = float(vals.max() - vals.min()) + 1e-12
        assert abs(res["lo"][f] - float(vals.min())) <= 1e-3 * span, f
        assert abs(res["hi"][f] - float(vals.max())) <= 1e-3 * span, f
    ctx.close()
    out = {}
    for K in [8, 0]:
        note(f"adjoint c5 full: T=64 K={K}")
        ctx = gpu_context(gpu_lib, scene)
        t0 = time.perf_counter()
        out[K] = ctx.adjoint(64, objective="com", axis=1, checkpoint_every=K)
        dt = time.perf_counter() - t0
        print(f"[c5] K={K} adjoint {dt * 1e3:.1f} ms recomputed={out[K]['recomputed']} "
              f"states={out[K]['states']} ws={out[K]['workspace_bytes'] / 2**20:.1f} MiB", flush=True)
        ctx.close()
    a, b = out[8], out[0]
    assert math.isclose(a["z"], b["z"], rel_tol=1e-12)
    for f in FIELDS:
        assert math.isfinite(a["g"][f]) and math.isfinite(a["G"][f]), f
    assert_weighted_close(a["g"], b["g"], steps, 1e-4, "c5 g", power=2)
    # a uniform shift of every position at any step moves the centre of
    # mass by the same amount (quadratic B-splines reproduce affine fields)
    assert abs(a["G"]["x"] - 65.0) <= 0.05 * 65.0, a["G"]["x"]


def full_precision_scheme(dim, seed=0):
    """Every field as raw float32 (F stored as F - I, like the quantized
    schemes), the full-precision run of Alg. 1."""
    return {"dim": dim, "seed": seed, "fields": [WL.raw("x"), WL.raw("v"), WL.raw("C"), WL.raw("F", rel_identity=True)]}


def test_alg1_error_bounded_scheme(gpu_lib):
    """Alg. 1 end to end: gradients and ranges from a full-precision run,
    bits from the error-bounded solver (Eq. 10), then the quantized run's
    objective stays within the requested relative error.  The scheme is
    dithered (Sec. 5): its rounding errors are unbiased and independent
    between steps as the error model of Eq. 8 assumes, with variance
    Delta^2 / 6 instead of Delta^2 / 12, so the RMS error bound is
    sqrt(2) eps z."""
    note("Alg. 1 error-bounded on the adjoint scene (16^3, 16 steps)")
    scene = WL.c5(seed=8, grid_res=16)
    T, eps = 16, 1e-3
    fp = WL.with_scheme(scene, full_precision_scheme(3, 8))
    ctx = gpu_context(gpu_lib, fp)
    ref = ctx.adjoint(T, objective="ke", checkpoint_every=4)
    ctx.close()
    base = WL.scheme_c1(3, True, 8)
    scheme, sol = gpu_lib.auto_scheme(base, ref, scene["n"], mode="error", eps=eps, min_bits=4)
    print(f"[alg1] z={ref['z']:.6e} bits={sol['bits']} g={ref['g']}", flush=True)
    assert sol["expected_error"] <= (eps * ref["z"]) ** 2
    errs = []
    for seed in range(3):
        scheme["seed"] = 100 + seed
        q = gpu_context(gpu_lib, WL.with_scheme(scene, scheme))
        errs.append(q.adjoint(T, objective="ke", checkpoint_every=4)["z"] - ref["z"])
        q.close()
    rms = math.sqrt(sum(e * e for e in errs) / len(errs))
    print(f"[alg1] errors {errs} rms/z {rms / ref['z']:.3e} (eps {eps})", flush=True)
    assert rms <= 3.0 * math.sqrt(2.0) * eps * abs(ref["z"]), (errs, ref["z"])


def test_alg1_memory_bounded_scheme(gpu_lib):
    note("Alg. 1 memory-bounded on the adjoint scene (16^3, 16 steps)")
    scene = WL.c5(seed=9, grid_res=16)
    T = 16
    fp = WL.with_scheme(scene, full_precision_scheme(3, 9))
    ctx = gpu_context(gpu_lib, fp)
    ref = ctx.adjoint(T, objective="ke", checkpoint_every=0)
    ctx.close()
    scheme, sol = gpu_lib.auto_scheme(WL.scheme_c1(3, True, 9), ref, scene["n"], mode="memory", eps=0.5, min_bits=4)
    n = scene["n"]
    assert sol["total_bits"] <= 0.5 * 32 * n * (3 + 3 + 9 + 9)
    sizes = gpu_lib.mpmq_query_sizes(scheme, scene["params"], n)
    assert sizes["record_bits"] == sum(f["bits"] * (3 if f["field"] in "xv" else 9) for f in scheme["fields"])
    q = gpu_context(gpu_lib, WL.with_scheme(scene, scheme))
    zq = q.adjoint(T, objective="ke", checkpoint_every=0)["z"]
    q.close()
    assert math.isfinite(zq) and abs(zq - ref["z"]) <= 0.05 * abs(ref["z"]), (zq, ref["z"])


@pytest.mark.parametrize("dim", [2, 3])
def test_adjoint_tile_fallback_vs_oracle(gpu_lib, orc, dim):
    """A fast cube, sorted once: stencils leave the node tiles of their sort
    blocks, so the forward and the G2P backward also take their grid-wide
    atomic paths; lambda_0, G and g still match the oracle."""
    # 2D node blocks are 16 cells wide: a finer grid, so that there are several
    res, T = (64, 8) if dim == 2 else (16, 8)
    dt = 5e-4 if dim == 2 else 1e-3
    side = 6 / res
    # just above a node-block boundary, moving towards it
    corners = np.array([[0.26, 0.27]]) if dim == 2 else np.array([[0.35, 0.4, 0.35]])
    vels = np.array([[-17.0, -11.0, -14.0]])[:, :dim]
    scheme = WL.scheme_c1(dim, True, 4)
    scene = WL.cubes_scene("fast", 4, res, corners, side, [8 * 6 ** dim], vels, dt, T, scheme, 0, dim=dim)
    note(f"adjoint tile fallback dim={dim} n={scene['n']} T={T}")
    ctx = gpu_context(gpu_lib, scene)
    res_g = ctx.adjoint(T, objective="ke", axis=1, checkpoint_every=3, want_lambda0=True)
    st = ctx.stats()
    assert st["fallback"] > 0 and st["sorts"] == 1, st
    lg = res_g["lambda0"].cpu().numpy().astype(np.float64)
    states = oracle_trajectory(orc, scene, T)
    z, G, g, A, lo = orc.adjoint_full(scene["params"], states, "ke", 1)
    assert math.isclose(res_g["z"], z, rel_tol=2e-3), (res_g["z"], z)
    steps = field_steps(scene["scheme"])
    assert_weighted_close(split_lambda(lg, dim), split_lambda(lo, dim), steps, 2e-2, "lambda_0")
    assert_weighted_close(res_g["g"], g, steps, 3e-2, "g", power=2)
    assert_weighted_close(res_g["G"], G, steps, 2e-2, "G")
    ctx.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", ["ke", "com"])
def test_adjoint_c5_T64_vs_oracle(gpu_lib, kind):
    """The adjoint workload at its own horizon: 262,144 particles, 64
    dithered substeps, checkpoint every 8, against the oracle's adjoint of
    the same scene (tests/golden/c5_adjoint_T64.json, written by
    make_c5_adjoint.py from the oracle alone).  Both sides run their own
    quantized trajectory with the same slots and dither streams, so they
    differ where FP32 flips a rounding near a tie; z, G, g, the recorded
    ranges and lambda_0 of 512 sampled particles are compared in units of
    the objective (each field weighted by its quantization step), at the
    bars of the short-horizon trajectory tests."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_adjoint_T64.json")
    ref = json.load(open(path))
    o = ref["objectives"][kind]
    scene = WL.c5(seed=0)
    note(f"adjoint c5 T=64 K=8 objective={kind} vs golden")
    ctx = gpu_context(gpu_lib, scene)
    res = ctx.adjoint(64, objective=kind, axis=o["axis"], checkpoint_every=8, want_lambda0=True)
    lg = res["lambda0"].cpu().numpy().astype(np.float64)[:, ref["sample"]]
    ctx.close()
    steps = field_steps(scene["scheme"])
    print(f"[c5 T=64 {kind}] z gpu {res['z']:.9e} oracle {o['z']:.9e}; G {res['G']} vs {o['G']}; "
          f"g {res['g']} vs {o['g']}", flush=True)
    assert math.isclose(res["z"], o["z"], rel_tol=1e-5 if kind == "com" else 2e-3), (res["z"], o["z"])
    assert_weighted_close(split_lambda(lg, 3), split_lambda(np.asarray(o["lambda0_sample"]), 3), steps, 2e-2,
                          "lambda_0")
    assert_weighted_close(res["g"], o["g"], steps, 3e-2, "g", power=2)
    assert_weighted_close(res["G"], o["G"], steps, 2e-2, "G")
    for f in FIELDS:
        span = ref["hi"][f] - ref["lo"][f] + 1e-12
        assert abs(res["lo"][f] - ref["lo"][f]) <= 1e-3 * span, f
        assert abs(res["hi"][f] - ref["hi"][f]) <= 1e-3 * span, f
