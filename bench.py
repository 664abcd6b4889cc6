"""Benchmark of the quantized MLS-MPM substep on one MI355X.

Metric: particle-substeps/s and bytes/particle, quantized vs the float32
layout, for the 3D elastic workload of 3e8 particles (186 cubes of 60^3
cells in a 512^3 grid, dt = 1e-4; x 3x21-bit fixed, v 3x13-bit
shared-exponent, C 9x16-bit shared-exponent, F 9x14-bit, all dithered: 48 B per particle
against 96 B for float32).  A step is one full substep of the hot path
(P2G, grid update, G2P, dithered re-encode and store), with the packed
state resident in HBM; the particle sort runs once at set-up (during the
warm-up) and its time is reported separately.

Prints one JSON line on stdout; progress goes to stderr.

  python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--config c3|c2|c1]
                  [--no-fp32] [--no-cpu] [--only quant|fp32]
  python bench.py --calib-copy   # plain copy of known size (counter calibration)
  python bench.py --calib-atomics  # 64-bit global atomic throughput (the flush's peak)
  python bench.py --config c4 [--batch-streams 4] [--max-particles N]   # serving stream
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-substeps/s and bytes/particle, quantized vs FP32 layout, at 1e-4 pos error"
HBM_PEAK_GBS = 8000.0
# the fused kernel's sources, and the run-time specialization that compiles it
KERNEL_SOURCES = ["paper_2207_04658_amd/csrc/substep.hpp", "paper_2207_04658_amd/csrc/mpmq_device.hpp",
                  "paper_2207_04658_amd/csrc/mpmq_internal.hpp", "paper_2207_04658_amd/csrc/jit.hip"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    """Hash of what the fused kernel is compiled from: its sources and the
    device flags that the build hands to the compiler (and to hipRTC)."""
    from paper_2207_04658_amd import build as _build
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    h.update(" ".join(_build.DEVICE_FLAGS).encode())
    return h.hexdigest()[:16]


VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: one VALU lane-instruction per cycle


def read_valu(config):
    """VALU wave-instructions per substep launch from the committed counter
    summary (same source hash as the traffic), or None."""
    path = os.path.join(ROOT, "profiles", f"substep_{config}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_sources_sha256_16:\s*([0-9a-f]+)", txt)
    m = re.search(r"valu_wave_instructions_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not m_hash or m_hash.group(1) != kernel_hash():
        return None
    return float(m.group(1))


def read_traffic(config):
    """HBM bytes per substep launch from the committed rocprofv3 counter
    summary, if it was taken with the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"substep_{config}_counters.md")
    if not os.path.exists(path):
        return None, None
    txt = open(path).read()
    m_hash = re.search(r"kernel_sources_sha256_16:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes:
        return None, None
    if m_hash.group(1) != kernel_hash():
        return None, "stale"
    return float(m_bytes.group(1)), "ok"


# ----------------------------------------------------------------------------- scenes
def build_scene(config, device):
    """Returns (scene dict without host state, device SoA tensors x, v, C, F)."""
    import numpy as np
    import torch
    import workloads as WL

    if config == "c3":
        lay = WL.c3_layout()
        n = sum(lay["counts"])
        params = WL.c3_params()
        scheme = WL.scheme_c3()
        x = torch.empty((3, n), dtype=torch.float32, device=device)
        v = torch.empty((3, n), dtype=torch.float32, device=device)
        off = 0
        t0 = time.time()
        for i in range(len(lay["counts"])):
            xi, vi = WL.cube_particles(0, i, lay["corners"][i], lay["side"], lay["counts"][i], lay["vels"][i])
            c = xi.shape[1]
            x[:, off:off + c].copy_(torch.from_numpy(xi))
            v[:, off:off + c].copy_(torch.from_numpy(vi))
            off += c
            if i % 40 == 0:
                log(f"generated cube {i}/{len(lay['counts'])} ({time.time() - t0:.1f}s)")
        desc = ("3D MLS-MPM elastic, 300M particles in 186 cubes of 60^3 cells, 512^3 grid, dt=1e-4, "
                "fixed-corotated E=100 nu=0.2; x 3x21b fixed, v 3x13b shared-exp (6b), C 9x16b shared-exp (6b), "
                "F 9x14b fixed (F-I), dithered")
        scene = {"name": "c3", "scheme": scheme, "params": params, "n": n, "desc": desc, "grid": 512,
                 "steps_cfg": 10}
    elif config == "fluid":
        # 3D fluid dam break: a column [0.1,0.4]x[0.1,0.6]x[0.3,0.7] of a 512^3 grid, 8 particles
        # per cell (64.4M particles), generated on the device from a seeded torch generator
        res, ppc = 512, 8
        lo = torch.tensor([0.1, 0.1, 0.3], dtype=torch.float64)
        hi = torch.tensor([0.4, 0.6, 0.7], dtype=torch.float64)
        n = int(round(float(torch.prod((hi - lo) * res)) * ppc))
        gen = torch.Generator(device=device)
        gen.manual_seed(7)
        x = torch.rand((3, n), generator=gen, device=device, dtype=torch.float32)
        x = (lo.to(device).float()[:, None] + (hi - lo).to(device).float()[:, None] * x).contiguous()
        v = torch.zeros((3, n), dtype=torch.float32, device=device)
        J = torch.ones((1, n), dtype=torch.float32, device=device)
        C = torch.zeros((9, n), dtype=torch.float32, device=device)
        vol = float(torch.prod(hi - lo))
        params = WL.params(3, res, 5e-5, vol / n, sort_every=0, material="fluid", E=WL.FLUID_E)
        desc = (f"3D MLS-MPM fluid dam break, {n} particles (8 per cell) in [0.1,0.4]x[0.1,0.6]x[0.3,0.7] of a "
                "512^3 grid, dt=5e-5, pressure coefficient 400; x 3x20b fixed, v 3x16b fixed, C 9x16b shared-exp "
                "(6b), J 16b fixed (J-1), dithered")
        scene = {"name": "fluid", "scheme": WL.scheme_fluid(3, True, 0), "params": params, "n": n, "desc": desc,
                 "grid": res, "steps_cfg": 10, "fp32_scheme": WL.scheme_fluid_fp32(3)}
        return scene, (x, v, C, J)
    else:
        sc = WL.c2() if config == "c2" else WL.c1()
        xh, vh, _, _ = sc["state"]
        n = sc["n"]
        x = torch.from_numpy(xh).to(device)
        v = torch.from_numpy(vh).to(device)
        desc = {"c2": "3D MLS-MPM elastic, 2^20 particles in 4 cubes, 128^3 grid, dt=2e-4, 52 B/particle dithered",
                "c1": "2D MLS-MPM elastic block, 8192 particles, 128^2 grid, dt=1e-4, 28 B/particle"}[config]
        scene = {"name": config, "scheme": sc["scheme"], "params": sc["params"], "n": n, "desc": desc,
                 "grid": sc["params"]["grid_res"], "steps_cfg": sc["steps"]}
    dim = scene["params"]["dim"]
    C = torch.zeros((dim * dim, n), dtype=torch.float32, device=device)
    F = torch.zeros((dim * dim, n), dtype=torch.float32, device=device)
    for a in range(dim):
        F[a * dim + a].fill_(1.0)
    return scene, (x, v, C, F)


def run_layout(mq, scene, scheme, state, steps, warmup, label, specialize=True):
    import torch
    n = scene["n"]
    ctx = mq.Context(scheme, scene["params"], n, track_ids=False)
    jit_s = 0.0
    if specialize:
        t0 = time.perf_counter()
        ctx.specialize(True)
        jit_s = time.perf_counter() - t0
        log(f"{label}: scheme-specialized kernels ready in {jit_s:.2f} s")
    sz = ctx.sizes
    log(f"{label}: W={sz['words_per_particle']} words, state {sz['packed_bytes'] / 1e9:.2f} GB, "
        f"scratch {sz['scratch_bytes'] / 1e9:.2f} GB, grid 2x{sz['grid_bytes'] / 1e9:.2f} GB")
    ctx.encode(*state)
    ctx.set_timing(True)
    ctx.step(warmup)  # includes the set-up sort
    warm = ctx.kernel_times()
    ctx.kernel_times(clear=True)
    sort_ms = warm.get("sort", (0, 0.0))[1]
    torch.cuda.synchronize()
    ctx.reset_stats()
    log(f"{label}: warm-up done (sort {sort_ms:.1f} ms); timing {steps} steps")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(ctx.stream)
    ctx.step(steps)
    stop.record(ctx.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    kt = ctx.kernel_times()
    st = ctx.stats()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    per_step = ms / max(steps, 1)
    log(f"{label}: {per_step:.3f} ms/step, kernels " +
        ", ".join(f"{k}={v[1] / max(v[0], 1):.3f}ms" for k, v in kt.items()))
    return {"ms_per_step": per_step, "value": n * steps / (ms / 1e3) if ms > 0 else 0.0,
            "kernels": {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)} for k, v in kt.items()},
            "sort_ms": sort_ms, "stats": st, "W": sz["words_per_particle"], "specialize_s": jit_s,
            "bytes_per_particle": 4 * sz["words_per_particle"],
            "footprint_bytes": sz["packed_bytes"] + 2 * sz["grid_bytes"] + sz["scratch_bytes"]}


def roofline(res, n, steps):
    """Algorithmic HBM bytes of one fused substep launch over its measured
    average duration: 8W bytes per particle (packed state read + written once)
    plus 32 bytes per active grid node (velocity gathered once, momentum and
    mass scattered once)."""
    k = res["kernels"].get("substep")
    if not k:
        return None
    active = res["stats"]["active_nodes"] / max(steps, 1)
    algo = 8.0 * res["W"] * n + 32.0 * active
    achieved = algo / (k["avg_ms"] / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_substep",
            "algorithmic_bytes_per_launch": algo, "avg_launch_ms": k["avg_ms"],
            "active_nodes_per_step": active}


def host_cpu():
    """CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable, os.cpu_count() or 1


def _oracle_cube_rate(args):
    """One worker of the parallel baseline: cube `i` of the 3e8-particle
    workload through the unchanged oracle, one warm-up substep (with the
    sort) and `reps` timed substeps.  Returns (particles, seconds)."""
    i, reps = args
    import oracle
    import workloads as WL
    sub = WL.c3(only=[i])
    x, v, C, F = sub["state"]
    words, _ = oracle.encode(sub["scheme"], x, v, C, F, 0, 2)
    sim = oracle.Sim(sub["scheme"], sub["params"], words)
    sim.step(1)
    t0 = time.perf_counter()
    sim.step(reps)
    dt = time.perf_counter() - t0
    sim.close()
    return sub["n"] * reps, dt


def cpu_baseline(scene):
    """The oracle (FP64) on a bounded sample of the workload: one thread
    (median of three timed substeps after a warm-up substep) and, for the
    3e8-particle workload, independent cubes in concurrent processes, one
    per usable core (at most 16), unchanged oracle code."""
    import numpy as np
    import oracle
    import workloads as WL
    model, usable, logical = host_cpu()
    if scene["name"] == "c3":
        sub = WL.c3(only=[0])
        sample = f"cube 0 of 186 ({sub['n']} particles) on the full 512^3 grid"
    elif scene["name"] == "c2":
        sub = WL.c2(cubes=1)
        sample = f"cube 0 of 4 ({sub['n']} particles) on the 128^3 grid"
    elif scene["name"] == "fluid":
        # a slab x in [0.1, 0.1075) of the column at the same density (8 per cell) on the 512^3 grid
        rng = np.random.default_rng(3)
        lo, hi = np.array([0.1, 0.1, 0.3]), np.array([0.1075, 0.6, 0.7])
        ns = int(round(float(np.prod((hi - lo) * 512)) * 8))
        xs = (lo[:, None] + (hi - lo)[:, None] * rng.random((3, ns))).astype(np.float32)
        state = (xs, np.zeros((3, ns), np.float32), np.zeros((9, ns), np.float32), np.ones((1, ns), np.float32))
        sub = {"scheme": scene["scheme"], "params": scene["params"], "n": ns, "state": state}
        sample = f"a slab of {ns} particles of the dam-break column (same density) on the full 512^3 grid"
    else:
        sub = WL.c1()
        sample = "the full scene (8192 particles)"
    x, v, C, F = sub["state"]
    words, _ = oracle.encode(sub["scheme"], x, v, C, F, 0, 2)
    sim = oracle.Sim(sub["scheme"], sub["params"], words)
    sim.step(1)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        sim.step(1)
        times.append(time.perf_counter() - t0)
    sim.close()
    med = float(np.median(times))
    single = sub["n"] / med
    out = {"value": single, "unit": "particle-substeps/s", "cores": 1, "kind": "oracle",
           "sample": sample + ": one warm-up substep (with the sort), then the median of three timed substeps",
           "seconds": round(sum(times), 3),
           "host_cpu": model, "usable_cores": usable, "logical_cpus": logical,
           "single_thread": {"value": round(single, 1), "substep_s": [round(t, 3) for t in times]}}
    if scene["name"] == "c3" and usable > 1:
        import multiprocessing as mp
        procs = min(usable, 16)
        reps = 2
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        with ctx.Pool(procs) as pool:
            res = pool.map(_oracle_cube_rate, [(i, reps) for i in range(procs)])
        wall = time.perf_counter() - t0
        work = sum(r[0] for r in res)
        slowest = max(r[1] for r in res)
        out.update(value=work / slowest, cores=procs,
                   sample=(f"cubes 0-{procs - 1} of 186 ({work // reps} particles), one per process on "
                           f"{procs} cores, each on the full 512^3 grid: {reps} timed substeps after a warm-up "
                           "substep (with the sort); rate = particle-substeps / the slowest process's timed "
                           f"seconds; single-thread figure: {sample}"),
                   parallel={"processes": procs, "timed_s": [round(r[1], 3) for r in res],
                             "wall_s_incl_setup": round(wall, 2)})
    return out


def atomics_peak(mq):
    """Device-wide 64-bit global atomic adds per second of the library's
    calibration kernel (mpmq_calib_atomics, stride 1: each wave instruction
    covers 64 consecutive words) over 2^27 words."""
    import torch
    n = 1 << 27
    buf = torch.zeros(n, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream()
    mq.calib_atomics(buf, passes=1, stream=st)
    torch.cuda.synchronize()
    passes = 4
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    mq.calib_atomics(buf, passes=passes, stream=st)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ok = bool(torch.all(buf == passes + 1).item())
    del buf
    torch.cuda.empty_cache()
    return {"peak_per_s": n * passes / (ms / 1e3), "words": n, "passes": passes, "ms": round(ms, 3),
            "pattern": "stride 1 (64 consecutive 8-byte words per wave instruction)", "checked": ok}


def calib_copy():
    import torch
    nbytes = 4 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": nbytes}))


def bench_serving(a):
    """Serving stream: throughput over the makespan and latency percentiles."""
    import numpy as np
    import workloads as WL
    from paper_2207_04658_amd.serving import Server
    t0 = time.time()
    scenes = [WL.c4_scene(0, i, materialize=False, n_max=a.max_particles) for i in range(a.scenes)]
    arrivals = WL.c4_arrivals(0, a.scenes, a.rate)
    log(f"generated {a.scenes} scenes ({sum(s['n'] for s in scenes)} particles) in {time.time() - t0:.1f}s")
    for batched in (True, False):  # loads the kernels of both paths
        warm = Server(streams=2, steps_per_tick=10, batched=batched).run(scenes[:2])
    log(f"warm-up: {len(warm.latencies_s)} scenes")
    # per-scene launches on 8 streams, for comparison
    per = Server(hbm_budget_bytes=200e9, streams=8, steps_per_tick=10, batched=False).run(scenes, arrivals)
    lat_per = np.array(list(per.latencies_s.values()))
    log(f"per-scene launches: {per.throughput():.3e} particle-substeps/s, p50 {np.percentile(lat_per, 50):.3f} s")
    res = Server(hbm_budget_bytes=200e9, streams=a.batch_streams, steps_per_tick=10, batched=True).run(scenes, arrivals)
    lat = np.array(list(res.latencies_s.values()))
    log(f"batched launches: {res.throughput():.3e} particle-substeps/s, p50 {np.percentile(lat, 50):.3f} s")
    line = {
        "metric": "serving throughput (particle-substeps/s) with per-scene latency",
        "value": round(res.throughput(), 1), "unit": "particle-substeps/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.scenes} MLS-MPM scenes (2D/3D), Poisson arrivals at {a.rate}/s, "
                               f"particles log-uniform 4096-{a.max_particles}, grids 32-256 per axis, 100 steps "
                               "each, random 12-24-bit schemes, 200 GB HBM budget"},
        "latency_s": {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
                      "max": round(float(lat.max()), 4)},
        "makespan_s": round(res.makespan_s, 4), "particle_substeps": res.particle_substeps,
        "max_active_scenes": res.max_active, "peak_hbm_bytes": res.peak_bytes,
        "queue_wait_s_max": round(max(res.queue_wait_s.values()), 4),
        "launches": "batched: one grid-update and one fused-substep launch per substep for all active scenes "
                    f"of a stream and dimension (mpmq_step_batch), scenes spread over {a.batch_streams} streams",
        "per_scene_launches": {"value": round(per.throughput(), 1),
                               "latency_s": {"p50": round(float(np.percentile(lat_per, 50)), 4),
                                             "p99": round(float(np.percentile(lat_per, 99)), 4)},
                               "makespan_s": round(per.makespan_s, 4), "streams": 8},
    }
    print(json.dumps(line), flush=True)


def bench_adjoint(a):
    """Adjoint scene at full size: forward + backward of 64 substeps."""
    import torch
    import numpy as np
    import oracle
    import workloads as WL
    import paper_2207_04658_amd as mq
    sc = WL.c5(seed=0)
    T = sc["steps"]
    res = {}
    for K in (8, 0):
        ctx = mq.Context(sc["scheme"], sc["params"], sc["n"], specialize=not a.generic)
        ts = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in sc["state"]]
        ctx.encode(*ts)
        ctx.adjoint(2, objective="ke", checkpoint_every=K)  # warm-up
        ms = []
        for _ in range(3):
            ctx.encode(*ts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.adjoint(T, objective="ke", checkpoint_every=K)
            ms.append((time.perf_counter() - t0) * 1e3)
        res[K] = (min(ms), r)
        log(f"adjoint K={K}: {min(ms):.1f} ms, recomputed {r['recomputed']}, states {r['states']}")
        ctx.close()
    # oracle: the FP64 adjoint of one substep on the same scene at 16^3 (4096 particles)
    small = WL.c5(seed=0, grid_res=16)
    x, v, C, F = small["state"]
    s0 = oracle.pack_state(*(np.asarray(t, dtype=np.float64) for t in (x, v, C, F)))
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < 5.0:
        oracle.step_vjp(small["params"], s0, s0)
        reps += 1
    cpu_rate = reps * small["n"] / (time.perf_counter() - t0)
    n = sc["n"]
    ms8, r8 = res[8]
    line = {
        "metric": "adjoint particle-substeps/s (forward + backward through the quantized substep)",
        "value": round(n * T / (ms8 / 1e3), 1), "unit": "particle-substeps/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D elastic cube, 262144 particles, 64^3 grid, 64 steps, checkpoint every 8, "
                               "kinetic-energy objective, c2 scheme"},
        "ms": {"checkpoint_every_8": round(ms8, 2), "bisection": round(res[0][0], 2)},
        "states_held": {"checkpoint_every_8": r8["states"], "bisection": res[0][1]["states"]},
        "recomputed_substeps": {"checkpoint_every_8": r8["recomputed"], "bisection": res[0][1]["recomputed"]},
        "g": r8["g"],
        "kernels_specialized": not a.generic,
        "cpu_baseline": {"value": round(cpu_rate, 1), "unit": "particle-substeps/s (backward only)", "cores": 1,
                         "kind": "oracle", "sample": "orc_step_vjp on the 16^3 version of the scene (4096 particles)"},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5", "fluid"])
    ap.add_argument("--scenes", type=int, default=256, help="c4: scenes in the stream")
    ap.add_argument("--rate", type=float, default=200.0, help="c4: Poisson arrival rate (scenes/s)")
    ap.add_argument("--batch-streams", type=int, default=4, help="c4: streams of the batched server")
    ap.add_argument("--max-particles", type=int, default=2 ** 21, help="c4: largest scene (log-uniform from 4096)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["quant", "fp32"], default=None)
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--calib-atomics", action="store_true",
                    help="64-bit global atomic adds per second of the calibration kernel")
    ap.add_argument("--generic", action="store_true", help="run the generic (run-time scheme) kernels")
    ap.add_argument("--sort-every", type=int, default=None,
                    help="c3: re-sort every S substeps (default: the workload's set-up sort only)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X: the library has no multi-GPU path (it would shard the grid "
              "by spatial slabs and exchange the node shells of shared faces); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if a.calib_copy:
        calib_copy()
        return
    if a.calib_atomics:
        import paper_2207_04658_amd as mq
        mq.load()
        print(json.dumps({"calib_atomics": atomics_peak(mq)}))
        return
    import torch
    import paper_2207_04658_amd as mq
    import workloads as WL
    mq.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.config == "c4":
        return bench_serving(a)
    if a.config == "c5":
        return bench_adjoint(a)
    scene, state = build_scene(a.config, dev)
    if a.sort_every is not None:
        scene["params"] = dict(scene["params"], sort_every=int(a.sort_every))
        scene["desc"] += f"; re-sorted every {a.sort_every} substeps"
    n = scene["n"]
    log(f"scene {scene['name']}: {n} particles")
    out = {}
    if a.only in (None, "quant"):
        out["quant"] = run_layout(mq, scene, scene["scheme"], state, a.steps, a.warmup, "quantized",
                                  specialize=not a.generic)
    if a.only == "fp32" or (a.only is None and not a.no_fp32):
        fp32_scheme = scene.get("fp32_scheme") or WL.scheme_fp32(scene["params"]["dim"])
        out["fp32"] = run_layout(mq, scene, fp32_scheme, state, a.steps, a.warmup, "fp32 layout",
                                 specialize=not a.generic)
    del state
    torch.cuda.empty_cache()
    main_res = out.get("quant") or out["fp32"]
    rf = roofline(main_res, n, a.steps)
    traffic, tstate = read_traffic(scene["name"]) if not a.generic else (None, "counters are of the specialized kernel")
    if rf is not None:
        rf["traffic"] = traffic
        rf["traffic_status"] = tstate or "no counter summary"
        valu = read_valu(scene["name"]) if not a.generic else None
        if valu is not None:
            # the fused kernel is limited by vector-ALU issue: its counted VALU
            # lane-instructions per second against one per lane per cycle
            ach = valu * 64 / (rf["avg_launch_ms"] / 1e3)
            rf["valu_issue"] = {"achieved": round(ach / 1e12, 2), "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
                                "unit": "T lane-instr/s", "frac": round(ach / VALU_PEAK_LANE_OPS, 4),
                                "instructions_per_launch": valu}
    if rf is not None:
        # the P2G tile flushes' 64-bit global atomics (counted by the kernel)
        # against the calibration kernel's rate
        peak = atomics_peak(mq)
        per_launch = main_res["stats"].get("atomics", 0) / max(a.steps, 1)
        ach = per_launch / (rf["avg_launch_ms"] / 1e3)
        rf["atomics"] = {"achieved": round(ach / 1e9, 3), "peak": round(peak["peak_per_s"] / 1e9, 3),
                         "unit": "G atomic adds/s", "frac": round(ach / peak["peak_per_s"], 4),
                         "per_launch": per_launch, "calibration": peak}
        log(f"atomics: {per_launch:.3e} per launch, {ach:.3e}/s against {peak['peak_per_s']:.3e}/s")
    cpu = None
    if not a.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(scene)
        log(f"cpu baseline {cpu['value']:.3g} particle-substeps/s in {cpu['seconds']} s")
    q, f = out.get("quant"), out.get("fp32")
    line = {
        "metric": METRIC,
        "value": round(main_res["value"], 1),
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": scene["desc"], "particles": n, "grid": scene["grid"],
                   "layout": "quantized" if q else "fp32"},
        "bytes_per_particle": main_res["bytes_per_particle"],
        "footprint_bytes_per_particle": round(main_res["footprint_bytes"] / n, 2),
        "sort_ms": round(main_res["sort_ms"], 3),
        "kernels_specialized": not a.generic, "specialize_s": round(main_res["specialize_s"], 3),
        "kernels_avg_ms": {k: round(v["avg_ms"], 4) for k, v in main_res["kernels"].items()},
        "roofline": rf,
        "cpu_baseline": cpu,
    }
    if q and f:
        line["fp32_layout"] = {"value": round(f["value"], 1), "ms_per_step": round(f["ms_per_step"], 4),
                               "bytes_per_particle": f["bytes_per_particle"],
                               "footprint_bytes_per_particle": round(f["footprint_bytes"] / n, 2),
                               "kernels_avg_ms": {k: round(v["avg_ms"], 4) for k, v in f["kernels"].items()}}
        line["speedup_vs_fp32"] = round(q["value"] / f["value"], 4)
        line["compression_vs_fp32"] = round(f["bytes_per_particle"] / q["bytes_per_particle"], 4)
        line["fp32_roofline"] = roofline(f, n, a.steps)
    fields = [k for k in ("x", "v", "C", "F", "J") if k in main_res["stats"]]
    line["saturations"] = {k: main_res["stats"][k]["sat"] for k in fields}
    line["nan"] = {k: main_res["stats"][k]["nan"] for k in fields}
    line["fallback_stencils"] = main_res["stats"]["fallback"]
    line["wide_scatters"] = main_res["stats"]["wide"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
