"""Seeded synthetic inputs for the quantized MLS-MPM substep.

This module holds input descriptions and generators only -- no arithmetic of
the method.  The GPU library, the oracle, the tests and the benchmark all
take their schemes, parameters and initial particle states from here, and
nothing here depends on either solver.

Workloads (scenes of the shapes the paper measures, Sec. 8.1 and
Table "large_scale"):
  c1  2D elastic block at rest, 8192 particles uniform in [0.3,0.5]^2,
      128^2 grid, E=1e3 nu=0.2 rho=1, dt=1e-4, 50 steps; x 2x20-bit fixed in
      [0,1), v 2x16 in [-20,20], C 4x16 in [-50,50], F 4x16 (F-I in [-1,1]),
      round to nearest.
  c2  3D, 2^20 particles as 4 cubes of side 32 cells (8 particles per cell),
      each with one velocity drawn from U(-1,1)^3, 128^3 grid, dt=2e-4,
      100 steps; the c1 scheme in 3D with dithered rounding everywhere.
  c3  3D, 3e8 particles in 186 cubes of 60^3 cells, each centred in its own
      64^3 slot of the 8^3 slot lattice of a 512^3 grid (30% filled),
      dt=1e-4, 10 steps; x 3x21-bit fixed, v 3x13-bit shared-exponent float
      (6-bit exponent), F 9x14-bit fixed (F-I), C 9x16-bit shared-exponent
      float (6-bit exponent, |C| < 2048), all dithered: 384 bits = 12 words
      = 48 B per particle; E=100 (see c3_params).
  c5  3D adjoint scene: one cube of side 0.5 (8 particles per cell, so
      grid_res^3 particles: 262144 at 64^3), corner (0.25, 0.25, 0.25),
      velocity = one U(-1,1)^3 drift + a rigid spin with angular velocity
      U(-2,2)^3 about the cube centre + per-particle U(-0.1,0.1) noise;
      dt=2e-4, 64 steps, the c2 scheme, no re-sort.
  c4  serving stream: 256 scenes arriving as a Poisson process; per scene
      (seeded by its index) 2D or 3D with equal odds, a grid resolution from
      {32, 64, 128, 256} (per axis), a particle count log-uniform in
      [4096, 2^21] placed uniformly in a box of half the domain's side
      centred at (0.5, 0.6, 0.5), one velocity from U(-1,1)^d, a random
      scheme (12-24 bits per field, random kinds, dither and placement
      order), dt = 0.25 dx / c with c the P-wave speed, 100 steps.
  fp32 layout: the same scene with every field stored as raw float32.
"""
from __future__ import annotations

import copy
import math

import numpy as np

E_MODULUS = 1e3
POISSON = 0.2
DENSITY = 1.0


def fixed(field, bits, lo, hi, dither=False, rel_identity=False):
    return {"field": field, "kind": "fixed", "bits": bits, "lo": lo, "hi": hi,
            "dither": dither, "rel_identity": rel_identity, "exp_bits": 0}


def shared_exp(field, bits, exp_bits, hi, dither=False):
    return {"field": field, "kind": "shared_exp", "bits": bits, "exp_bits": exp_bits,
            "lo": -hi, "hi": hi, "dither": dither, "rel_identity": False}


def raw(field, rel_identity=False):
    return {"field": field, "kind": "raw_f32", "bits": 32, "lo": 0.0, "hi": 1.0,
            "dither": False, "rel_identity": rel_identity, "exp_bits": 0}


def scheme_c1(dim=2, dither=False, seed=0):
    return {"dim": dim, "seed": seed, "fields": [
        fixed("x", 20, 0.0, 1.0, dither),
        fixed("v", 16, -20.0, 20.0, dither),
        fixed("C", 16, -50.0, 50.0, dither),
        fixed("F", 16, -1.0, 1.0, dither, rel_identity=True)]}


def scheme_c3(seed=0):
    return {"dim": 3, "seed": seed, "fields": [
        fixed("x", 21, 0.0, 1.0, True),
        shared_exp("v", 13, 6, 20.0, True),
        shared_exp("C", 16, 6, 2048.0, True),
        fixed("F", 14, -1.0, 1.0, True, rel_identity=True)]}


def scheme_fluid(dim=2, dither=False, seed=0):
    """Fluid state x, v, C, J (Sec. 8.3: position, velocity, volume ratio,
    affine velocity): x 20-bit, v 16-bit in [-20, 20], C 16-bit shared
    exponent (|C| < 2048; the paper widens C's range for its fluid), J 16-bit
    stored as J - 1 in [-0.5, 0.5]."""
    return {"dim": dim, "seed": seed, "fields": [
        fixed("x", 20, 0.0, 1.0, dither),
        fixed("v", 16, -20.0, 20.0, dither),
        shared_exp("C", 16, 6, 2048.0, dither),
        fixed("J", 16, -0.5, 0.5, dither, rel_identity=True)]}


def scheme_fluid_fp32(dim=2, seed=0):
    return {"dim": dim, "seed": seed, "fields": [raw("x"), raw("v"), raw("C"), raw("J")]}


def scheme_fp32(dim=3, seed=0):
    return {"dim": dim, "seed": seed, "fields": [raw("x"), raw("v"), raw("C"), raw("F")]}


def params(dim, grid_res, dt, p_vol, sort_every=0, bound_cells=3, gravity=-9.8, material="elastic", E=None):
    g = [0.0, gravity, 0.0][:3]
    return {"dim": dim, "grid_res": grid_res, "bound_cells": bound_cells,
            "sort_every": sort_every, "dt": dt, "gravity": g, "E": E_MODULUS if E is None else E,
            "nu": POISSON, "rho": DENSITY, "p_vol": p_vol, "material": material}


FLUID_E = 400.0  # pressure coefficient of the fluid scenes


def rest_state(dim, n):
    """v = 0, C = 0, F = I as float32 SoA arrays."""
    v = np.zeros((dim, n), dtype=np.float32)
    C = np.zeros((dim * dim, n), dtype=np.float32)
    F = np.zeros((dim * dim, n), dtype=np.float32)
    for a in range(dim):
        F[a * dim + a] = 1.0
    return v, C, F


# ---------------------------------------------------------------- c1
def c1(seed=0, n=8192):
    rng = np.random.default_rng(seed)
    x = (0.3 + 0.2 * rng.random((n, 2))).astype(np.float32).T.copy()
    v, C, F = rest_state(2, n)
    return {"name": "c1", "scheme": scheme_c1(2, False, seed),
            "params": params(2, 128, 1e-4, 0.04 / n),
            "steps": 50, "n": n, "state": (x, v, C, F)}


# ---------------------------------------------------------------- cube scenes
def _non_overlapping_corners(rng, count, side, lo, hi, gap, dim=3):
    corners = []
    tries = 0
    while len(corners) < count:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place cubes")
        c = lo + (hi - lo) * rng.random(dim)
        ok = True
        for d in corners:
            if np.all(np.abs(c - d) < side + gap):
                ok = False
                break
        if ok:
            corners.append(c)
    return np.array(corners)


def cube_particles(seed, index, corner, side, count, vel, dim=3):
    """Particles of one cube, uniform inside it, all with velocity `vel`."""
    rng = np.random.default_rng([seed, 1000 + index])
    x = (np.asarray(corner)[:, None] + side * rng.random((dim, count))).astype(np.float32)
    v = np.repeat(np.asarray(vel, dtype=np.float32)[:, None], count, axis=1)
    return x, v


def cubes_scene(name, seed, grid_res, corners, side, counts, vels, dt, steps, scheme,
                sort_every, dim=3):
    xs, vs = [], []
    for i in range(len(corners)):
        x, v = cube_particles(seed, i, corners[i], side, counts[i], vels[i], dim)
        xs.append(x)
        vs.append(v)
    x = np.concatenate(xs, axis=1)
    n = x.shape[1]
    _, C, F = rest_state(dim, n)
    v = np.concatenate(vs, axis=1)
    p_vol = side ** dim / counts[0]
    return {"name": name, "scheme": scheme, "steps": steps, "n": n,
            "params": params(dim, grid_res, dt, p_vol, sort_every=sort_every),
            "state": (x, v, C, F), "cubes": {"corners": np.asarray(corners), "side": side,
                                            "counts": list(counts), "vels": np.asarray(vels)}}


def c2(seed=0, cubes=4, per_cube=262144, grid_res=128, steps=100, sort_every=10):
    rng = np.random.default_rng(seed)
    side = 0.25
    corners = _non_overlapping_corners(rng, cubes, side, 0.1, 0.65, gap=0.06)
    vels = rng.uniform(-1.0, 1.0, (cubes, 3))
    sc = scheme_c1(3, True, seed)
    return cubes_scene("c2", seed, grid_res, corners, side, [per_cube] * cubes, vels,
                       2e-4, steps, sc, sort_every)


def c5(seed=0, grid_res=64, steps=64):
    """Adjoint scene (see module docstring); n = grid_res^3 particles."""
    rng = np.random.default_rng([seed, 5])
    side = 0.5
    n = grid_res ** 3
    corner = np.array([0.25, 0.25, 0.25])
    x = (corner[:, None] + side * rng.random((3, n))).astype(np.float32)
    drift = rng.uniform(-1.0, 1.0, 3)
    omega = rng.uniform(-2.0, 2.0, 3)
    r = x.astype(np.float64) - (corner + 0.5 * side)[:, None]
    spin = np.cross(omega[:, None], r, axis=0)
    v = (drift[:, None] + spin + rng.uniform(-0.1, 0.1, (3, n))).astype(np.float32)
    _, C, F = rest_state(3, n)
    sc = scheme_c1(3, True, seed)
    return {"name": "c5", "scheme": sc, "steps": steps, "n": n,
            "params": params(3, grid_res, 2e-4, side ** 3 / n, sort_every=0),
            "state": (x, v, C, F)}


def dam_break(dim=2, seed=0, grid_res=128, ppc=4, steps=100, dither=False, sort_every=10):
    """Fluid dam break (Sec. 8.1): a column of fluid at rest in the corner,
    [0.1, 0.4] x [0.1, 0.6] (x [0.3, 0.7] in z), ppc particles per cell,
    J = 1, pressure coefficient 400, dt = 1e-4 (2D) / 5e-5 (3D)."""
    rng = np.random.default_rng([seed, 7])
    lo = np.array([0.1, 0.1, 0.3])[:dim]
    hi = np.array([0.4, 0.6, 0.7])[:dim]
    cells = np.prod((hi - lo) * grid_res)
    n = int(round(cells * ppc))
    x = (lo[:, None] + (hi - lo)[:, None] * rng.random((dim, n))).astype(np.float32)
    v = np.zeros((dim, n), dtype=np.float32)
    C = np.zeros((dim * dim, n), dtype=np.float32)
    J = np.ones((1, n), dtype=np.float32)
    dt = 1e-4 if dim == 2 else 5e-5
    vol = float(np.prod(hi - lo))
    return {"name": f"dam{dim}d", "scheme": scheme_fluid(dim, dither, seed), "steps": steps, "n": n,
            "params": params(dim, grid_res, dt, vol / n, sort_every=sort_every, material="fluid", E=FLUID_E),
            "state": (x, v, C, J)}


def c4_scene(stream_seed, index, steps=100, n_max=2 ** 21, materialize=True):
    """Scene `index` of the serving stream (see module docstring).  With
    materialize=False the state is described by "x" (float32 [dim, n]) and
    "vel" (one velocity for every particle; C = 0, F = I) and "state" is
    None; c4_state() builds the arrays."""
    rng = np.random.default_rng([stream_seed, 4, index])
    dim = int(rng.choice([2, 3]))
    res = int(rng.choice([32, 64, 128, 256]))
    n = int(round(math.exp(rng.uniform(math.log(4096), math.log(n_max)))))
    side = 0.5
    corner = np.array([0.25, 0.35, 0.25])[:dim]
    x = rng.random((dim, n), dtype=np.float32)
    x *= np.float32(side)
    x += corner.astype(np.float32)[:, None]
    vel = rng.uniform(-1.0, 1.0, dim).astype(np.float32)
    mu = E_MODULUS / (2 * (1 + POISSON))
    la = E_MODULUS * POISSON / ((1 + POISSON) * (1 - 2 * POISSON))
    c = math.sqrt((la + 2 * mu) / DENSITY)
    dt = 0.25 / (res * c)
    scheme = random_scheme(rng, dim, seed=int(rng.integers(0, 2 ** 63)))
    sc = {"name": f"c4-{index}", "index": index, "scheme": scheme, "steps": steps, "n": n,
          "params": params(dim, res, dt, side ** dim / n), "x": x, "vel": vel, "state": None}
    if materialize:
        sc["state"] = c4_state(sc)
    return sc


def c4_state(sc):
    x = sc["x"]
    dim, n = x.shape
    v = np.repeat(sc["vel"][:, None], n, axis=1)
    _, C, F = rest_state(dim, n)
    return (x, v, C, F)


def c4_arrivals(stream_seed, count=256, rate=100.0):
    """Poisson arrival times (seconds) of the serving stream."""
    rng = np.random.default_rng([stream_seed, 44])
    return np.cumsum(rng.exponential(1.0 / rate, count))


C3_TOTAL = 300_000_000
C3_CUBES = 186


def c3_layout(seed=0, total=C3_TOTAL, cubes=C3_CUBES, grid_res=512, cube_cells=60, slot_cells=64):
    """Cube placement for c3 without generating particles."""
    rng = np.random.default_rng(seed)
    slots_per_axis = grid_res // slot_cells
    nslots = slots_per_axis ** 3
    chosen = np.sort(rng.choice(nslots, size=cubes, replace=False))
    dx = 1.0 / grid_res
    corners = []
    for s in chosen:
        sx, sy, sz = s % slots_per_axis, (s // slots_per_axis) % slots_per_axis, s // slots_per_axis ** 2
        off = (slot_cells - cube_cells) // 2
        corners.append([(sx * slot_cells + off) * dx, (sy * slot_cells + off) * dx,
                        (sz * slot_cells + off) * dx])
    counts = [total // cubes + (1 if i < total % cubes else 0) for i in range(cubes)]
    vels = rng.uniform(-1.0, 1.0, (cubes, 3))
    side = cube_cells * dx
    return {"corners": np.asarray(corners), "side": side, "counts": counts, "vels": vels,
            "slots": chosen}


C3_YOUNG = 100.0  # config 3 names no material; see c3_params


def c3_params(seed=0, total=C3_TOTAL, cubes=C3_CUBES):
    """512^3 grid, dt = 1e-4.  The workload names no material: with the
    E = 1e3 of c1 the P-wave CFL number c dt / dx is 1.7 at dx = 1/512 and
    the explicit substep diverges (the FP64 oracle saturates C within six
    substeps); E = 100 (rho = 1, nu = 0.2) gives 0.54."""
    lay = c3_layout(seed, total, cubes)
    p_vol = lay["side"] ** 3 / lay["counts"][0]
    p = params(3, 512, 1e-4, p_vol, sort_every=0)
    p["E"] = C3_YOUNG
    return p


def c3(seed=0, total=C3_TOTAL, cubes=C3_CUBES, only=None):
    """c3 scene; `only` restricts the particles to a list of cube indices
    (the scene parameters, including particle volume, stay those of the full
    scene)."""
    lay = c3_layout(seed, total, cubes)
    idx = range(cubes) if only is None else only
    xs, vs = [], []
    for i in idx:
        x, v = cube_particles(seed, i, lay["corners"][i], lay["side"], lay["counts"][i], lay["vels"][i])
        xs.append(x)
        vs.append(v)
    x = np.concatenate(xs, axis=1)
    v = np.concatenate(vs, axis=1)
    n = x.shape[1]
    _, C, F = rest_state(3, n)
    return {"name": "c3", "scheme": scheme_c3(seed), "steps": 10, "n": n,
            "params": c3_params(seed, total, cubes), "state": (x, v, C, F), "cubes": lay}


def with_scheme(scene, scheme):
    s = copy.copy(scene)
    s["scheme"] = scheme
    return s


def random_state(rng, dim, n, x_lo=0.2, x_hi=0.8, v_scale=1.0, c_scale=5.0, f_scale=0.05):
    """Generic random particle state (float32 SoA) for codec and transfer tests."""
    x = rng.uniform(x_lo, x_hi, (dim, n)).astype(np.float32)
    v = (v_scale * rng.standard_normal((dim, n))).astype(np.float32)
    C = (c_scale * rng.standard_normal((dim * dim, n))).astype(np.float32)
    F = (f_scale * rng.standard_normal((dim * dim, n))).astype(np.float32)
    for a in range(dim):
        F[a * dim + a] += 1.0
    return x, v, C, F


def bounce_block(seed=0, dither=True, n=4096, steps=400):
    """2D elastic block [0.3, 0.5] x [0.04, 0.24] thrown at the floor with
    v = (0, -2): it hits the wall band at once and rings, so every field
    keeps changing by amounts comparable to its quantization step.  Coarse
    scheme (the regime of the paper's dithering study, Sec. 8.1): x 16-bit,
    v 10-bit in [-20, 20], C 10-bit in [-200, 200], F 10-bit (F - I in
    [-1, 1]); 128^2 grid, dt = 1e-4, sorted every 10 steps."""
    rng = np.random.default_rng(seed)
    x = np.stack([0.3 + 0.2 * rng.random(n), 0.04 + 0.2 * rng.random(n)]).astype(np.float32)
    v, C, F = rest_state(2, n)
    v[1] = -2.0
    sch = {"dim": 2, "seed": seed, "fields": [
        fixed("x", 16, 0.0, 1.0, dither), fixed("v", 10, -20.0, 20.0, dither),
        fixed("C", 10, -200.0, 200.0, dither), fixed("F", 10, -1.0, 1.0, dither, rel_identity=True)]}
    return {"name": "bounce", "scheme": sch, "steps": steps, "n": n,
            "params": params(2, 128, 1e-4, 0.04 / n, sort_every=10), "state": (x, v, C, F)}


def inverted_scene(dim, seed=0, n=3000, grid_res=32, frac=0.4):
    """Elastic particles with random deformation gradients of which about
    `frac` are inverted (det F < 0) or flattened (one singular value near
    zero): F = Q diag(s) P^T with random rotations Q, P and singular values
    in [0.6, 1.4], the last one negated (inverted) or set to 1e-4
    (flattened).  Particles uniform in [0.3, 0.7]^dim, velocities U(-0.5,
    0.5), C = 0, raw float32 layout (so the initial encode is exact)."""
    rng = np.random.default_rng([seed, 9])
    x = rng.uniform(0.3, 0.7, (dim, n)).astype(np.float32)
    v = rng.uniform(-0.5, 0.5, (dim, n)).astype(np.float32)
    C = np.zeros((dim * dim, n), dtype=np.float32)

    def rotation():
        q, r = np.linalg.qr(rng.standard_normal((dim, dim)))
        q = q * np.sign(np.diag(r))[None, :]
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        return q

    F = np.empty((dim * dim, n), dtype=np.float32)
    kind = rng.random(n)
    for p in range(n):
        s = rng.uniform(0.6, 1.4, dim)
        if kind[p] < frac * 0.75:
            s[-1] = -s[-1]
        elif kind[p] < frac:
            s[-1] = 1e-4
        F[:, p] = (rotation() @ np.diag(s) @ rotation().T).reshape(-1)
    return {"name": f"inverted{dim}d", "scheme": scheme_fp32(dim, seed), "steps": 1, "n": n,
            "params": params(dim, grid_res, 1e-4, 0.4 ** dim / n), "state": (x, v, C, F)}


def random_scheme(rng, dim, seed=0):
    """A random valid scheme: 12-24 bits per field, random dither and kinds."""
    fields = []
    order = list(rng.permutation(["x", "v", "C", "F"]))
    for name in order:
        bits = int(rng.integers(12, 25))
        dither = bool(rng.integers(0, 2))
        kind = rng.choice(["fixed", "fixed", "shared_exp"]) if name in ("v", "C") else "fixed"
        if name == "x":
            fields.append(fixed("x", max(bits, 16), 0.0, 1.0, dither))
        elif name == "F":
            fields.append(fixed("F", bits, -1.0, 1.0, dither, rel_identity=True))
        elif kind == "shared_exp":
            fields.append(shared_exp(name, bits, int(rng.integers(4, 7)), 20.0 if name == "v" else 50.0, dither))
        else:
            hi = 20.0 if name == "v" else 50.0
            fields.append(fixed(name, bits, -hi, hi, dither))
    return {"dim": dim, "seed": seed, "fields": fields}
