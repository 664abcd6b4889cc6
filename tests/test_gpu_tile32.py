"""The scheme-specialized fused kernel's 32-bit P2G node tile at its limits.
A work item's node sums are 32-bit integers at a scale chosen from the
item's particle count (a node's weight sum stays below N_item * 0.75^3) and
from its record of the previous substep; a particle whose node values lie
too far from the item's reference velocity goes through the exact 64-bit
global path instead (mpmq_stats_t.wide).

  - a dense clump: 4096 particles inside one grid cell, so that every
    work item's node weight sums come close to the bound the scale is
    chosen for, with random velocities;
  - a fast cube hitting the floor's wall band: the wall rule stops the
    particles that reach it, so their velocities leave their items'
    records and must take the global path.

Both runs are compared with the oracle at the bars of the other trajectory
tests, and with the generic kernels (exact 64-bit tile), which must be no
closer to the oracle (gpu_common.lsb_differences)."""
import numpy as np
import pytest

import workloads as WL
from gpu_common import gpu_context, lsb_differences, note, oracle_sim

pytestmark = pytest.mark.gpu


def _check(tag, dx, lsb):
    print(f"[{tag}] x max {np.max(dx):.2e}; " + "; ".join(
        f"{f}: <=1 {np.mean(d <= 1 + 1e-9):.5f} max {np.max(d):.1f}" for f, d in lsb.items() if f != "x"), flush=True)
    assert np.max(dx) <= 1e-4, (tag, np.max(dx))
    for f, d in lsb.items():
        if f != "x":
            assert np.mean(d <= 1.0 + 1e-9) >= 0.99, (tag, f)
            assert np.max(d) <= 8.0, (tag, f, np.max(d))


def _run(gpu_lib, orc, sc, steps):
    spe = gpu_context(gpu_lib, sc)
    spe.specialize(True)
    gen = gpu_context(gpu_lib, sc)
    sim, _, _ = oracle_sim(orc, sc)
    for c in (spe, gen, sim):
        c.step(steps)
    ow, oi = sim.words(), sim.ids()
    ds = lsb_differences(orc, sc["scheme"], spe.words(), spe.ids(), ow, oi, sc["params"], steps)
    dg = lsb_differences(orc, sc["scheme"], gen.words(), gen.ids(), ow, oi, sc["params"], steps)
    st = spe.stats()
    sim.close()
    spe.close()
    gen.close()
    return ds, dg, st


def test_dense_clump(gpu_lib, orc):
    rng = np.random.default_rng(31)
    n, res = 4096, 32
    dx = 1.0 / res
    x = (0.5 + dx * rng.random((3, n))).astype(np.float32)  # one cell
    v = rng.uniform(-1.0, 1.0, (3, n)).astype(np.float32)
    _, C, F = WL.rest_state(3, n)
    sc = {"scheme": WL.scheme_c1(3, True, 31), "params": WL.params(3, res, 1e-4, dx ** 3 / n, E=100.0),
          "state": (x, v, C, F), "n": n}
    note("tile32 dense clump")
    (dxs, ls), (dxg, lg), st = _run(gpu_lib, orc, sc, 6)
    _check("clump specialized", dxs, ls)
    _check("clump generic", dxg, lg)
    assert st["clamped"] == 0 and st["fallback"] == 0, st


def test_wall_impact_takes_the_wide_path(gpu_lib, orc):
    sc = WL.cubes_scene("impact", 32, 32, [[0.4, 0.1, 0.4]], 0.2, [20000], [[0.0, -15.0, 0.0]], 1e-4, 8,
                        WL.scheme_c1(3, True, 32), 0)
    sc["params"]["E"] = 100.0
    note("tile32 wall impact")
    (dxs, ls), (dxg, lg), st = _run(gpu_lib, orc, sc, 8)
    _check("impact specialized", dxs, ls)
    _check("impact generic", dxg, lg)
    assert st["wide"] > 0, st  # the stopped particles left their items' range
    assert st["clamped"] == 0, st
