"""GPU parity at the workloads' own horizons, on every field of the state,
for both the generic kernels and the scheme-specialized ones that the
benchmark times.

GPU and oracle run the same sub-scene from the same packed words, so every
particle occupies the same slot on both sides and draws the same dither
stream:
  - one cube of the 2^20-particle workload (262,144 particles) on its 128^3
    grid, sorted every 10 substeps, compared after 50 and 100 substeps;
  - cube 0 of the 3e8-particle workload (1,612,904 particles, next to the
    z = 0 wall band) on the 512^3 grid with its 2 x 4.3 GB grid buffers and
    its scheme (shared-exponent v and C), compared after 10 substeps.

Bars.  x: within 1e-4 of the unit domain (the metric's tolerance).  v, C, F:
compared per component in units of the quantization step of the stored
value (the larger of the two sides' steps for a shared exponent), or of the
change that a one-code flip of v induces (gpu_common.comparison_units)
where that is larger: a store whose unquantized value lies within FP32
error of a rounding boundary may round the other way on the GPU, and a
one-code change of v moves C' of the particles around it by up to
(4 / dx) Delta_v, which is hundreds of codes of a 16-bit C, and F
integrates dt C' F over the substeps.  Such flips
perturb the grid momenta around them, so later flips cluster near earlier
ones.  The bars: at least 99 % of components within one unit, and no
component more than 8 units apart.
"""
import numpy as np
import pytest

import workloads as WL
from gpu_common import gpu_context, lsb_differences, note

pytestmark = pytest.mark.gpu


def _report(tag, dx, lsb):
    parts = [f"x max {np.max(dx):.2e}"]
    for f, d in lsb.items():
        if f == "x":
            continue
        parts.append(f"{f}: eq {np.mean(d == 0):.4f} <=1 {np.mean(d <= 1.0 + 1e-9):.5f} max {np.max(d):.1f}")
    print(f"[{tag}] " + "; ".join(parts), flush=True)


def _check(tag, dx, lsb):
    _report(tag, dx, lsb)
    assert np.max(dx) <= 1e-4, (tag, np.max(dx))
    for f, d in lsb.items():
        if f == "x":
            continue
        assert np.mean(d <= 1.0 + 1e-9) >= 0.99, (tag, f, np.mean(d <= 1.0 + 1e-9))
        assert np.max(d) <= 8.0, (tag, f, np.max(d))


@pytest.fixture(scope="module")
def c2_cube_oracle(orc):
    """Oracle run of one cube at the 2^20-particle workload's settings:
    words and ids after 50 and 100 substeps."""
    sc = WL.c2(cubes=1)
    note(f"oracle: c2 one cube n={sc['n']} 100 steps")
    w0, _ = orc.encode(sc["scheme"], *sc["state"], 0, 2)
    sim = orc.Sim(sc["scheme"], sc["params"], w0)
    out = {}
    for t in (50, 100):
        sim.step(t - sim.step_count)
        out[t] = (sim.words(), sim.ids(), sim.stats())
    sim.close()
    return sc, w0, out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("specialized", [False, True])
def test_c2_cube_100_steps(gpu_lib, orc, c2_cube_oracle, specialized):
    sc, w0, ref = c2_cube_oracle
    note(f"c2 one cube n={sc['n']} 100 steps specialized={specialized}")
    ctx = gpu_context(gpu_lib, sc)
    if specialized:
        ctx.specialize(True)
    assert np.array_equal(ctx.words(), w0)
    for t in (50, 100):
        ctx.step(t - ctx.step_count())
        ow, oids, ost = ref[t]
        dx, lsb = lsb_differences(orc, sc["scheme"], ctx.words(), ctx.ids(), ow, oids, sc["params"], t)
        _check(f"c2 cube step {t} spec={specialized}", dx, lsb)
    st = ctx.stats()
    assert st["sorts"] == 10 and st["clamped"] == 0
    assert all(st[f]["sat"] == 0 and st[f]["nan"] == 0 for f in "xvCF")
    ctx.close()


@pytest.fixture(scope="module")
def c3_cube_oracle(orc):
    sc = WL.c3(only=[0])
    note(f"oracle: c3 cube 0 n={sc['n']} 10 steps on 512^3")
    w0, _ = orc.encode(sc["scheme"], *sc["state"], 0, 2)
    sim = orc.Sim(sc["scheme"], sc["params"], w0)
    sim.step(10)
    out = (sim.words(), sim.ids(), sim.stats())
    sim.close()
    return sc, w0, out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("specialized", [False, True])
def test_c3_cube_10_steps(gpu_lib, orc, c3_cube_oracle, specialized):
    sc, w0, (ow, oids, ost) = c3_cube_oracle
    note(f"c3 cube 0 n={sc['n']} 10 steps on 512^3 specialized={specialized}")
    ctx = gpu_context(gpu_lib, sc)
    if specialized:
        ctx.specialize(True)
    assert np.array_equal(ctx.words(), w0)
    ctx.step(10)
    dx, lsb = lsb_differences(orc, sc["scheme"], ctx.words(), ctx.ids(), ow, oids, sc["params"], 10)
    _check(f"c3 cube 0 step 10 spec={specialized}", dx, lsb)
    st = ctx.stats()
    assert st["clamped"] == 0 and all(st[f]["nan"] == 0 for f in "xvCF")
    for f in "xvCF":
        assert abs(st[f]["sat"] - ost[f]["sat"]) <= max(2, 0.01 * ost[f]["sat"]), (f, st[f]["sat"], ost[f]["sat"])
    ctx.close()


@pytest.mark.parametrize("specialized", [False, True])
def test_sparse_scene(gpu_lib, orc, specialized):
    """A sparse scene: 3000 particles in a cube of half the domain on a 128^3
    grid (about 0.01 per cell), so every work item holds a few particles and
    skips the node tiles (G2P and P2G straight through the grid buffers).
    Compared with the oracle after 20 dithered substeps at the bars above;
    the tile-less items are not counted as fallback stencils.

    Young's modulus 100 instead of 1000: a particle with no neighbour in its
    stencil is an explicit oscillator of its own, C' = C - 4 dt / (rho dx^2)
    tau(F), F' = (I + dt C') F, whose volumetric mode has
    (omega dt)^2 = 4 dt^2 (2 mu + 3 lambda) / (rho dx^2); that is 4.4 at
    E = 1000 (above 4: the mode grows and C saturates within ten substeps,
    on either side, so rounding differences are amplified) and 0.44 at
    E = 100."""
    sc = WL.cubes_scene("sparse", 11, 128, [[0.25, 0.25, 0.25]], 0.5, [3000], [[0.4, -0.7, 0.2]],
                        2e-4, 20, WL.scheme_c1(3, True, 11), 5)
    sc["params"]["E"] = 100.0
    note(f"sparse scene n={sc['n']} on 128^3, 20 steps, specialized={specialized}")
    ctx = gpu_context(gpu_lib, sc)
    if specialized:
        ctx.specialize(True)
    ctx.step(20)
    w0, _ = orc.encode(sc["scheme"], *sc["state"], 0, 2)
    sim = orc.Sim(sc["scheme"], sc["params"], w0)
    sim.step(20)
    dx, lsb = lsb_differences(orc, sc["scheme"], ctx.words(), ctx.ids(), sim.words(), sim.ids(), sc["params"], 20)
    sim.close()
    _check(f"sparse spec={specialized}", dx, lsb)
    st = ctx.stats()
    assert st["fallback"] == 0 and st["clamped"] == 0 and st["atomics"] == 0, st
    ctx.close()
