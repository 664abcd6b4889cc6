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
