"""Scheme-specialized kernels (mpmq_specialize), compiled at run time with
the scheme as constants.  Their fused substep sums P2G in the 32-bit node
tile at per-item scales, the generic kernels in the exact 64-bit tile, so:
  - with a sort before every substep (every P2G is the exact bootstrap
    P2G, the fused kernel scatters nothing) the two builds give the same
    packed words, ids and statistics bit for bit: decode, G2P, update and
    the dithered encode are the same arithmetic;
  - in ordinary runs the specialized build is no further from the oracle
    than the generic one: the 32-bit tile's roundings are of the order of
    the float32 noise that both builds carry in their node velocities."""
import numpy as np
import pytest

import workloads as WL
from gpu_common import gpu_context, lsb_differences, note, oracle_sim

pytestmark = pytest.mark.gpu


def scenes():
    out = {}
    c1 = WL.c1(seed=2, n=3000)
    c1["params"]["sort_every"] = 4
    out["c1_2d"] = c1
    c5 = WL.c5(seed=3, grid_res=16)
    c5["params"]["sort_every"] = 5
    out["c2scheme_3d_dither"] = c5
    out["c3scheme_3d"] = WL.with_scheme(c5, WL.scheme_c3(4))
    out["fp32_3d"] = WL.with_scheme(c5, WL.scheme_fp32(3, 1))
    out["random_2d"] = WL.with_scheme(c1, WL.random_scheme(np.random.default_rng(11), 2, seed=5))
    out["random_3d"] = WL.with_scheme(c5, WL.random_scheme(np.random.default_rng(12), 3, seed=6))
    return out


SCENES = scenes()


def _no_worse(tag, spe, gen):
    """The specialized build is no further from the oracle than the generic
    one (each a (x difference, {field: unit differences}) pair from
    lsb_differences against the same oracle run)."""
    (dxs, ls), (dxg, lg) = spe, gen
    assert np.max(dxs) <= max(1e-4, 2.0 * np.max(dxg)), (tag, np.max(dxs), np.max(dxg))
    for f in ls:
        if f == "x":
            continue
        fs, fg = np.mean(ls[f] <= 1.0 + 1e-9), np.mean(lg[f] <= 1.0 + 1e-9)
        assert fs >= fg - 0.02, (tag, f, fs, fg)
        assert np.max(ls[f]) <= np.max(lg[f]) + max(2.0, 0.25 * np.max(lg[f])), (tag, f, np.max(ls[f]), np.max(lg[f]))


@pytest.mark.parametrize("name", list(SCENES))
def test_specialized_equals_generic_exact_p2g(gpu_lib, name):
    note(f"specialized vs generic, sort every substep: {name}")
    sc = dict(SCENES[name], params=dict(SCENES[name]["params"], sort_every=1))
    gen = gpu_context(gpu_lib, sc)
    spe = gpu_context(gpu_lib, sc)
    spe.specialize(True)
    gen.set_stats(1)
    spe.set_stats(1)
    for k in (3, 4):
        gen.step(k)
        spe.step(k)
        assert np.array_equal(gen.words(), spe.words()), f"{name}: words differ after a chunk of {k}"
    assert np.array_equal(gen.ids(), spe.ids())
    sg, ss = gen.stats(), spe.stats()
    for f in "xvCF":
        assert sg[f] == ss[f], f
    assert sg["fallback"] == ss["fallback"] and sg["active_nodes"] == ss["active_nodes"]
    assert sg["wide"] == ss["wide"] == 0
    gen.close()
    spe.close()


@pytest.mark.parametrize("name", list(SCENES))
def test_specialized_vs_generic(gpu_lib, orc, name):
    """Ordinary runs: both builds against the oracle on the same scene (the
    schemes here include 24-bit velocities without dither, whose float32
    noise the oracle comparisons' bars do not cover after a few substeps:
    the check is that the 32-bit tile adds nothing measurable to it)."""
    note(f"specialized vs generic: {name}")
    sc = SCENES[name]
    gen = gpu_context(gpu_lib, sc)
    spe = gpu_context(gpu_lib, sc)
    spe.specialize(True)
    sim, _, _ = oracle_sim(orc, sc)
    t = 0

    def check(tag):
        ow, oi = sim.words(), sim.ids()
        _no_worse(tag, lsb_differences(orc, sc["scheme"], spe.words(), spe.ids(), ow, oi, sc["params"], t),
                  lsb_differences(orc, sc["scheme"], gen.words(), gen.ids(), ow, oi, sc["params"], t))

    for k in (3, 4, 6):
        gen.step(k)
        spe.step(k)
        sim.step(k)
        t += k
        check(f"{name} step {t}")
    sg, ss = gen.stats(), spe.stats()
    assert sg["steps"] == ss["steps"] and sg["sorts"] == ss["sorts"]
    assert ss["clamped"] == sg["clamped"] == 0
    # back to the generic kernels mid-run, and to the specialized ones again
    spe.specialize(False)
    for c in (gen, spe, sim):
        c.step(2)
    spe.specialize(True)
    for c in (gen, spe, sim):
        c.step(2)
    t += 4
    check(f"{name} after switching")
    sim.close()
    gen.close()
    spe.close()
