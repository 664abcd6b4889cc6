"""Scheme-specialized kernels (mpmq_specialize): the fused substep and the
bootstrap P2G compiled at run time with the scheme as constants give the same
packed words, ids and statistics as the generic kernels, bit for bit."""
import numpy as np
import pytest

import workloads as WL
from gpu_common import gpu_context, note

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


@pytest.mark.parametrize("name", list(SCENES))
def test_specialized_equals_generic(gpu_lib, name):
    note(f"specialized vs generic: {name}")
    sc = SCENES[name]
    gen = gpu_context(gpu_lib, sc)
    spe = gpu_context(gpu_lib, sc)
    spe.specialize(True)
    gen.set_stats(1)
    spe.set_stats(1)
    for k in (3, 4, 6):
        gen.step(k)
        spe.step(k)
        assert np.array_equal(gen.words(), spe.words()), f"{name}: words differ after a chunk of {k}"
    assert np.array_equal(gen.ids(), spe.ids())
    sg, ss = gen.stats(), spe.stats()
    for f in "xvCF":
        assert sg[f] == ss[f], f
    assert sg["fallback"] == ss["fallback"] and sg["active_nodes"] == ss["active_nodes"]
    # back to the generic kernels mid-run
    spe.specialize(False)
    gen.step(2)
    spe.step(2)
    assert np.array_equal(gen.words(), spe.words())
    gen.close()
    spe.close()
