"""Inverted and flattened elements: the fixed-corotated rotation of an F with
det F <= 0 is the proper rotation closest to F (the reflection is carried by
the direction of the smallest singular value), on the GPU as in the oracle.

One substep from the same float32 state in the raw float32 layout (the
encode is exact, so both sides start from identical values and only FP32
against FP64 arithmetic differs), compared field by field, then lambda_0 of
the one-step adjoint, whose stress VJP depends on the same rotation.  About
30 % of the particles are inverted and 10 % flattened (one singular value
1e-4): with an improper rotation for those, their stresses differ from the
oracle's by the size of the stress itself.
"""
import numpy as np
import pytest

import workloads as WL
from gpu_common import by_id, gpu_context, gpu_decode_np, note, oracle_sim

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim", [2, 3])
def test_inverted_one_step(gpu_lib, orc, dim):
    sc = WL.inverted_scene(dim, seed=dim)
    note(f"inverted elements dim={dim} n={sc['n']}")
    ctx = gpu_context(gpu_lib, sc)
    sim, ow0, _ = oracle_sim(orc, sc)
    assert np.array_equal(ctx.words(), ow0)
    ctx.step(1)
    sim.step(1)
    g = [by_id(a, ctx.ids()) for a in gpu_decode_np(ctx)]
    o = [by_id(a, sim.ids()) for a in orc.decode(sc["scheme"], sim.words())]
    # float32 state after one substep: x' = x + dt v' is formed from float32
    # v' (relative error ~1e-6 of |v'| <= ~10, times dt = 1e-4); v, C, F are
    # float32 results of sums whose terms reach the stress magnitude, so they
    # are compared to 1e-4 of each field's largest value
    assert np.max(np.abs(g[0] - o[0])) <= 1e-7, np.max(np.abs(g[0] - o[0]))
    for name, a, b in zip("vCF", g[1:], o[1:]):
        err = np.max(np.abs(a - b))
        top = np.max(np.abs(b))
        print(f"dim {dim} field {name}: max err {err:.3e} of max {top:.3e}")
        assert err <= 1e-4 * top, (name, err, top)
    ctx.close()
    sim.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_inverted_adjoint_lambda0(gpu_lib, orc, dim):
    from test_gpu_adjoint import assert_weighted_close, field_steps, oracle_trajectory, split_lambda
    sc = WL.inverted_scene(dim, seed=10 + dim)
    note(f"inverted elements adjoint dim={dim} n={sc['n']}")
    ctx = gpu_context(gpu_lib, sc)
    res = ctx.adjoint(1, objective="ke", checkpoint_every=1, want_lambda0=True)
    lg = res["lambda0"].cpu().numpy().astype(np.float64)
    states = oracle_trajectory(orc, sc, 1)
    z, G, g, A, lo = orc.adjoint_full(sc["params"], states, "ke", 1)
    # raw float32 fields: every field is weighted alike (step 2^-23), so
    # lambda_0 is compared to 1e-2 of its largest component (the kinetic
    # energy objective's lambda_1 depends on the FP32 velocities)
    assert_weighted_close(split_lambda(lg, dim), split_lambda(lo, dim), field_steps(sc["scheme"]), 1e-2, "lambda_0")
    assert abs(res["z"] - z) <= 1e-3 * abs(z)
    ctx.close()
