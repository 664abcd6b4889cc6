"""The allocation-free adjoint (mpmq_adjoint_static, workspace in the
library's static device array) against mpmq_adjoint with a caller-owned
workspace, on two calls in a row, the second with a smaller scene and a
shorter horizon, plus the size limit.

Bars: the forward trajectory is bit-reproducible, so the final packed words
and the value ranges (integer min / max) are equal exactly; z is a sum of
binary64 atomics (1e-12 relative); G, g and lambda_0 go through float
atomics whose order varies between runs, so they are compared at the 1e-4
relative agreement the checkpoint modes are held to."""
import math

import numpy as np
import pytest

import workloads as WL
from gpu_common import gpu_context, note

pytestmark = pytest.mark.gpu

FIELDS = "xvCF"


def _run_pair(mq, scene, steps, K, objective):
    import torch
    a = gpu_context(mq, scene)
    b = gpu_context(mq, scene)
    rows = 2 * a.dim + a.dim * a.dim + a.nc3
    lam = torch.empty((rows, a.n), dtype=torch.float32, device=a.device)
    ra = a.adjoint_static(steps, objective=objective, axis=1, checkpoint_every=K, lambda0=lam)
    rb = b.adjoint(steps, objective=objective, axis=1, checkpoint_every=K, want_lambda0=True)
    assert np.array_equal(a.words(), b.words())
    assert a.step_count() == b.step_count() == steps
    la, lb = lam.cpu().numpy().astype(np.float64), rb["lambda0"].cpu().numpy().astype(np.float64)
    a.close()
    b.close()
    assert math.isclose(ra["z"], rb["z"], rel_tol=1e-12, abs_tol=1e-300)
    assert ra["recomputed"] == rb["recomputed"] and ra["states"] == rb["states"]
    for f in FIELDS:
        assert ra["lo"][f] == rb["lo"][f] and ra["hi"][f] == rb["hi"][f], f
        assert math.isclose(ra["G"][f], rb["G"][f], rel_tol=1e-4, abs_tol=1e-4 * max(abs(rb["G"][k]) for k in FIELDS)), f
        assert math.isclose(ra["g"][f], rb["g"][f], rel_tol=1e-4, abs_tol=1e-8 * max(rb["g"][k] for k in FIELDS)), f
    assert np.max(np.abs(la - lb)) <= 1e-4 * np.max(np.abs(lb))
    return ra


def test_static_adjoint_two_calls(gpu_lib):
    note("adjoint_static: 16^3 scene (4096 particles) T=8 K=4, then 12^3 (1728) T=3 K=0")
    big = WL.c5(seed=3, grid_res=16)
    small = WL.c5(seed=4, grid_res=12)
    assert small["n"] < big["n"]
    _run_pair(gpu_lib, big, 8, 4, "ke")
    _run_pair(gpu_lib, small, 3, 0, "com")


def test_static_adjoint_size_limit(gpu_lib):
    note("adjoint_static: workspace above the static limit is refused")
    scene = WL.c5(seed=3, grid_res=16)
    ctx = gpu_context(gpu_lib, scene)
    need = ctx.adjoint_workspace_bytes(1000, checkpoint_every=1000)
    assert need > gpu_lib.STATIC_WORKSPACE_BYTES
    with pytest.raises(gpu_lib.MpmqError) as e:
        ctx.adjoint_static(1000, checkpoint_every=1000)
    assert e.value.status == -2 and "static workspace" in str(e.value)
    assert ctx.step_count() == 0
    ctx.close()
