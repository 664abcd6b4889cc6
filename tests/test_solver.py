"""mpmq_solve_scheme (host code of the C-ABI library) against the oracle
solver on random instances, and its input checks."""
import math

import numpy as np
import pytest

from oracle import solver as S


@pytest.fixture(scope="module")
def mq():
    import paper_2207_04658_amd as m
    m.load()
    return m


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("mode", ["error", "memory"])
def test_solver_matches_oracle(mq, seed, mode):
    rng = np.random.default_rng(seed)
    H = int(rng.integers(1, 9))
    P = list(rng.integers(1, 50, H).astype(float) * 512.0)
    g = list(10.0 ** rng.uniform(-10, 1, H))
    if H > 2:
        g[int(rng.integers(0, H))] = 0.0
    R = list(10.0 ** rng.uniform(-2, 2, H))
    if mode == "error":
        z, eps = float(rng.uniform(0.1, 10.0)), float(10.0 ** rng.uniform(-4, -1))
        d, b, bits = S.error_bounded(P, g, R, z, eps, 2, 30)
        got = mq.solve_scheme(P, g, R, "error", eps, z, 2, 30)
    else:
        eps = float(rng.uniform(0.2, 0.8))
        d, b, bits = S.memory_bounded(P, g, R, eps, 2, 30)
        got = mq.solve_scheme(P, g, R, "memory", eps, 0.0, 2, 30)
    assert got["bits"] == bits
    for h in range(H):
        if math.isinf(d[h]):
            assert math.isinf(got["delta"][h])
        else:
            assert math.isclose(got["delta"][h], d[h], rel_tol=1e-12)
            assert math.isclose(got["b_cont"][h], b[h], rel_tol=1e-12, abs_tol=1e-12)
    assert math.isclose(got["expected_error"], S.expected_error(g, R, bits), rel_tol=1e-12)
    assert got["total_bits"] == sum(p * x for p, x in zip(P, bits))


@pytest.mark.parametrize("bad", [
    dict(P=[0.0]), dict(R=[-1.0]), dict(g=[float("nan")]), dict(eps=0.0), dict(z=0.0),
    dict(min_bits=0), dict(max_bits=33), dict(P=[1.0] * 17, g=[1.0] * 17, R=[1.0] * 17)])
def test_solver_rejects_invalid_input(mq, bad):
    args = dict(P=[100.0], g=[1e-3], R=[1.0], mode="error", eps=1e-3, z=1.0, min_bits=1, max_bits=32)
    args.update(bad)
    with pytest.raises(mq.MpmqError):
        mq.solve_scheme(**args)
