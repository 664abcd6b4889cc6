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


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mode", ["error", "memory"])
def test_auto_scheme_matches_oracle(mq, seed, mode):
    """mpmq_auto_scheme (Alg. 1 from a recorded run) against the oracle's
    widen_range + solver on the same record; placement order, dither and
    REL_IDENTITY follow the base scheme."""
    import workloads as WL
    rng = np.random.default_rng(100 + seed)
    dim = 2 + seed % 2
    base = WL.random_scheme(rng, dim, seed=seed)
    if seed % 3 == 0:
        base = WL.scheme_fluid(dim, True, seed)
    names = ["x", "v", "C", "J" if any(f["field"] == "J" for f in base["fields"]) else "F"]
    ncomp = {"x": dim, "v": dim, "C": dim * dim, "F": dim * dim, "J": 1}
    lo = {f: float(rng.uniform(-5, 0)) for f in names}
    hi = {f: lo[f] + float(rng.uniform(0, 5)) for f in names}
    hi[names[1]] = lo[names[1]]  # a zero-width record
    rec = {"z": float(rng.uniform(0.5, 2.0)), "g": {f: float(10.0 ** rng.uniform(-8, 0)) for f in names},
           "lo": lo, "hi": hi}
    n = int(rng.integers(100, 100000))
    factor = 2.0
    eps = 1e-3 if mode == "error" else 0.5
    scheme, sol = mq.auto_scheme(base, rec, n, mode=mode, eps=eps, range_factor=factor, min_bits=2, max_bits=30)
    wl, wh = [], []
    for f in names:
        a, b = S.widen_range(lo[f], hi[f], factor)
        mid = 0.5 * (lo[f] + hi[f])
        floor_half = 2.0 ** -20 * max(1.0, abs(mid))  # the C call's minimum half-width
        if 0.5 * (b - a) < floor_half:
            a, b = mid - floor_half, mid + floor_half
        wl.append(a)
        wh.append(b)
    P = [float(n * ncomp[f]) for f in names]
    g = [rec["g"][f] for f in names]
    R = [b - a for a, b in zip(wl, wh)]
    if mode == "error":
        d, b, bits = S.error_bounded(P, g, R, rec["z"], eps, 2, 30)
    else:
        d, b, bits = S.memory_bounded(P, g, R, eps, 2, 30)
    assert sol["bits"] == bits
    by_name = {f["field"]: f for f in scheme["fields"]}
    assert [f["field"] for f in scheme["fields"]] == [f["field"] for f in base["fields"]]
    for i, f in enumerate(names):
        got = by_name[f]
        ref = next(x for x in base["fields"] if x["field"] == f)
        assert got["kind"] == "fixed" and got["bits"] == bits[i]
        assert got["dither"] == bool(ref.get("dither", False))
        assert got["rel_identity"] == bool(ref.get("rel_identity", False))
        assert got["lo"] == wl[i] and got["hi"] == wh[i]
    assert math.isclose(sol["expected_error"], S.expected_error(g, R, bits), rel_tol=1e-12)


def test_auto_scheme_rejects_invalid(mq):
    import workloads as WL
    base = WL.scheme_c1(3, True, 0)
    rec = {"z": 1.0, "g": {f: 1e-3 for f in "xvCF"}, "lo": {f: 0.0 for f in "xvCF"}, "hi": {f: 1.0 for f in "xvCF"}}
    with pytest.raises(mq.MpmqError):
        mq.auto_scheme(base, rec, 0)
    with pytest.raises(mq.MpmqError):
        mq.auto_scheme(base, rec, 100, range_factor=0.5)
    bad = dict(rec, lo=dict(rec["lo"], v=2.0))
    with pytest.raises(mq.MpmqError):
        mq.auto_scheme(base, bad, 100)
