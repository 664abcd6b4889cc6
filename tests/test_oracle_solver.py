"""Pins of the oracle quantization solver (Sec. 4, Eqs. 6-10, Alg. 1).

The closed forms are checked against facts that do not come from them:
the constraint each optimum must meet with equality, a general-purpose
constrained optimizer (scipy SLSQP) on the same continuous problems, single
type special cases that reduce to one line of algebra, and invariances of the
problem (scaling of g)."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import solver as S


def instance(rng, H):
    P = rng.integers(1, 10, H).astype(float) * 1000.0
    g = 10.0 ** rng.uniform(-8, 0, H)
    R = 10.0 ** rng.uniform(-1, 2, H)
    return list(P), list(g), list(R)


def cont_error(g, R, b):
    return sum(gh * (r * 2.0 ** -bh) ** 2 for gh, r, bh in zip(g, R, b)) / 12.0


@pytest.mark.parametrize("seed", range(6))
def test_error_bounded_meets_bound_with_equality(seed):
    rng = np.random.default_rng(seed)
    P, g, R = instance(rng, 4)
    z, eps = 0.37, 1e-3
    delta, bstar, bits = S.error_bounded(P, g, R, z, eps)
    e = sum(d * d * gh for d, gh in zip(delta, g)) / 12.0
    assert math.isclose(e, (eps * z) ** 2, rel_tol=1e-12)
    assert cont_error(g, R, bstar) == pytest.approx((eps * z) ** 2, rel=1e-12)
    # integer widths: ceil (clamped to >= 1 bit) keeps the error under the bound
    assert S.expected_error(g, R, bits) <= (eps * z) ** 2
    for b, bs in zip(bits, bstar):
        assert b == max(math.ceil(bs), 1)


@pytest.mark.parametrize("seed", range(4))
def test_error_bounded_is_the_constrained_optimum(seed):
    rng = np.random.default_rng(100 + seed)
    P, g, R = instance(rng, 3)
    z, eps = 1.3, 2e-3
    _, bstar, _ = S.error_bounded(P, g, R, z, eps)
    Pn = np.array(P) / sum(P)
    cons = {"type": "ineq", "fun": lambda b: 1.0 - cont_error(g, R, b) / (eps * z) ** 2}
    res = minimize(lambda b: float(Pn @ b), x0=np.array(bstar) + 3.0, constraints=[cons], method="SLSQP",
                   options={"ftol": 1e-14, "maxiter": 500})
    assert res.success
    np.testing.assert_allclose(res.x, bstar, atol=2e-4)


@pytest.mark.parametrize("seed", range(6))
def test_memory_bounded_uses_the_whole_budget(seed):
    rng = np.random.default_rng(200 + seed)
    P, g, R = instance(rng, 4)
    eps = 0.45
    delta, bstar, bits = S.memory_bounded(P, g, R, eps)
    M = 32.0 * sum(P)
    assert math.isclose(sum(p * b for p, b in zip(P, bstar)), eps * M, rel_tol=1e-12)
    assert sum(p * b for p, b in zip(P, bits)) <= eps * M
    for b, bs in zip(bits, bstar):
        assert bs >= 1 and 0 <= bs - b < 1


@pytest.mark.parametrize("seed", range(4))
def test_memory_bounded_is_the_constrained_optimum(seed):
    rng = np.random.default_rng(300 + seed)
    P, g, R = instance(rng, 3)
    eps = 0.5
    _, bstar, _ = S.memory_bounded(P, g, R, eps)
    budget = eps * 32.0 * sum(P)
    e0 = cont_error(g, R, bstar)
    cons = {"type": "eq", "fun": lambda b: (np.array(P) @ b - budget) / sum(P)}
    res = minimize(lambda b: cont_error(g, R, b) / e0, x0=np.full(3, budget / sum(P)), constraints=[cons],
                   method="SLSQP", options={"ftol": 1e-15, "maxiter": 1000})
    assert res.success
    np.testing.assert_allclose(res.x, bstar, atol=2e-4)


def test_single_type_closed_forms():
    # one type: Delta = sqrt(12 / g) eps z; memory: all 32 eps bits
    P, g, R = [5000.0], [4e-3], [8.0]
    d, b, bits = S.error_bounded(P, g, R, 2.0, 1e-2)
    assert math.isclose(d[0], math.sqrt(12.0 / 4e-3) * 2e-2, rel_tol=1e-14)
    assert math.isclose(b[0], math.log2(8.0 / d[0]), rel_tol=1e-14)
    d, b, bits = S.memory_bounded(P, g, R, 0.5)
    assert math.isclose(b[0], 16.0, rel_tol=1e-14) and bits[0] == 16


def test_identical_types_get_identical_widths():
    P, g, R = [1000.0] * 3, [1e-3] * 3, [4.0] * 3
    for fn in (lambda: S.error_bounded(P, g, R, 1.0, 1e-3), lambda: S.memory_bounded(P, g, R, 0.4)):
        _, b, bits = fn()
        assert len(set(bits)) == 1 and max(b) - min(b) == 0.0


def test_scaling_g():
    rng = np.random.default_rng(7)
    P, g, R = instance(rng, 4)
    # memory-bounded: widths do not depend on the scale of g
    _, b1, _ = S.memory_bounded(P, g, R, 0.5)
    _, b2, _ = S.memory_bounded(P, [1e3 * x for x in g], R, 0.5)
    np.testing.assert_allclose(b1, b2, rtol=0, atol=1e-9)
    # error-bounded: g x 4 means every Delta halves, one more bit each
    _, b3, _ = S.error_bounded(P, g, R, 1.0, 1e-3)
    _, b4, _ = S.error_bounded(P, [4.0 * x for x in g], R, 1.0, 1e-3)
    np.testing.assert_allclose(np.array(b4) - np.array(b3), 1.0, atol=1e-9)


def test_zero_gradient_types_take_min_bits():
    P, g, R = [1000.0, 2000.0], [0.0, 1e-2], [1.0, 1.0]
    _, _, bits = S.error_bounded(P, g, R, 1.0, 1e-3, min_bits=3)
    assert bits[0] == 3
    _, bs, bits = S.memory_bounded(P, g, R, 0.5, min_bits=3)
    assert bits[0] == 3
    # the live type gets the rest of the budget: 0.5*32*3000 - 3*1000 over 2000 variables
    assert math.isclose(bs[1], (0.5 * 32 * 3000 - 3000) / 2000.0, rel_tol=1e-12)


def test_widen_range():
    assert S.widen_range(-1.0, 3.0, 2.0) == (-3.0, 5.0)
    assert S.widen_range(0.0, 1.0, 1.0) == (0.0, 1.0)
