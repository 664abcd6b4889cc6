"""Oracle of the automatic quantization solver (Sec. 4, Eqs. 6-10, Alg. 1).

TEST INFRASTRUCTURE ONLY: plain Python in binary64, written from the
paper; nothing in the GPU library imports it.

Notation: H data types; type h has P_h variables, accumulated squared
gradient g_h (Eq. 8) and range width R_h; the quantization step is
Delta_h = R_h 2^-b_h (Eq. 3), and the expected squared error of the
objective under uniformly distributed rounding errors is
E = (1/12) sum_h Delta_h^2 g_h (Eq. 8).

Error-bounded (Eqs. 6, 9, 10): minimize sum_h P_h b_h subject to
E <= (eps z)^2; the Lagrange solution is
Delta_h = sqrt(12 P_h (eps z)^2 / (g_h sum P)), b_h = ceil(log2(R_h / Delta_h)).

Memory-bounded (Eq. 7, M = 32 sum P bits of FP32 storage): minimize E
subject to sum_h P_h b_h <= eps_mem M.  The paper defers the solution to a
supplement that is not available; the Lagrange conditions
Delta_h g_h / 6 = mu P_h / (Delta_h ln 2) give Delta_h = K sqrt(P_h / g_h),
and the active constraint fixes
log2 K = [sum P_h log2 R_h - 1/2 sum P_h log2(P_h / g_h) - eps_mem M] / sum P_h.
Reading: integer bits b_h = floor(b*_h), which keeps the memory bound.

Types with g_h = 0 do not affect z: they get the minimum width (and, in the
memory-bounded case, their bits leave the budget first).  Bits are clamped
to [min_bits, max_bits].
"""
import math


def expected_error(g, R, bits):
    """E[delta z] = (1/12) sum Delta_h^2 g_h with Delta_h = R_h 2^-b_h (Eq. 8)."""
    return sum((r * 2.0 ** -b) ** 2 * gh for gh, r, b in zip(g, R, bits)) / 12.0


def error_bounded(P, g, R, z, eps, min_bits=1, max_bits=32):
    """Returns (Delta, b_continuous, bits) of the error-bounded scheme."""
    sumP = float(sum(P))
    target = (eps * z) ** 2
    delta, bstar, bits = [], [], []
    for p, gh, r in zip(P, g, R):
        if gh > 0.0:
            d = math.sqrt(12.0 * p * target / (gh * sumP))
            b = math.log2(r / d)
            delta.append(d)
            bstar.append(b)
            bits.append(min(max(math.ceil(b), min_bits), max_bits))
        else:
            delta.append(math.inf)
            bstar.append(-math.inf)
            bits.append(min_bits)
    return delta, bstar, bits


def memory_bounded(P, g, R, eps_mem, min_bits=1, max_bits=32):
    """Returns (Delta, b_continuous, bits) of the memory-bounded scheme."""
    budget = eps_mem * 32.0 * float(sum(P))
    live = [h for h in range(len(P)) if g[h] > 0.0]
    dead = [h for h in range(len(P)) if not g[h] > 0.0]
    budget -= sum(P[h] * min_bits for h in dead)
    sumP = float(sum(P[h] for h in live))
    delta = [math.inf] * len(P)
    bstar = [-math.inf] * len(P)
    bits = [min_bits] * len(P)
    if live:
        log2K = (sum(P[h] * math.log2(R[h]) for h in live)
                 - 0.5 * sum(P[h] * math.log2(P[h] / g[h]) for h in live) - budget) / sumP
        for h in live:
            d = 2.0 ** log2K * math.sqrt(P[h] / g[h])
            b = math.log2(R[h] / d)
            delta[h] = d
            bstar[h] = b
            bits[h] = min(max(math.floor(b), min_bits), max_bits)
    return delta, bstar, bits


def widen_range(lo, hi, factor=2.0):
    """Range of a type from the values a full-precision run recorded (Alg. 1),
    widened about its centre by `factor` against overflow (Sec. 3.2)."""
    mid = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo) * factor
    return mid - half, mid + half
