"""Pins of the oracle codec, layout and RNG against what the paper and the
mathematics fix (no GPU).

- Eq. 3: decoding is exact, encoding rounds to the nearest lattice point, so
  re-encoding a decoded code returns it and the error is at most Delta/2;
  brute force over every code confirms "nearest".
- Eq. 11 and the rounding-probability statement of Sec. 5: with dither the
  probability of rounding up equals the fractional part Y, so the mean error
  vanishes; the error variance is Delta^2/12 for round-to-nearest on uniform
  fractions and E[Y(1-Y)] Delta^2 = Delta^2/6 with dither.
- Fig. 4: adding 1.4 Delta per step and rounding to nearest gives the same
  -0.4 Delta error every step; dithering removes the drift on average.
- Sec. 7 / Fig. 7: three 17-bit values fit in two 32-bit words when they may
  span words; the float32 2D state p, v, F, C is 48 bytes (Sec. 8.1).
- Philox4x32-10 against AMD rocRAND's independent implementation.
"""
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import workloads as WL

HERE = os.path.dirname(os.path.abspath(__file__))


def scheme_with_x(bits, lo=0.0, hi=1.0, dither=False, dim=2, seed=0):
    """A scheme whose first field is an x field under test."""
    s = WL.scheme_c1(dim, False, seed)
    s["fields"][0] = WL.fixed("x", bits, lo, hi, dither)
    return s


def enc_x(orc, scheme, xs, step=0, tag=2, f64=False):
    dim = scheme["dim"]
    n = xs.size
    x = np.zeros((dim, n), dtype=np.float64 if f64 else np.float32)
    x[0] = xs
    x[1:] = 0.5
    v, C, F = WL.rest_state(dim, n)
    if f64:
        v, C, F = v.astype(np.float64), C.astype(np.float64), F.astype(np.float64)
    words, st = orc.encode(scheme, x, v, C, F, step, tag)
    return words, st


def x_codes(orc, scheme, words):
    comp, _, _, _ = orc.layout(scheme)
    off = int(comp[0, 0])
    bits = scheme["fields"][0]["bits"]
    w = words.astype(np.uint64)
    lo_word = w[off // 32]
    hi_word = w[off // 32 + 1] if off // 32 + 1 < w.shape[0] else np.zeros_like(lo_word)
    both = lo_word | (hi_word << np.uint64(32))
    return ((both >> np.uint64(off % 32)) & np.uint64((1 << bits) - 1)).astype(np.int64)


# ------------------------------------------------------------------ layout
def test_layout_fig7_three_17bit_fields_in_two_words(orc):
    s = WL.scheme_c1(3)
    s["fields"][0] = WL.fixed("x", 17, 0.0, 1.0)
    comp, fo, total, W = orc.layout(s)
    assert list(comp[0, :3]) == [0, 17, 34]
    # the second component spans words 0 and 1 (bits 17..33)
    assert comp[0, 1] // 32 == 0 and (comp[0, 1] + 16) // 32 == 1
    # with only the x field counted, 51 bits -> 2 words (bit struct needs 3)
    assert -(-51 // 32) == 2


def test_layout_spanning_bits_by_hand(orc):
    # x = 3 x 17 bits; write codes 0x1ABCD, 0x0F0F1, 0x15555 and read the words
    s = WL.scheme_c1(3)
    s["fields"][0] = WL.fixed("x", 17, 0.0, 1.0)
    codes = [0x1ABCD, 0x0F0F1, 0x15555]
    delta = 2.0 ** -17
    x = np.array([[c * delta] for c in codes], dtype=np.float64)
    v, C, F = WL.rest_state(3, 1)
    words, _ = orc.encode(s, x, v.astype(np.float64), C.astype(np.float64), F.astype(np.float64))
    rec = 0
    for k in range(words.shape[0]):
        rec |= int(words[k, 0]) << (32 * k)
    expect = codes[0] | (codes[1] << 17) | (codes[2] << 34)
    assert rec & ((1 << 51) - 1) == expect
    assert int(words[0, 0]) == (codes[0] | ((codes[1] & 0x7FFF) << 17))
    assert int(words[1, 0]) & 0x7FFFF == ((codes[1] >> 15) | (codes[2] << 2)) & 0x7FFFF


@pytest.mark.parametrize("dim,nbytes", [(2, 48), (3, 96)])
def test_fp32_layout_size(orc, dim, nbytes):
    _, _, total, W = orc.layout(WL.scheme_fp32(dim))
    assert 4 * W == nbytes and total == 8 * nbytes


@pytest.mark.parametrize("dim", [2, 3])
def test_raw_f32_codec_is_the_float32_bit_pattern(orc, dim):
    """RAW_F32 stores each component's IEEE float32 bits (F - I on the
    diagonal of a REL_IDENTITY field, formed in binary64 and rounded once);
    decoding gives the float32 value back (+ 1 on that diagonal).  Checked
    against NumPy's own float32 casts and bit views, in placement order,
    including signed zeros, subnormals, infinities and NaN."""
    rng = np.random.default_rng(7 + dim)
    n = 257
    x, v, C, F = WL.random_state(rng, dim, n, c_scale=1e3, f_scale=0.5)
    special = np.array([0.0, -0.0, 1e-40, -3e-39, np.inf, -np.inf, np.nan, 3.4e38, 1.0 + 2 ** -23, 1e-8],
                       dtype=np.float32)
    v[0, :special.size] = special
    C[-1, :special.size] = special[::-1]
    F[0, :special.size] = special
    scheme = WL.scheme_fp32(dim, 0)
    scheme["fields"] = [scheme["fields"][i] for i in (2, 0, 3, 1)]  # placement C, x, F, v
    scheme["fields"][2]["rel_identity"] = True
    words, st = orc.encode(scheme, x, v, C, F)
    diag = np.array([(i % (dim + 1)) == 0 for i in range(dim * dim)])
    Frel = F.astype(np.float64) - np.where(diag[:, None], 1.0, 0.0)
    expect = np.concatenate([C, x, Frel.astype(np.float32), v], axis=0).view(np.uint32)
    assert words.shape == expect.shape and np.array_equal(words, expect)
    assert all(st[f]["sat"] == 0 and st[f]["nan"] == 0 for f in "xvCF")
    dx, dv, dC, dF = orc.decode(scheme, words)
    for got, ref in ((dx, x), (dv, v), (dC, C)):
        same = (got == ref.astype(np.float64)) | (np.isnan(got) & np.isnan(ref))
        assert same.all()
    refF = Frel.astype(np.float32).astype(np.float64) + np.where(diag[:, None], 1.0, 0.0)
    assert (((dF == refF) | (np.isnan(dF) & np.isnan(refF)))).all()


def test_config_record_sizes(orc):
    assert orc.layout(WL.scheme_c1(2))[3] == 7       # 200 bits
    assert orc.layout(WL.scheme_c1(3, True))[3] == 13  # 396 bits
    _, _, total, W = orc.layout(WL.scheme_c3())
    assert total == 384 and W == 12                   # 48 B vs 96 B


def test_invalid_schemes_rejected(orc):
    s = WL.scheme_c1(2)
    s["fields"][1]["hi"] = s["fields"][1]["lo"]
    assert not orc.validate(s)
    s = WL.scheme_c1(2)
    s["fields"][0]["bits"] = 0
    assert not orc.validate(s)
    s = WL.scheme_c1(2)
    s["fields"][2]["rel_identity"] = True
    assert not orc.validate(s)
    s = WL.scheme_c1(2)
    s["fields"][3] = WL.fixed("C", 16, -1, 1)  # duplicate field
    assert not orc.validate(s)
    assert orc.validate(WL.scheme_c3())


# ------------------------------------------------------------------ Eq. 3
@pytest.mark.parametrize("bits", [1, 5, 12, 17, 21])
def test_exhaustive_roundtrip(orc, bits):
    s = scheme_with_x(bits)
    u = np.arange(2 ** bits, dtype=np.int64)
    xs = u * 2.0 ** -bits  # lattice points, exact in float32
    words, st = enc_x(orc, s, xs.astype(np.float32))
    assert np.array_equal(x_codes(orc, s, words), u)
    assert st["x"]["sat"] == 0
    xd, _, _, _ = orc.decode(s, words)
    assert np.array_equal(xd[0], xs)


def test_roundtrip_nonpow2_range(orc):
    s = scheme_with_x(16, -20.0, 20.0)
    u = np.arange(2 ** 16, dtype=np.int64)
    delta = 40.0 / 2 ** 16
    xs = -20.0 + u * delta
    words, _ = enc_x(orc, s, xs, f64=True)
    assert np.array_equal(x_codes(orc, s, words), u)
    xd, _, _, _ = orc.decode(s, words)
    assert np.array_equal(xd[0], xs)


@pytest.mark.parametrize("bits,lo,hi", [(10, 0.0, 1.0), (12, -20.0, 20.0), (8, -0.3, 0.7)])
def test_nearest_by_brute_force(orc, bits, lo, hi):
    rng = np.random.default_rng(1)
    s = scheme_with_x(bits, lo, hi)
    xs = rng.uniform(lo, hi - (hi - lo) * 2.0 ** -bits, 3000)
    words, _ = enc_x(orc, s, xs, f64=True)
    codes = x_codes(orc, s, words)
    delta = (hi - lo) / 2 ** bits
    lattice = lo + np.arange(2 ** bits) * delta
    dist = np.abs(xs[:, None] - lattice[None, :])
    best = dist.min(axis=1)
    got = np.abs(xs - (lo + codes * delta))
    assert np.all(got <= best * (1 + 1e-12) + 1e-300)
    assert np.all(got <= delta / 2 * (1 + 2.0 ** -40))


def test_ties_round_up_and_saturation(orc):
    s = scheme_with_x(4)  # Delta = 1/16
    xs = np.array([0.5 / 16, 1.5 / 16, 15.4 / 16, 15.6 / 16, 1.2, -0.3])
    words, st = enc_x(orc, s, xs, f64=True)
    assert list(x_codes(orc, s, words)) == [1, 2, 15, 15, 15, 0]
    assert st["x"]["sat"] == 3


def test_nan_counted(orc):
    s = scheme_with_x(8)
    xs = np.array([np.nan, 0.25, np.inf, -np.inf])
    words, st = enc_x(orc, s, xs, f64=True)
    assert list(x_codes(orc, s, words)) == [0, 64, 255, 0]
    assert st["x"]["nan"] == 1 and st["x"]["sat"] == 2


# ------------------------------------------------------------------ Eq. 11
def test_dither_round_up_probability_equals_fraction(orc):
    bits = 10
    s = scheme_with_x(bits, dither=True)
    delta = 2.0 ** -bits
    fracs = np.array([0.1, 0.25, 0.5, 0.73, 0.9])
    n_each = 20000
    for Y in fracs:
        xs = np.full(n_each, (100 + Y) * delta)
        words, st = enc_x(orc, s, xs, f64=True)
        up = np.mean(x_codes(orc, s, words) == 101)
        assert abs(up - Y) < 4 * np.sqrt(Y * (1 - Y) / n_each) + 2.0 ** -16
        assert st["x"]["up"] + st["x"]["down"] == 2 * n_each  # both x components


def test_dither_unbiased_and_error_variances(orc):
    bits = 12
    delta = 2.0 ** -bits
    rng = np.random.default_rng(3)
    n = 200000
    xs = rng.uniform(0.1, 0.9, n)
    e_near = []
    for dither in (False, True):
        s = scheme_with_x(bits, dither=dither)
        words, _ = enc_x(orc, s, xs, f64=True)
        err = (x_codes(orc, s, words) * delta - xs) / delta
        e_near.append(err)
    near, dith = e_near
    # nearest: uniform on [-1/2, 1/2], variance 1/12
    assert abs(near.var() - 1 / 12) < 0.003
    # dithered: unbiased, variance E[Y(1-Y)] = 1/6 for uniform Y
    assert abs(dith.mean()) < 4 * np.sqrt(1 / 6 / n) + 2.0 ** -17
    assert abs(dith.var() - 1 / 6) < 0.004
    assert np.all(np.abs(dith) < 1.0)


def test_fig4_correlated_error_and_dither(orc):
    """Adding 1.4 Delta per step: rounding to nearest gives a constant
    -0.4 Delta error every step; dithering keeps the mean increment."""
    bits = 16
    delta = 2.0 ** -bits
    steps = 200
    for dither, check in ((False, "constant"), (True, "unbiased")):
        s = scheme_with_x(bits, dither=dither)
        y = np.zeros(4096)  # 4096 independent copies
        errs = []
        for t in range(steps):
            target = y + 1.4 * delta
            words, _ = enc_x(orc, s, target, step=t, tag=1, f64=True)
            y = x_codes(orc, s, words) * delta
            errs.append((y - target) / delta)
        errs = np.array(errs)
        if check == "constant":
            assert np.allclose(errs, -0.4, atol=1e-9)
        else:
            mean_inc = y.mean() / (steps * delta)
            assert abs(mean_inc - 1.4) < 0.01
            assert abs(errs.mean()) < 0.01


# ------------------------------------------------------------------ shared exponent
def sexp_scheme(bits=13, exp_bits=6, hi=20.0, dither=False):
    s = WL.scheme_c3()
    for f in s["fields"]:
        f["dither"] = False
    s["fields"][1] = WL.shared_exp("v", bits, exp_bits, hi, dither)
    return s


def v_codes(orc, scheme, words):
    comp, fo, _, _ = orc.layout(scheme)
    f = scheme["fields"][1]
    w = [int(words[k, 0]) for k in range(words.shape[0])]
    rec = sum(wk << (32 * k) for k, wk in enumerate(w))
    e = (rec >> int(fo[1])) & ((1 << f["exp_bits"]) - 1)
    comps = [(rec >> int(comp[1, c])) & ((1 << f["bits"]) - 1) for c in range(3)]
    return e, comps


def enc_v(orc, scheme, vvec):
    x = np.full((3, 1), 0.5)
    v = np.asarray(vvec, dtype=np.float64).reshape(3, 1)
    _, C, F = WL.rest_state(3, 1)
    return orc.encode(scheme, x, v, C.astype(np.float64), F.astype(np.float64))


def test_shared_exp_zero_and_power_of_two(orc):
    s = sexp_scheme()
    words, _ = enc_v(orc, s, [0.0, 0.0, 0.0])
    e, comps = v_codes(orc, s, words)
    assert e == 0 and comps == [0, 0, 0]  # E = E_min, all magnitudes 0
    _, v, _, _ = orc.decode(s, words)
    assert np.all(v == 0)
    # max component exactly 2^k: E = k + 1, magnitude 2^11 of 12 bits
    words, _ = enc_v(orc, s, [4.0, -1.0, 0.5])
    e, comps = v_codes(orc, s, words)
    Emax = 5  # ceil(log2 20)
    Emin = Emax - 63
    assert e + Emin == 3
    assert comps[0] == 2048 and comps[1] == (512 | 4096) and comps[2] == 256
    _, v, _, _ = orc.decode(s, words)
    assert list(v[:, 0]) == [4.0, -1.0, 0.5]


def test_shared_exp_error_bound_and_roundtrip(orc):
    s = sexp_scheme()
    rng = np.random.default_rng(5)
    for _ in range(400):
        vec = rng.standard_normal(3) * 10.0 ** rng.uniform(-6, 1)
        words, st = enc_v(orc, s, vec)
        e, comps = v_codes(orc, s, words)
        E = e + (5 - 63)
        _, v, _, _ = orc.decode(s, words)
        assert np.all(np.abs(v[:, 0] - vec) <= 0.5 * 2.0 ** (E - 12) * (1 + 1e-15))
        # max magnitude uses the top bit unless E hit the bottom of its range
        assert max(c & 4095 for c in comps) >= 2048 or E == 5 - 63
        # decode -> encode is the identity
        w2, _ = enc_v(orc, s, v[:, 0])
        assert np.array_equal(w2, words)


def test_shared_exp_exponent_bump_on_round_up(orc):
    s = sexp_scheme()
    # |v| just below 2: ilogb -> E = 1, magnitude rounds to 4096 -> E = 2
    vec = [2.0 - 2.0 ** -14, 0.0, 0.0]
    words, _ = enc_v(orc, s, vec)
    e, comps = v_codes(orc, s, words)
    assert e + (5 - 63) == 2 and comps[0] == 2048
    _, v, _, _ = orc.decode(s, words)
    assert v[0, 0] == 2.0


def test_shared_exp_saturates(orc):
    s = sexp_scheme()
    words, st = enc_v(orc, s, [100.0, 1.0, -1.0])
    _, v, _, _ = orc.decode(s, words)
    assert st["v"]["sat"] == 1
    assert v[0, 0] == 4095 * 2.0 ** (5 - 12)


# ------------------------------------------------------------------ Philox
def test_philox_matches_rocrand(orc, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "philox_ref")
    subprocess.run([hipcc, "-O2", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "pins", "philox_rocrand.cpp"), "-o", exe],
                   check=True, capture_output=True)
    rng = np.random.default_rng(7)
    cases = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6]]
    cases += rng.integers(0, 2 ** 32, (60, 6), dtype=np.uint64).tolist()
    cases += [[p, s, j, t, 0x12345678, 0x9ABCDEF0] for p in (0, 77, 2 ** 31 - 1)
              for s in (0, 5) for j in (0, 2) for t in (1, 2)]
    inp = "\n".join(" ".join("%x" % int(c) for c in case) for case in cases) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [[int(t, 16) for t in line.split()] for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for case, r in zip(cases, ref):
        got = orc.philox(case[:4], case[4:])
        assert [int(g) for g in got] == r, case


def test_philox_statistics(orc):
    n = 4096
    vals = np.array([orc.philox([i, 3, 0, 1], [11, 0]) for i in range(n)], dtype=np.uint64)
    halves = np.concatenate([(vals & 0xFFFF).ravel(), (vals >> 16).ravel()]).astype(np.float64)
    # chi-square over 64 bins of the 16-bit draws
    hist = np.bincount((halves // 1024).astype(np.int64), minlength=64)
    exp = halves.size / 64
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 120  # 63 dof, p ~ 1e-5
    u = halves / 65536.0
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 4 / np.sqrt(u.size)


@pytest.mark.parametrize("dither", [False, True])
def test_oracle_round_up_down_ratio(orc, dither):
    """Simulation-scale dithering (Sec. 5, the round-up / round-down study of
    Sec. 8.1): an elastic block that hits the floor and rings, stored at
    coarse widths.  Round to nearest locks C and F onto lattice points
    (mostly rounding down: overall ratio ~0.75); dithered stores round up
    and down about equally often (ratio within 3 % of 1)."""
    sc = WL.bounce_block(seed=1, dither=dither)
    w, _ = orc.encode(sc["scheme"], *sc["state"], 0, 2)
    sim = orc.Sim(sc["scheme"], sc["params"], w)
    sim.step(sc["steps"])
    st = sim.stats()
    sim.close()
    up = sum(st[f]["up"] for f in "xvCF")
    down = sum(st[f]["down"] for f in "xvCF")
    if dither:
        assert abs(up / down - 1.0) <= 0.03
    else:
        assert up / down < 0.85
        assert st["F"]["up"] < 0.8 * st["F"]["down"] and st["C"]["up"] < 0.8 * st["C"]["down"]
