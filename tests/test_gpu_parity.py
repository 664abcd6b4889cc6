"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Bars: packed words bit-exact for the codec on identical float32 inputs and
for config c1 (whose closed form has a margin of 0.0108 LSB at every
rounding); positions within 1e-4 of the unit domain for dithered scenes,
where FP32 arithmetic on the GPU may flip a rounding that lies within FP32
error of a lattice tie.
"""
import numpy as np
import pytest

import workloads as WL
from gpu_common import by_id, gpu_context, gpu_decode_np, lsb_differences, note, oracle_sim

pytestmark = pytest.mark.gpu


def edge_state(rng, dim, n):
    x, v, C, F = WL.random_state(rng, dim, n)
    # out-of-range, ties, denormals, NaN / Inf, exact lattice points
    k = min(n, 16)
    x[0, :k] = np.array([0.0, 1.0, 1.5, -0.1, 0.5, 2.0 ** -21, 1e-40, np.nan,
                         0.25 + 2.0 ** -21, 3 * 2.0 ** -22, 0.999999, 0.7, 0.1, 0.2, 0.3, 0.4],
                        dtype=np.float32)[:k]
    v[0, :k] = np.array([25.0, -25.0, np.inf, -np.inf, 0.0, -0.0, 19.9999, 40.0 / 2 ** 17,
                         1e-30, -1e-30, 7.0, -7.0, 3.0, 2.0, 1.0, 0.5], dtype=np.float32)[:k]
    C[0, :k] = 100.0
    F[0, :k] = 3.0
    return x, v, C, F


SCHEMES = {
    "c1_2d": lambda: WL.scheme_c1(2, False, 1),
    "c2_3d_dither": lambda: WL.scheme_c1(3, True, 5),
    "c3_sexp": lambda: WL.scheme_c3(11),
    "fp32_3d": lambda: WL.scheme_fp32(3, 0),
    "fp32_2d": lambda: WL.scheme_fp32(2, 0),
}


@pytest.mark.parametrize("name", list(SCHEMES))
@pytest.mark.parametrize("n", [1, 300, 5003])
def test_encode_decode_bit_exact(gpu_lib, orc, name, n):
    note(f"encode/decode {name} n={n}")
    scheme = SCHEMES[name]()
    dim = scheme["dim"]
    rng = np.random.default_rng(n)
    state = edge_state(rng, dim, n)
    scene = {"scheme": scheme, "params": WL.params(dim, 64, 1e-4, 1e-6), "state": state}
    ctx = gpu_context(gpu_lib, scene)
    gw = ctx.words()
    ow, ost = orc.encode(scheme, *state, 0, 2)
    assert gw.shape == ow.shape
    assert np.array_equal(gw, ow), f"{np.sum(gw != ow)} words differ"
    gst = ctx.stats()
    for f in "xvCF":
        assert gst[f] == ost[f], f
    # decode: binary64 value rounded once to float32
    dec = gpu_decode_np(ctx)
    odec = orc.decode(scheme, ow)
    for g, o in zip(dec, odec):
        o32 = o.astype(np.float32).astype(np.float64)
        bad = int(np.sum(~((g == o32) | (np.isnan(g) & np.isnan(o32)))))
        assert bad == 0, f"{bad} decoded values differ"
    ctx.close()


def test_encode_random_schemes(gpu_lib, orc):
    rng = np.random.default_rng(42)
    for trial in range(12):
        dim = 2 + trial % 2
        scheme = WL.random_scheme(rng, dim, seed=trial)
        note(f"random scheme {trial}: {[(f['field'], f['kind'], f['bits']) for f in scheme['fields']]}")
        state = WL.random_state(rng, dim, 2000)
        scene = {"scheme": scheme, "params": WL.params(dim, 64, 1e-4, 1e-6), "state": state}
        ctx = gpu_context(gpu_lib, scene)
        ow, _ = orc.encode(scheme, *state, 0, 2)
        assert np.array_equal(ctx.words(), ow)
        ctx.close()


def c1_codes(words, off, bits):
    w = words.astype(np.uint64)
    lo = w[off // 32]
    hi = w[off // 32 + 1] if off // 32 + 1 < w.shape[0] else np.zeros_like(lo)
    return (((lo | (hi << np.uint64(32))) >> np.uint64(off % 32)) & np.uint64((1 << bits) - 1)).astype(np.int64)


def test_c1_closed_form_bit_exact(gpu_lib, orc):
    """Config c1, 50 steps: GPU words equal the oracle's and the closed form."""
    note("c1 50 steps")
    sc = WL.c1()
    ctx = gpu_context(gpu_lib, sc)
    w0 = ctx.words()
    ctx.step(50)
    gw, gids = ctx.words(), ctx.ids()
    sim, ow0, _ = oracle_sim(orc, sc)
    assert np.array_equal(w0, ow0)
    sim.step(50)
    ow, oids = sim.words(), sim.ids()
    assert np.array_equal(gids, oids)  # same sort permutation
    assert np.array_equal(gw, ow)
    # closed form: x (20 bits at 0, 20), v (16 at 40, 56), C (64..), F (128..)
    assert np.all(c1_codes(gw, 56, 16) == 32768 - 100)
    assert np.all(c1_codes(gw, 40, 16) == 32768)
    assert np.array_equal(c1_codes(gw, 20, 20), c1_codes(w0, 20, 20)[gids] - 161)
    assert np.array_equal(c1_codes(gw, 0, 20), c1_codes(w0, 0, 20)[gids])
    for c in range(8):
        assert np.all(c1_codes(gw, 72 + 16 * c, 16) == 32768)
    st = ctx.stats()
    assert st["fallback"] == 0 and st["sorts"] == 1 and st["steps"] == 50
    ctx.close()


def small_scene(dim, seed, dither=True, sort_every=4, n_extra=1234):
    """Two cubes with different velocities plus a ragged cloud, 32^dim grid."""
    rng = np.random.default_rng(seed)
    res = 32
    side = 10 / res
    corners = np.array([[0.2, 0.3, 0.25], [0.55, 0.35, 0.5]])[:, :dim]
    vels = rng.uniform(-1, 1, (2, dim))
    counts = [int(8 * 10 ** dim * 0.9), int(8 * 10 ** dim * 0.9)]
    sch = WL.scheme_c1(dim, dither, seed)
    sc = WL.cubes_scene("small", seed, res, corners, side, counts, vels, 5e-4, 20, sch, sort_every, dim=dim)
    x, v, C, F = sc["state"]
    xe = rng.uniform(0.15, 0.85, (dim, n_extra)).astype(np.float32)
    ve = rng.uniform(-0.5, 0.5, (dim, n_extra)).astype(np.float32)
    _, Ce, Fe = WL.rest_state(dim, n_extra)
    sc["state"] = (np.concatenate([x, xe], 1), np.concatenate([v, ve], 1), np.concatenate([C, Ce], 1),
                   np.concatenate([F, Fe], 1))
    sc["n"] = sc["state"][0].shape[1]
    return sc


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dither", [False, True])
def test_small_scene_trajectory(gpu_lib, orc, dim, dither):
    sc = small_scene(dim, 3 + dim, dither)
    steps = 20
    note(f"small scene dim={dim} dither={dither} n={sc['n']} steps={steps}")
    ctx = gpu_context(gpu_lib, sc)
    sim, ow0, _ = oracle_sim(orc, sc)
    assert np.array_equal(ctx.words(), ow0)
    for chunk in (1, 9, 10):
        ctx.step(chunk)
        sim.step(chunk)
        if chunk == 1:
            # after one substep only roundings within FP32 error of a tie differ
            same = np.mean(by_id(ctx.words(), ctx.ids()) == by_id(sim.words(), sim.ids()))
            assert same > 0.9, same
        # every field, in units of its quantization step (see test_gpu_horizon
        # for the reasoning behind the bars)
        dx, lsb = lsb_differences(orc, sc["scheme"], ctx.words(), ctx.ids(), sim.words(), sim.ids(), sc["params"],
                                  sim.step_count)
        assert np.max(dx) <= 1e-4, np.max(dx)
        for f in "vCF":
            print(f"dim {dim} dither {dither} step {sim.step_count} {f}: "
                  f"<=1 code {np.mean(lsb[f] <= 1 + 1e-9):.5f} max {np.max(lsb[f]):.1f}")
            assert np.mean(lsb[f] <= 1 + 1e-9) >= 0.99, f
            assert np.max(lsb[f]) <= 8, f
    st = ctx.stats()
    assert st["steps"] == steps and st["sorts"] == 5 and st["clamped"] == 0
    ctx.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_grid_mass_conservation(gpu_lib, dim):
    import torch
    sc = small_scene(dim, 11, True, 0)
    note(f"grid mass dim={dim}")
    ctx = gpu_context(gpu_lib, sc)
    ctx.step(3)
    ctx.stream.synchronize()
    m_p = sc["params"]["rho"] * sc["params"]["p_vol"]
    s = ctx.step_count()
    # P2G target of the next substep: int64 fixed-point sums, 2^-32 per unit particle mass
    g = (ctx.grid_a if s % 2 == 0 else ctx.grid_b).view(torch.int64).view(-1, 4)
    mass = g[:, 3].sum().item() * 2.0 ** -32 * m_p
    mom = [g[:, a].sum().item() * 2.0 ** -32 * m_p for a in range(dim)]
    # the weights of one particle sum to 1 up to FP32 rounding of the
    # B-spline products (a few ulp of 2^-24 each), plus 2^-33 per node
    assert abs(mass - m_p * sc["n"]) <= 1e-6 * m_p * sc["n"]
    # P2G conserves momentum: sum over nodes = sum over particles of m v (decoded state)
    _, gv, _, _ = gpu_decode_np(ctx)
    for a in range(dim):
        assert abs(mom[a] - m_p * gv[a].sum()) <= 1e-6 * m_p * np.abs(gv[a]).sum() + 1e-12
    ctx.close()


def test_empty_and_resume(gpu_lib, orc):
    note("empty scene, resume")
    sc = WL.c1()
    empty = dict(sc, state=tuple(a[:, :0] for a in sc["state"]))
    ctx = gpu_context(gpu_lib, empty, capacity=16)
    ctx.step(3)
    assert ctx.step_count() == 3
    ctx.close()
    sc["scheme"] = WL.scheme_c1(2, True, 9)
    sc["params"]["sort_every"] = 8
    a = gpu_context(gpu_lib, sc)
    a.step(20)
    b = gpu_context(gpu_lib, sc)
    b.step(7)
    b.step(13)
    # P2G sums are exact integers, so the GPU path is bit-reproducible
    assert np.array_equal(a.words(), b.words())
    assert np.array_equal(a.ids(), b.ids())
    a.close()
    b.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_run_to_run_bit_identical(gpu_lib, dim):
    sc = small_scene(dim, 21, True, 4)
    note(f"determinism dim={dim}")
    runs = []
    for _ in range(2):
        ctx = gpu_context(gpu_lib, sc)
        ctx.step(12)
        runs.append((ctx.words(), ctx.ids()))
        ctx.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


def test_step_before_encode_is_state_error(gpu_lib):
    sc = WL.c1()
    ctx = gpu_lib.Context(sc["scheme"], sc["params"], 100)
    with pytest.raises(gpu_lib.MpmqError) as e:
        ctx.step(1)
    assert e.value.status == -4
    with pytest.raises(gpu_lib.MpmqError) as e:
        ctx.adjoint(1)
    assert e.value.status == -4
    ctx.close()


def fast_scene(dim, seed, vmax):
    """small_scene with particles fast enough to leave the node tile of
    their sort block (sorted once: sort_every = 0)."""
    sc = small_scene(dim, seed, True, 0)
    x, v, C, F = sc["state"]
    v = np.clip(v * (vmax / max(1e-6, float(np.max(np.abs(v))))), -vmax, vmax).astype(np.float32)
    sc["state"] = (x, v, C, F)
    return sc


@pytest.mark.parametrize("dim", [2, 3])
def test_tile_fallback_trajectory(gpu_lib, orc, dim):
    """Stencils that left their tile go through the global P2G / G2P paths
    (int64 atomics straight into the grid): same trajectory as the oracle,
    and as the GPU with a sort every substep (no stencil leaves a tile)."""
    sc = fast_scene(dim, 21 + dim, 18.0)
    steps = 16
    note(f"tile fallback dim={dim} n={sc['n']} steps={steps}")
    ctx = gpu_context(gpu_lib, sc)
    ctx.step(steps)
    st = ctx.stats()
    assert st["sorts"] == 1 and st["fallback"] > 0, st
    resorted = dict(sc, params=dict(sc["params"], sort_every=1))
    ctx1 = gpu_context(gpu_lib, resorted)
    ctx1.step(steps)
    assert ctx1.stats()["sorts"] == steps
    sim, _, _ = oracle_sim(orc, sc)
    sim.step(steps)
    gx = by_id(gpu_decode_np(ctx)[0], ctx.ids())
    gx1 = by_id(gpu_decode_np(ctx1)[0], ctx1.ids())
    ox = by_id(orc.decode(sc["scheme"], sim.words())[0], sim.ids())
    assert np.max(np.abs(gx - ox)) <= 1e-4, np.max(np.abs(gx - ox))
    assert np.max(np.abs(gx - gx1)) <= 1e-4, np.max(np.abs(gx - gx1))
    ctx.close()
    ctx1.close()


def test_p2g_clamp_is_counted(gpu_lib):
    """Velocities above the fixed-point P2G range (|v| > 2^12) are clamped so
    that the int64 node sums cannot overflow, and every clamped particle is
    counted.  With a sort every substep the fused kernel scatters nothing,
    so one substep's count is exactly the bootstrap P2G's."""
    note("p2g clamp counter")
    rng = np.random.default_rng(5)
    n = 1000
    x, v, C, F = WL.random_state(rng, 3, n, c_scale=0.0, f_scale=0.0)
    v[:] = rng.uniform(-1, 1, v.shape).astype(np.float32)
    v[0, :10] = 5000.0
    scene = {"scheme": WL.scheme_fp32(3, 0), "params": WL.params(3, 32, 1e-6, 1e-6, sort_every=1),
             "state": (x, v, C, F)}
    ctx = gpu_context(gpu_lib, scene)
    ctx.step(1)
    assert ctx.stats()["clamped"] == 10
    ctx.close()


@pytest.mark.parametrize("mode", ["generic", "specialized", "stats"])
def test_nan_position_substep(gpu_lib, orc, mode):
    """A NaN position (stored raw) gives NaN B-spline weights, so G2P hands
    the encoder NaN velocity, affine and deformation components: the
    shared-exponent fields v and C and the fixed-point F store code 0 for
    each and count it (Eq. 11; E from the finite components, here none), on
    the generic and the scheme-specialized fused kernels and with the
    round-up/down counters on.  A NaN position clamps to stencil base 0, so
    the NaN particles touch only the grid corner, far from the others, which
    are compared at the usual bars."""
    rng = np.random.default_rng(17)
    n = 3000
    x, v, C, F = WL.random_state(rng, 3, n, x_lo=0.3, x_hi=0.7)
    nan_ids = np.array([5, 100, 1777, 2999])
    x[1, nan_ids] = np.nan
    scheme = {"dim": 3, "seed": 9, "fields": [WL.raw("x"), WL.shared_exp("v", 13, 6, 20.0, True),
                                              WL.shared_exp("C", 16, 6, 2048.0, True),
                                              WL.fixed("F", 14, -1.0, 1.0, True, rel_identity=True)]}
    sc = {"scheme": scheme, "params": WL.params(3, 64, 1e-4, 1e-6), "state": (x, v, C, F)}
    note(f"NaN positions n={n} mode={mode}")
    ctx = gpu_context(gpu_lib, sc)
    if mode == "specialized":
        ctx.specialize(True)
    if mode == "stats":
        ctx.set_stats(1)
    sim, ow0, _ = oracle_sim(orc, sc)
    ctx.reset_stats()
    ctx.step(1)
    sim.step(1)
    gw, gids, ow, oids = ctx.words(), ctx.ids(), sim.words(), sim.ids()
    g = [by_id(a, gids) for a in orc.decode(scheme, gw)]
    o = [by_id(a, oids) for a in orc.decode(scheme, ow)]
    # the NaN particles: position NaN, v = C = 0 (code 0), F - I = lo (code 0)
    f0 = np.full(9, -1.0)
    f0[[0, 4, 8]] = 0.0
    for side in (g, o):
        assert np.all(np.isnan(side[0][:, nan_ids]))
        assert np.all(side[1][:, nan_ids] == 0.0) and np.all(side[2][:, nan_ids] == 0.0)
        assert np.all(side[3][:, nan_ids] == f0[:, None])
    # everyone else
    keep = np.setdiff1d(np.arange(n), nan_ids)
    dx, lsb = lsb_differences(orc, scheme, gw, gids, ow, oids, sc["params"], 1)
    assert np.max(dx[:, keep]) <= 1e-4, np.max(dx[:, keep])
    for f in "vCF":
        d = lsb[f][:, keep]
        assert np.mean(d <= 1 + 1e-9) >= 0.99 and np.max(d) <= 8, (f, np.max(d))
    # counters: one NaN per component of each NaN particle, as the oracle counts
    gst, ost = ctx.stats(), sim.stats()
    for f, nc in (("v", 3), ("C", 9), ("F", 9)):
        assert gst[f]["nan"] == ost[f]["nan"] == nc * len(nan_ids), (f, gst[f]["nan"], ost[f]["nan"])
        assert gst[f]["sat"] == ost[f]["sat"], f
    if mode == "stats":
        for f in "vCF":
            tot_g = gst[f]["up"] + gst[f]["down"]
            tot_o = ost[f]["up"] + ost[f]["down"]
            assert tot_g == tot_o, (f, tot_g, tot_o)
    ctx.close()
    sim.close()
