"""Pins of the oracle's fluid material (state x, v, C, J; Kirchhoff stress
E (J - 1) I, J' = J (1 + dt tr C')) and of its adjoint (no GPU).

- The J field's codec: record sizes (2D fluid state 36 B in FP32, Sec. 8.3),
  round trip, J - 1 storage.
- P2G against a brute-force sum over every node with the B-spline kernel.
- G2P on an affine grid field: C' = B exactly, so J' = J (1 + dt tr B).
- P2G conserves mass and momentum; a fluid at rest with J = 1 has no stress.
- The VJP against central finite differences (per field and mixed), and the
  trajectory sensitivities G against finite differences of the whole run.
"""
import numpy as np
import pytest

import workloads as WL


def N1(r):
    r = np.abs(r)
    return np.where(r < 0.5, 0.75 - r * r, np.where(r < 1.5, 0.5 * (1.5 - r) ** 2, 0.0))


def node_positions(dim, res):
    g = np.arange(res) / res
    if dim == 2:
        X, Y = np.meshgrid(g, g, indexing="xy")
        return np.stack([X.ravel(), Y.ravel()])
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()])


def fluid_scene(dim, seed, n=40, res=16):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.35, 0.65, (dim, n))
    v = 0.3 * rng.standard_normal((dim, n))
    C = 2.0 * rng.standard_normal((dim * dim, n))
    J = 1.0 + 0.05 * rng.standard_normal((1, n))
    p = WL.params(dim, res, 2e-4, (0.3 / res) ** dim, material="fluid", E=WL.FLUID_E)
    return p, (x, v, C, J)


def test_fluid_record_sizes(orc):
    _, _, total, W = orc.layout(WL.scheme_fluid(2))
    assert total == 2 * 20 + 2 * 16 + (6 + 4 * 16) + 16 and W == 5
    _, _, total, W = orc.layout(WL.scheme_fluid_fp32(2))
    assert total == 9 * 32 and 4 * W == 36  # 2D fluid state: 36 B in FP32
    _, _, total, W = orc.layout(WL.scheme_fluid_fp32(3))
    assert total == 16 * 32
    # F and J share a slot: a scheme may not hold both
    bad = WL.scheme_fluid(2)
    bad["fields"][0] = WL.fixed("F", 8, -1.0, 1.0)
    assert not orc.validate(bad)


def test_fluid_codec_round_trip(orc):
    sc = WL.scheme_fluid(3)
    rng = np.random.default_rng(2)
    n = 500
    x, v, C, F = WL.random_state(rng, 3, n)
    J = (1.0 + 0.2 * rng.uniform(-1, 1, (1, n))).astype(np.float32)
    words, st = orc.encode(sc, x, v, C, J)
    xd, vd, Cd, Jd = orc.decode(sc, words)
    assert Jd.shape == (1, n)
    step = 1.0 / 2 ** 16
    assert np.max(np.abs(Jd - J)) <= 0.5 * step * (1 + 1e-12)
    # decode -> encode is the identity on codes
    w2, _ = orc.encode(sc, xd, vd, Cd, Jd)
    assert np.array_equal(words, w2)
    assert st["J"]["sat"] == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_fluid_p2g_brute_force(orc, dim):
    p, (x, v, C, J) = fluid_scene(dim, 3, n=12)
    res = p["grid_res"]
    dx = 1.0 / res
    gm, gmom = orc.p2g(p, x, v, C, J)
    xi = node_positions(dim, res)
    m_p = p["rho"] * p["p_vol"]
    bm = np.zeros(xi.shape[1])
    bmom = np.zeros((dim, xi.shape[1]))
    for q in range(x.shape[1]):
        tau = p["E"] * (J[0, q] - 1.0) * np.eye(dim)
        A = -p["dt"] * p["p_vol"] * 4 / dx ** 2 * tau + m_p * C[:, q].reshape(dim, dim)
        d = xi - x[:, q:q + 1]
        w = np.prod(N1(d / dx), axis=0)
        bm += w * m_p
        bmom += w * (m_p * v[:, q:q + 1] + A @ d)
    assert np.allclose(gm, bm, rtol=1e-12, atol=1e-15)
    assert np.allclose(gmom, bmom, rtol=1e-12, atol=1e-13)
    # conservation
    assert abs(gm.sum() - m_p * x.shape[1]) <= 1e-12 * m_p * x.shape[1]
    for a in range(dim):
        assert abs(gmom[a].sum() - m_p * v[a].sum()) <= 1e-12 * m_p * np.abs(v[a]).sum()


@pytest.mark.parametrize("dim", [2, 3])
def test_fluid_g2p_volume_ratio(orc, dim):
    p, (x, v, C, J) = fluid_scene(dim, 4, n=30, res=32)
    rng = np.random.default_rng(9)
    a = rng.standard_normal(dim)
    B = rng.standard_normal((dim, dim))
    gv = a[:, None] + B @ node_positions(dim, p["grid_res"])
    x1, v1, C1, J1 = orc.g2p(p, x, J, gv)
    assert J1.shape == (1, x.shape[1])
    assert np.allclose(C1, np.repeat(B.reshape(-1, 1), x.shape[1], axis=1), atol=1e-10)
    assert np.allclose(J1[0], J[0] * (1.0 + p["dt"] * np.trace(B)), rtol=1e-12, atol=1e-13)


def test_fluid_at_rest_has_no_stress(orc):
    # J = 1, v = 0, C = 0: P2G momentum is exactly zero; after the grid
    # update every node falls at g dt
    p, (x, v, C, J) = fluid_scene(2, 5, n=30)
    v[:] = 0.0
    C[:] = 0.0
    J[:] = 1.0
    gm, gmom = orc.p2g(p, x, v, C, J)
    assert np.all(gmom == 0.0)
    gvel = orc.grid_update(p, gm, gmom)
    inner = gm > 0
    assert np.allclose(gvel[1][inner], -9.8 * p["dt"])


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("field", ["x", "v", "C", "J", None])
def test_fluid_step_vjp(orc, dim, field):
    p, st = fluid_scene(dim, 20 + dim)
    s = orc.pack_state(*st)
    assert s.shape[0] == 2 * dim + dim * dim + 1
    rows = orc.field_rows(dim, "fluid")
    rng = np.random.default_rng(8)
    lam = rng.standard_normal(s.shape)
    d = np.zeros_like(s)
    if field is None:
        d = rng.standard_normal(s.shape)
    else:
        a, b = rows[field]
        d[a:b] = rng.standard_normal((b - a, s.shape[1]))
    h = 1e-6
    fd = (orc.step_exact(p, s + h * d) - orc.step_exact(p, s - h * d)) / (2 * h)
    lhs = float((lam * fd).sum())
    rhs = float((orc.step_vjp(p, s, lam) * d).sum())
    assert abs(lhs - rhs) <= 1e-6 * (abs(lhs) + abs(rhs)) + 1e-9, (lhs, rhs)


@pytest.mark.parametrize("kind,axis", [("com", 1), ("ke", 0)])
def test_fluid_trajectory_sensitivity(orc, kind, axis):
    dim = 2
    p, st = fluid_scene(dim, 31, n=30)
    s0 = orc.pack_state(*st)
    T = 10
    rows = orc.field_rows(dim, "fluid")

    def run(shift=None, h=0.0):
        s = s0.copy()
        out = []
        if shift:
            s[shift[0]:shift[1]] += h
        out.append(s)
        for _ in range(T):
            s = orc.step_exact(p, s)
            if shift:
                s[shift[0]:shift[1]] += h
            out.append(s)
        return out

    states = run()
    z, G, g = orc.adjoint(p, states, kind, axis)
    assert set(G) == {"x", "v", "C", "J"}
    h = 1e-6
    for f, r in rows.items():
        zp, _ = orc.objective(p, run(r, h)[-1], kind, axis)
        zm, _ = orc.objective(p, run(r, -h)[-1], kind, axis)
        fd = (zp - zm) / (2 * h)
        assert abs(fd - G[f]) <= 1e-3 * abs(fd) + 1e-9 * (1 + abs(z)), (f, fd, G[f])


def test_fluid_sim_checks_material(orc):
    sc = WL.dam_break(2, grid_res=32, ppc=2)
    words, _ = orc.encode(sc["scheme"], *sc["state"])
    bad = dict(sc["params"], material="elastic")
    with pytest.raises(ValueError):
        orc.Sim(sc["scheme"], bad, words)
    sim = orc.Sim(sc["scheme"], sc["params"], words)
    sim.step(3)
    x, v, C, J = orc.decode(sc["scheme"], sim.words())
    assert J.shape == (1, sc["n"]) and np.all(np.isfinite(J))
    sim.close()
