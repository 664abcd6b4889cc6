"""Pins of the oracle adjoint (Sec. 6, Eqs. 12-13) by central finite
differences of the FP64 substep, and of the accumulated sensitivities of
Eq. 8 by finite differences of the whole trajectory (no GPU).

The quantization error is an additive perturbation of the stored state, so
d z / d e_t = lambda_t, the adjoint of the state stored at step t.  Adding
h to every stored component of field f at every store (t = 0..T) changes
z by h * G_f + O(h^2), G_f = sum_t sum_i lambda_{t,f,i}.
"""
import numpy as np
import pytest

import workloads as WL


def scene(dim, seed, n=60, res=24, deform=0.08):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.35, 0.65, (dim, n))
    v = 0.3 * rng.standard_normal((dim, n))
    C = 2.0 * rng.standard_normal((dim * dim, n))
    F = np.zeros((dim * dim, n))
    for a in range(dim):
        F[a * dim + a] = 1.0
    F += deform * rng.standard_normal((dim * dim, n))
    p = WL.params(dim, res, 2e-4, (0.3 / res) ** dim)
    return p, (x, v, C, F)


@pytest.mark.parametrize("dim", [2, 3])
def test_step_vjp_matches_central_differences(orc, dim):
    p, st = scene(dim, 1 + dim)
    s = orc.pack_state(*st)
    rng = np.random.default_rng(7)
    for trial in range(4):
        lam = rng.standard_normal(s.shape)
        d = rng.standard_normal(s.shape)
        h = 1e-6
        fd = (orc.step_exact(p, s + h * d) - orc.step_exact(p, s - h * d)) / (2 * h)
        lhs = float((lam * fd).sum())
        rhs = float((orc.step_vjp(p, s, lam) * d).sum())
        assert abs(lhs - rhs) <= 1e-6 * (abs(lhs) + abs(rhs)) + 1e-9, (trial, lhs, rhs)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("field", ["x", "v", "C", "F"])
def test_step_vjp_per_field(orc, dim, field):
    """Each field's block of the Jacobian on its own (catches a term that
    cancels in a random mixture)."""
    p, st = scene(dim, 11 + dim)
    s = orc.pack_state(*st)
    rows = orc.field_rows(dim)
    a, b = rows[field]
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(s.shape)
    d = np.zeros_like(s)
    d[a:b] = rng.standard_normal((b - a, s.shape[1]))
    h = 1e-6
    fd = (orc.step_exact(p, s + h * d) - orc.step_exact(p, s - h * d)) / (2 * h)
    lhs = float((lam * fd).sum())
    rhs = float((orc.step_vjp(p, s, lam) * d).sum())
    assert abs(lhs - rhs) <= 1e-6 * (abs(lhs) + abs(rhs)) + 1e-9


def trajectory(orc, p, s0, T, shift=None, h=0.0):
    """Exact FP64 trajectory; optionally adds h to every stored component of
    the rows `shift` at every store (t = 0..T)."""
    states = []
    s = s0.copy()
    if shift is not None:
        s[shift[0]:shift[1]] += h
    states.append(s)
    for _ in range(T):
        s = orc.step_exact(p, s)
        if shift is not None:
            s[shift[0]:shift[1]] += h
        states.append(s)
    return states


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind,axis", [("com", 1), ("ke", 0)])
def test_trajectory_sensitivity_matches_fd(orc, dim, kind, axis):
    p, st = scene(dim, 21 + dim, n=40)
    s0 = orc.pack_state(*st)
    T = 12
    states = trajectory(orc, p, s0, T)
    z, G, g = orc.adjoint(p, states, kind, axis)
    rows = orc.field_rows(dim)
    h = 1e-6
    for f, r in rows.items():
        zp, _ = orc.objective(p, trajectory(orc, p, s0, T, r, h)[-1], kind, axis)
        zm, _ = orc.objective(p, trajectory(orc, p, s0, T, r, -h)[-1], kind, axis)
        fd = (zp - zm) / (2 * h)
        assert abs(fd - G[f]) <= 1e-3 * abs(fd) + 1e-9 * (1 + abs(z)), (f, fd, G[f])
        assert g[f] >= 0.0


def test_objective_gradients(orc):
    p, st = scene(3, 5)
    s = orc.pack_state(*st)
    z, lam = orc.objective(p, s, "com", 2)
    assert np.isclose(z, st[0][2].mean())
    assert np.allclose(lam[2], 1.0 / s.shape[1]) and np.count_nonzero(lam) == s.shape[1]
    z, lam = orc.objective(p, s, "ke", 0)
    m = p["rho"] * p["p_vol"]
    assert np.isclose(z, 0.5 * m * (st[1] ** 2).sum())
    assert np.allclose(lam[3:6], m * st[1])


@pytest.mark.parametrize("dim", [2, 3])
def test_centre_of_mass_invariants(orc, dim):
    """Away from the walls a uniform shift of every stored position moves the
    centre of mass by the same amount (quadratic B-splines reproduce affine
    velocity fields), and internal forces and the affine term conserve
    momentum, so C and F do not move it: G_x = T + 1 along the axis, 0 across
    it, and G_C = G_F = 0 up to round-off."""
    p, st = scene(dim, 40 + dim, n=50)
    s0 = orc.pack_state(*st)
    T = 6
    states = trajectory(orc, p, s0, T)
    rows = orc.field_rows(dim)
    for axis in range(dim):
        z, G, g, A, lam0 = orc.adjoint_full(p, states, "com", axis)
        assert abs(G["x"] - (T + 1)) <= 1e-9 * (T + 1), G["x"]
        # per axis: sum over the particles of lambda_x along `axis` is 1 at every step
        assert abs(lam0[axis].sum() - 1.0) <= 1e-9
        for b in range(dim):
            if b != axis:
                assert abs(lam0[b].sum()) <= 1e-9
        for f in ("C", "F"):
            assert abs(G[f]) <= 1e-9 * A["x"], (f, G[f])
