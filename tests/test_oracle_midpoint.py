"""Pins of the oracle's implicit midpoint step (Sec. 3.3 at lambda = 1/2,
Sec. 4.1, 4.2) against what the paper and the mathematics fix, independently
of the oracle's own formulas:

* the stress differential against central differences of the stress;
* the grid force against central differences of the potential energy
  (f_i = -dPhi/dx_i), and the force-derivative product against central
  differences of the force;
* the converged step against the midpoint equations in their two-equation
  form, before the elimination of xt (Sec. 4.1);
* conservation of linear and angular momentum by the whole step (the
  lambda family conserves both, Sec. 3.3; the proof in Sec. 5);
* constant acceleration integrated exactly (model without force);
* the midpoint and the symplectic-Euler step agree to O(dt^2);
* sticky nodes do not move;
* an implosion whose full Newton steps would invert elements: the line
  search halves them (an inverted trial has infinite energy) and the step
  still solves the midpoint equations.
"""
import numpy as np
import pytest

import oracle
from paper_1603_06188_amd import scenes


def ogrid(s):
    return oracle.Grid(s.dim, s.degree, s.cells, s.dx)


def _scene(dim=3, degree=2, n=400, seed=3, cells=8, **kw):
    args = dict(precision="fp64", vel_sigma=0.5, f_sigma=0.05, b_sigma=0.05, model=1)
    args.update(kw)
    return scenes.random_particles(n, dim=dim, cells=cells, degree=degree, seed=seed, **args)


def _fd(fun, x, h):
    return (fun(x + h) - fun(x - h)) / (2 * h)


@pytest.mark.parametrize("d", [2, 3])
def test_stress_differential_matches_differences_of_the_stress(d):
    rng = np.random.default_rng(1)
    mu, lam = 3.0, 5.0
    for _ in range(5):
        F = np.eye(d) + 0.2 * rng.standard_normal((d, d))
        if np.linalg.det(F) <= 0.2:
            continue
        dF = rng.standard_normal((d, d))
        fd = _fd(lambda t: oracle.neo_hookean_P(F + t * dF, mu, lam), 0.0, 1e-6)
        got = oracle.neo_hookean_dP(F, mu, lam, dF)
        np.testing.assert_allclose(got, fd, rtol=1e-7, atol=1e-8 * np.abs(fd).max())


@pytest.mark.parametrize("dim,degree", [(3, 2), (2, 3)])
def test_force_is_minus_the_energy_gradient(dim, degree):
    s = _scene(dim, degree, n=150, cells=6)
    g = ogrid(s)
    rng = np.random.default_rng(2)
    u = 0.01 * s.dx * rng.standard_normal((g.node_count, dim))
    f, _ = oracle.forces_at(g, s.x, s.F, s.V, s.mu, s.lam, u)
    busy = np.argsort(-np.abs(f).sum(axis=1))[:6]
    h = 1e-6 * s.dx
    for i in busy:
        for a in range(dim):
            def phi(t):
                uu = u.copy()
                uu[i, a] += t
                return oracle.forces_at(g, s.x, s.F, s.V, s.mu, s.lam, uu)[1]
            fd = -_fd(phi, 0.0, h)
            assert abs(f[i, a] - fd) <= 1e-6 * np.abs(f).max(), (i, a, f[i, a], fd)


@pytest.mark.parametrize("dim,degree", [(3, 3), (2, 2)])
def test_force_differential_matches_differences_of_the_force(dim, degree):
    s = _scene(dim, degree, n=150, cells=6)
    g = ogrid(s)
    rng = np.random.default_rng(3)
    u = 0.01 * s.dx * rng.standard_normal((g.node_count, dim))
    du = rng.standard_normal((g.node_count, dim))
    got = oracle.force_differential(g, s.x, s.F, s.V, s.mu, s.lam, u, du)
    h = 1e-6 * s.dx
    fd = _fd(lambda t: oracle.forces_at(g, s.x, s.F, s.V, s.mu, s.lam, u + t * du)[0], 0.0, h)
    assert np.abs(got - fd).max() <= 1e-6 * np.abs(fd).max()


@pytest.mark.parametrize("dim,degree", [(3, 2), (2, 3)])
def test_step_solves_the_midpoint_equations(dim, degree):
    """m_i (vt_i - v_i) = dt f_i((x_i + xt_i)/2) + dt m_i g with
    xt_i = x_i + dt (v_i + vt_i)/2, at every free node."""
    s = _scene(dim, degree, n=500, cells=8, seed=4)
    g = ogrid(s)
    r = oracle.midpoint_step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, s.dt, s.gravity, s.band)
    assert r["stats"]["newton"] >= 2 and r["stats"]["halvings"] == 0
    xi = g.node_positions()
    u = 0.5 * (r["xt"] - xi)
    f, _ = oracle.forces_at(g, s.x, s.F, s.V, s.mu, s.lam, u)
    free = r["m"] > 0
    grav = np.asarray(s.gravity[:dim])
    lhs = r["m"][free, None] * (r["vt"][free] - r["v"][free])
    rhs = s.dt * f[free] + s.dt * r["m"][free, None] * grav
    scale = np.abs(rhs).max()
    assert np.abs(lhs - rhs).max() <= 1e-11 * scale
    np.testing.assert_allclose(r["xt"], xi + s.dt * 0.5 * (r["v"] + r["vt"]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim,degree", [(3, 2), (3, 3), (2, 2)])
def test_step_conserves_linear_and_angular_momentum(dim, degree):
    s = _scene(dim, degree, n=500, cells=8, seed=5)
    g = ogrid(s)
    x, v, B, F = s.x, s.v, s.B, s.F
    t0 = oracle.particle_totals(x, v, B, s.m)
    for _ in range(3):
        r = oracle.midpoint_step(g, x, v, B, F, s.m, s.V, 1, s.mu, s.lam, 4 * s.dt)
        x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
    t1 = oracle.particle_totals(x, v, B, s.m)
    S = float(np.sum(s.m * (np.linalg.norm(s.x, axis=1) * np.linalg.norm(s.v, axis=1) + np.linalg.norm(s.v, axis=1))))
    assert np.abs(t1[:6] - t0[:6]).max() <= 1e-11 * S, (t1[:6], t0[:6])


def test_constant_acceleration_is_integrated_exactly():
    """No force, uniform v, B = 0: x' = x + dt v + dt^2 g / 2, v' = v + dt g,
    B' = 0 and F' = F (the midpoint rule on a constant force)."""
    s = _scene(3, 2, n=300, cells=8, seed=6, vel_sigma=0.0, b_sigma=0.0)
    v0 = np.array([0.3, -0.2, 0.1])
    gvec = np.array([0.5, -9.8, 1.5])
    dt = 0.01
    v = np.tile(v0, (s.n, 1))
    B = np.zeros_like(s.B)
    g = ogrid(s)
    r = oracle.midpoint_step(g, s.x, v, B, s.F, s.m, s.V, 0, dt=dt, gravity=gvec)
    np.testing.assert_allclose(r["x_new"], s.x + dt * v0 + 0.5 * dt * dt * gvec, rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["v_new"], np.tile(v0 + dt * gvec, (s.n, 1)), rtol=0, atol=1e-14)
    assert np.abs(r["B_new"]).max() <= 1e-15
    np.testing.assert_allclose(r["F_new"], s.F, rtol=0, atol=1e-15)


def test_midpoint_and_symplectic_euler_agree_to_second_order():
    """vt differs between the two grid updates by dt (f(x_hat) - f(x)) / m =
    O(dt^2): halving dt divides the particle-velocity difference by ~4."""
    s = _scene(3, 2, n=400, cells=8, seed=7, vel_sigma=1.0)
    g = ogrid(s)
    diffs = []
    for dt in (2e-3, 1e-3, 5e-4):
        mid = oracle.midpoint_step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, dt)
        exp = oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, dt)
        diffs.append(np.abs(mid["v_new"] - exp["v_new"]).max())
    for a, b in zip(diffs, diffs[1:]):
        assert 3.5 < a / b < 4.5, diffs


def test_sticky_band_nodes_stay_put():
    s = _scene(3, 2, n=600, cells=8, seed=8, margin=1.0, vel_sigma=1.0)
    g = ogrid(s)
    band = [2, 2, 2, 2, 2, 2]
    r = oracle.midpoint_step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, s.dt, s.gravity, band)
    sticky = oracle.band_mask(g, band)
    assert (sticky & (r["m"] > 0)).any()
    assert not r["vt"][sticky].any()
    np.testing.assert_array_equal(r["xt"][sticky], g.node_positions()[sticky])


def implosion_scene(E=1e2, rate=10.0, dt=0.1):
    """2D particles collapsing toward the centre (v = -rate (x - c)) on a
    soft material with a large step: the first Newton steps overshoot into
    inverted elements."""
    import dataclasses
    s = _scene(2, 2, n=300, cells=8, seed=3, vel_sigma=0.5, f_sigma=0.05, E=E)
    s = s.with_state(v=-rate * (s.x - np.array([0.5, 0.5])))
    return dataclasses.replace(s, dt=dt)


def test_line_search_halves_inverted_trials_and_the_step_still_solves():
    s = implosion_scene()
    g = ogrid(s)
    r = oracle.midpoint_step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, s.dt, newton_tol=1e-10,
                             cg_tol=1e-8, max_newton=30, max_cg=500)
    st = r["stats"]
    assert st["halvings"] > 0
    assert st["res"] <= 1e-10 * st["res0"]
    xi = g.node_positions()
    f, _ = oracle.forces_at(g, s.x, s.F, s.V, s.mu, s.lam, 0.5 * (r["xt"] - xi))
    free = r["m"] > 0
    lhs = r["m"][free, None] * (r["vt"][free] - r["v"][free])
    rhs = s.dt * f[free]
    assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(rhs).max()
    assert (np.linalg.det(r["F_new"]) > 0).all()

