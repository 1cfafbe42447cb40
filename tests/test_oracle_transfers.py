"""Pins of the oracle's transfers and grid update against what the paper
proves (Sec. 5.2 linear momentum, Sec. 5.3 angular momentum, Sec. 5.4
one-particle stability, Sec. 5.5 affine round trip, Sec. 5.7 the lambda = 0
forms, Sec. 4.3 the CFL bound), against calculus (force = -grad of the
potential) and against a brute-force evaluation over every grid node."""
import numpy as np
import pytest

import oracle
from paper_1603_06188_amd import scenes
from tests import bruteforce as bf


def _grid(s):
    return oracle.Grid(s.dim, s.degree, s.cells, s.dx)


def _scale_l(x, v, B, m):
    """Natural magnitude of the angular-momentum sums: sum m (|x||v| + |B|)."""
    return float(np.sum(m * (np.linalg.norm(x, axis=1) * np.linalg.norm(v, axis=1)
                             + np.linalg.norm(B.reshape(len(m), -1), axis=1))))


def _lcomp(t, d):
    return t[3:6] if d == 3 else t[5:6]


CASES = [(d, k) for d in (2, 3) for k in (2, 3)]


@pytest.mark.parametrize("dim,degree", CASES)
def test_p2g_conserves_mass_momentum_and_angular_momentum(dim, degree):
    s = scenes.random_particles(60 if dim == 3 else 80, dim=dim, cells=8, degree=degree, seed=1,
                                b_sigma=0.05)
    g = _grid(s)
    out = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V)
    u = oracle.grid_update(g, out["m"], out["mv"], None, 0.0)
    tp = oracle.particle_totals(s.x, s.v, s.B, s.m)
    tg = oracle.grid_totals(g, out["m"], u["v"])
    S = _scale_l(s.x, s.v, s.B, s.m)
    assert tg[7] == pytest.approx(tp[7], rel=1e-14)
    np.testing.assert_allclose(tg[:3], tp[:3], atol=1e-13 * S)
    np.testing.assert_allclose(_lcomp(tg, dim), _lcomp(tp, dim), atol=1e-13 * S)
    # the B term of the particle angular momentum is needed (Sec. 5.3)
    t_noB = oracle.particle_totals(s.x, s.v, None, s.m)
    assert np.max(np.abs(_lcomp(t_noB, dim) - _lcomp(tg, dim))) > 1e-6 * S


@pytest.mark.parametrize("dim,degree", CASES)
def test_force_sums_and_torques_vanish(dim, degree):
    """Sum_i f_i = 0 (Sec. 5.2) and sum_i x_i x f_i = 0 at lambda = 0 (Sec. 5.3)."""
    s = scenes.random_particles(40, dim=dim, cells=8, degree=degree, seed=2)
    g = _grid(s)
    out = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam)
    f = out["f"]
    scale = np.abs(f).sum()
    assert scale > 0
    np.testing.assert_allclose(f.sum(axis=0), 0.0, atol=1e-13 * scale)
    xi = g.node_positions()
    if dim == 2:
        torque = np.sum(xi[:, 0] * f[:, 1] - xi[:, 1] * f[:, 0])
    else:
        torque = np.cross(xi, f).sum(axis=0)
    np.testing.assert_allclose(torque, 0.0, atol=1e-13 * scale)


def _potential_at(g, s, xt_minus_x):
    """Phi(x~) = sum_p V_p Psi((I + sum_i (x~_i - x_i) grad w_ip^T) F_p^n)."""
    Fn = np.empty_like(s.F)
    for p in range(s.n):
        nodes, w, gw = oracle.weights(g, s.x[p])
        G = np.eye(s.dim) + xt_minus_x[nodes].T @ gw
        Fn[p] = G @ s.F[p]
    return oracle.potential(Fn, s.V, s.mu, s.lam)


@pytest.mark.parametrize("dim,degree", [(2, 2), (3, 2), (3, 3)])
def test_force_is_minus_gradient_of_potential(dim, degree):
    """f_i = -dPhi/dx~_i at x~ = x (the energy-based force of Sec. 3.3; this
    fixes the sign that the printed formula drops)."""
    s = scenes.random_particles(6, dim=dim, cells=6, degree=degree, seed=3, f_sigma=0.15)
    g = _grid(s)
    out = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam)
    f = out["f"]
    nn = g.node_count
    order = np.argsort(-np.abs(f).sum(axis=1))[:8]
    h = 1e-6
    for i in order:
        for a in range(dim):
            dxt = np.zeros((nn, dim))
            dxt[i, a] = h
            fd = (_potential_at(g, s, dxt) - _potential_at(g, s, -dxt)) / (2 * h)
            assert f[i, a] == pytest.approx(-fd, rel=1e-5, abs=1e-8 * np.abs(f).max())


def test_stretched_block_contracts():
    """A block stretched along x (F = diag(1.1, 1, 1)) is pulled back: grid
    forces on its +x half point to -x and on its -x half to +x."""
    s = scenes.cube3d(cells=16, lo=0.25, hi=0.75, precision="fp64", steps=1)
    s.F[:] = np.diag([1.1, 1.0, 1.0])
    g = _grid(s)
    f = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam)["f"]
    xi = g.node_positions()
    assert f[xi[:, 0] > 0.5, 0].sum() < 0
    assert f[xi[:, 0] < 0.5, 0].sum() > 0


@pytest.mark.parametrize("dim,degree", CASES)
def test_g2p_and_whole_step_conserve_momenta(dim, degree):
    """p^{P,n+1} = p~^{G,n+1} = p^{P,n}, l^{P,n+1} = l~^{G,n+1} = l^{P,n}
    with forces and no gravity or walls (Sec. 5.2, 5.3)."""
    s = scenes.random_particles(50, dim=dim, cells=8, degree=degree, seed=4, b_sigma=0.05)
    g = _grid(s)
    out = oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, dt=2e-3)
    t0 = oracle.particle_totals(s.x, s.v, s.B, s.m)
    tg = oracle.grid_totals(g, out["m"], out["vt"], out["xt"])
    t1 = oracle.particle_totals(out["x_new"], out["v_new"], out["B_new"], s.m)
    S = _scale_l(s.x, s.v, s.B, s.m) + _scale_l(out["x_new"], out["v_new"], out["B_new"], s.m)
    np.testing.assert_allclose(t1[:3], tg[:3], atol=1e-13 * S)
    np.testing.assert_allclose(t1[:3], t0[:3], atol=1e-13 * S)
    np.testing.assert_allclose(_lcomp(t1, dim), _lcomp(tg, dim), atol=1e-13 * S)
    np.testing.assert_allclose(_lcomp(t1, dim), _lcomp(t0, dim), atol=1e-13 * S)


@pytest.mark.parametrize("dim,degree", CASES)
def test_lambda0_forms(dim, degree):
    """Sec. 5.7: at lambda = 0 the general B update equals
    sum_i w vt_i (x_i - x_p)^T and sum_i w x~_i equals x_p + dt v_p^{n+1}."""
    s = scenes.random_particles(30, dim=dim, cells=8, degree=degree, seed=5)
    g = _grid(s)
    dt = 3e-3
    out = oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, dt=dt)
    xi = g.node_positions()
    for p in range(s.n):
        nodes, w, _ = oracle.weights(g, s.x[p])
        r = xi[nodes] - s.x[p]
        B0 = (w[:, None] * out["vt"][nodes]).T @ r
        np.testing.assert_allclose(out["B_new"][p], B0, atol=1e-15)
        np.testing.assert_allclose(out["x_new"][p], s.x[p] + dt * out["v_new"][p], atol=1e-15)


@pytest.mark.parametrize("dim,degree", CASES)
def test_affine_round_trip(dim, degree):
    """Sec. 5.5: v_p = v + C x_p, B_p = C D_p is reproduced on the grid
    (v_i = v + C x_i) and returned unchanged at dt = 0."""
    rng = np.random.default_rng(6)
    s = scenes.random_particles(70, dim=dim, cells=8, degree=degree, seed=6, model=0)
    vbar = rng.normal(size=dim)
    C = rng.normal(size=(dim, dim))
    k = (0.25 if degree == 2 else 1.0 / 3.0) * s.dx ** 2
    v = vbar[None] + s.x @ C.T
    B = np.broadcast_to(C * k, (s.n, dim, dim)).copy()
    g = _grid(s)
    out = oracle.step(g, s.x, v, B, s.F, s.m, s.V, 0, dt=0.0)
    xi = g.node_positions()
    has = out["m"] > 0
    np.testing.assert_allclose(out["v"][has], vbar[None] + xi[has] @ C.T, atol=1e-13)
    np.testing.assert_allclose(out["v_new"], v, atol=1e-13)
    np.testing.assert_allclose(out["B_new"], B, atol=1e-15)
    np.testing.assert_allclose(out["x_new"], s.x, atol=1e-15)
    # with dt > 0 (no forces) the grid field is still affine, so
    # F^{n+1} = (I + dt C) F^n exactly
    dt = 1e-2
    out = oracle.step(g, s.x, v, B, s.F, s.m, s.V, 0, dt=dt)
    np.testing.assert_allclose(out["F_new"], (np.eye(dim) + dt * C)[None] @ s.F, atol=1e-13)


@pytest.mark.parametrize("dim,degree", CASES)
def test_one_particle_stability(dim, degree):
    """Sec. 5.4: a lone force-free particle keeps v and B and moves by dt v."""
    rng = np.random.default_rng(8)
    for trial in range(5):
        x = 0.35 + 0.3 * rng.random(dim)
        v = rng.normal(size=dim)
        B = 0.01 * rng.normal(size=(dim, dim))
        s = scenes.single_particle(x, v, B, dim=dim, cells=8, degree=degree)
        g = _grid(s)
        dt = 1e-2
        out = oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, 0, dt=dt)
        np.testing.assert_allclose(out["v_new"][0], v, atol=1e-14)
        np.testing.assert_allclose(out["B_new"][0], B, atol=1e-15)
        np.testing.assert_allclose(out["x_new"][0], s.x[0] + dt * v, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_free_fall_closed_form(dim):
    """No stress, gravity g, no walls: p gains dt M g and l gains
    dt (sum m_p x_p) x g in one step (partition of unity and linear
    reproduction make the grid mass moments equal the particle ones)."""
    s = scenes.random_particles(40, dim=dim, cells=8, degree=2, seed=9, b_sigma=0.05)
    g = _grid(s)
    grav = np.zeros(3)
    grav[dim - 1] = -9.8
    dt = 1e-3
    out = oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, 0, dt=dt, gravity=grav)
    t0 = oracle.particle_totals(s.x, s.v, s.B, s.m)
    t1 = oracle.particle_totals(out["x_new"], out["v_new"], out["B_new"], s.m)
    M = s.m.sum()
    S = _scale_l(s.x, s.v, s.B, s.m)
    np.testing.assert_allclose(t1[:3] - t0[:3], dt * M * grav, atol=1e-13 * S)
    mx = np.zeros(3)
    mx[:dim] = (s.m[:, None] * s.x).sum(axis=0)
    dl = dt * np.cross(mx, grav)
    np.testing.assert_allclose(t1[3:6] - t0[3:6], dl, atol=1e-13 * S)


@pytest.mark.parametrize("dim,degree", CASES)
def test_p2g_matches_brute_force_over_all_nodes(dim, degree):
    s = scenes.random_particles(4, dim=dim, cells=6, degree=degree, seed=10, b_sigma=0.1)
    g = _grid(s)
    out = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V)
    idx, gm, gmv = bf.p2g_all_nodes(degree, s.cells, s.dx, s.x, s.v, s.B, s.m)
    lin = bf.ij_to_oracle(idx, s.cells)
    np.testing.assert_allclose(out["m"][lin], gm, atol=1e-14)
    np.testing.assert_allclose(out["mv"][lin], gmv, atol=1e-13)


@pytest.mark.parametrize("dim,degree", CASES)
def test_cfl_bound_on_grid_velocity(dim, degree):
    """Sec. 4.3: |v_i| <= max_p (|v_p| + (6 sqrt(d)/dx) |B_p|_F), and the CFL
    step moves the fastest such velocity by exactly nu dx."""
    s = scenes.random_particles(60, dim=dim, cells=8, degree=degree, seed=12, b_sigma=0.1)
    g = _grid(s)
    out = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V)
    u = oracle.grid_update(g, out["m"], out["mv"], None, 0.0)
    bound = np.max(np.linalg.norm(s.v, axis=1)
                   + 6 * np.sqrt(dim) / s.dx * np.linalg.norm(s.B.reshape(s.n, -1), axis=1))
    assert np.linalg.norm(u["v"], axis=1).max() <= bound * (1 + 1e-14)
    assert oracle.cfl_dt(s.dx, s.v, s.B, nu=0.5) * bound == pytest.approx(0.5 * s.dx, rel=1e-14)


def test_empty_nodes_and_sticky_band():
    s = scenes.random_particles(20, dim=3, cells=8, degree=2, seed=13)
    g = _grid(s)
    out = oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, dt=1e-3,
                      gravity=(0, 0, -9.8), band=(0, 0, 0, 0, 3, 2))
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in g.nodes], indexing="ij"), -1).reshape(-1, 3)
    lin = bf.ij_to_oracle(idx, s.cells)
    iz = np.empty(g.node_count, dtype=int)
    iz[lin] = idx[:, 2]
    in_band = (iz < 3) | (iz > s.cells[2] - 2)
    assert np.all(out["vt"][in_band] == 0.0)
    assert np.all(out["vt"][out["m"] == 0.0] == 0.0)
    np.testing.assert_array_equal(out["xt"][in_band], g.node_positions()[in_band])
    free = (~in_band) & (out["m"] > 0)
    assert np.all(np.abs(out["vt"][free]).sum(axis=1) > 0)
