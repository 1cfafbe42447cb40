"""Pins of the oracle's RPIC and PIC transfers (Sec. 2.1, Sec. 5.1, Sec. 5.6).

The oracle's RPIC transfer to particles solves omega_p = K_p^{-1} l_p with
K_p and l_p summed over the stencil; its transfer to grid reads a stored B_p
through the rotation of C_p = B_p D_p^{-1}.  The checks below come from
elsewhere:

* closed forms for linear grid fields v_i = v0 + A x_i, which the B-splines
  reproduce exactly: RPIC keeps C = skew(A), APIC C = A, PIC C = 0, and
  D_p = c dx^2 I with c = 1/4 (quadratic) or 1/3 (cubic);
* the identity that, at lambda = 0, the RPIC state is the skew part of the
  APIC one (K_p = 2 m_p c dx^2 I in 3D, 2 m_p c dx^2 about z in 2D);
* the conservation statements proved in Sec. 5.1 (both directions) and the
  exact angular momentum PIC loses on a rigid rotation, sum_p K_p omega.
"""
import numpy as np
import pytest

import oracle
from paper_1603_06188_amd import scenes

CASES = [(d, k) for d in (2, 3) for k in (2, 3)]
RPIC, PIC, APIC = oracle.TRANSFER_RPIC, oracle.TRANSFER_PIC, oracle.TRANSFER_APIC


def _grid(s):
    return oracle.Grid(s.dim, s.degree, s.cells, s.dx)


def _dc(s):
    return (0.25 if s.degree == 2 else 1.0 / 3.0) * s.dx ** 2


def _lcomp(t, d):
    return t[3:6] if d == 3 else t[5:6]


def _rigid(dim, rng):
    """A random rigid velocity gradient (omega^*) and its angular velocity."""
    if dim == 3:
        w = rng.normal(size=3)
        W = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    else:
        w = rng.normal(size=1)
        W = np.array([[0.0, -w[0]], [w[0], 0.0]])
    return W, w


def _linear_field(g, vbar, A, dt):
    xi = g.node_positions()
    vt = vbar[None] + xi @ A.T
    return vt, xi + dt * vt


@pytest.mark.parametrize("dim,degree", CASES)
def test_rigid_grid_field(dim, degree):
    """v_i = v0 + omega x x_i: RPIC and APIC return v_p = v0 + omega x x_p and
    B_p = omega^* D_p; PIC returns the same v_p and B_p = 0."""
    rng = np.random.default_rng(11)
    s = scenes.random_particles(40, dim=dim, cells=8, degree=degree, seed=11)
    g = _grid(s)
    W, _ = _rigid(dim, rng)
    vbar = rng.normal(size=dim)
    dt = 1e-2
    vt, xt = _linear_field(g, vbar, W, dt)
    want_v = vbar[None] + s.x @ W.T
    for tr, want_B in ((RPIC, W * _dc(s)), (APIC, W * _dc(s)), (PIC, np.zeros((dim, dim)))):
        out = oracle.g2p(g, s.x, s.F, vt, xt, transfer=tr)
        np.testing.assert_allclose(out["v"], want_v, atol=1e-13)
        np.testing.assert_allclose(out["B"], np.broadcast_to(want_B, out["B"].shape), atol=1e-14)
        np.testing.assert_allclose(out["x"], s.x + dt * want_v, atol=1e-14)


@pytest.mark.parametrize("dim,degree", CASES)
def test_linear_grid_field(dim, degree):
    """v_i = v0 + A x_i with a general A: APIC keeps A, RPIC its skew part,
    PIC nothing; F advances by (I + dt A) in every variant."""
    rng = np.random.default_rng(12)
    s = scenes.random_particles(40, dim=dim, cells=8, degree=degree, seed=12)
    g = _grid(s)
    A = rng.normal(size=(dim, dim))
    vbar = rng.normal(size=dim)
    dt = 1e-2
    vt, xt = _linear_field(g, vbar, A, dt)
    for tr, C in ((APIC, A), (RPIC, 0.5 * (A - A.T)), (PIC, np.zeros((dim, dim)))):
        out = oracle.g2p(g, s.x, s.F, vt, xt, transfer=tr)
        np.testing.assert_allclose(out["B"], np.broadcast_to(C * _dc(s), out["B"].shape), atol=1e-14)
        np.testing.assert_allclose(out["F"], (np.eye(dim) + dt * A)[None] @ s.F, atol=1e-13)


@pytest.mark.parametrize("dim,degree", CASES)
def test_rpic_state_is_skew_part_of_apic_state(dim, degree):
    """Any grid field: B_RPIC = (B_APIC - B_APIC^T) / 2, v, x and F agree."""
    rng = np.random.default_rng(13)
    s = scenes.random_particles(50, dim=dim, cells=8, degree=degree, seed=13)
    g = _grid(s)
    vt = rng.normal(size=(g.node_count, dim))
    xt = g.node_positions() + 1e-2 * vt
    a = oracle.g2p(g, s.x, s.F, vt, xt, transfer=APIC)
    r = oracle.g2p(g, s.x, s.F, vt, xt, transfer=RPIC)
    p = oracle.g2p(g, s.x, s.F, vt, xt, transfer=PIC)
    skew = 0.5 * (a["B"] - np.swapaxes(a["B"], 1, 2))
    scale = float(np.abs(a["B"]).max())
    np.testing.assert_allclose(r["B"], skew, atol=1e-14 * scale)
    assert float(np.abs(a["B"] - skew).max()) > 1e-3 * scale  # the field has a symmetric part
    for key in ("v", "x", "F"):
        np.testing.assert_array_equal(r[key], a[key])
        np.testing.assert_array_equal(p[key], a[key])
    assert not p["B"].any()


@pytest.mark.parametrize("dim,degree", CASES)
def test_rpic_p2g_reads_the_rotation_of_b(dim, degree):
    """RPIC's transfer to grid uses only the rotation of C_p = B_p D_p^{-1}:
    a general B_p gives the grid of its skew part under APIC; PIC gives the
    grid of B_p = 0."""
    s = scenes.random_particles(50, dim=dim, cells=8, degree=degree, seed=14, b_sigma=0.1)
    g = _grid(s)
    skew = 0.5 * (s.B - np.swapaxes(s.B, 1, 2))
    r = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V, transfer=RPIC)
    a = oracle.p2g(g, s.x, s.v, skew, s.F, s.m, s.V, transfer=APIC)
    p = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V, transfer=PIC)
    z = oracle.p2g(g, s.x, s.v, np.zeros_like(s.B), s.F, s.m, s.V, transfer=APIC)
    scale = float(np.abs(a["mv"]).max())
    np.testing.assert_allclose(r["mv"], a["mv"], atol=1e-14 * scale)
    np.testing.assert_allclose(p["mv"], z["mv"], atol=1e-14 * scale)
    np.testing.assert_array_equal(r["m"], a["m"])


@pytest.mark.parametrize("dim,degree", CASES)
def test_rpic_conserves_momenta_both_ways(dim, degree):
    """Sec. 5.1: after P2G p^P = p^G and l^P = l^G (l^P = sum x_p x m_p v_p +
    K_p omega_p, which the B term of the particle totals evaluates); after
    G2P the same for the updated grid state, at x_i and at x~_i."""
    rng = np.random.default_rng(15)
    s = scenes.random_particles(50, dim=dim, cells=8, degree=degree, seed=15, b_sigma=0.1)
    g = _grid(s)
    out = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V, transfer=RPIC)
    u = oracle.grid_update(g, out["m"], out["mv"], None, 0.0)
    tp = oracle.particle_totals(s.x, s.v, s.B, s.m)
    tg = oracle.grid_totals(g, out["m"], u["v"])
    S = float(np.sum(s.m * (np.linalg.norm(s.x, axis=1) * np.linalg.norm(s.v, axis=1) + 1.0)))
    np.testing.assert_allclose(tg[:3], tp[:3], atol=1e-13 * S)
    np.testing.assert_allclose(_lcomp(tg, dim), _lcomp(tp, dim), atol=1e-13 * S)
    # an arbitrary updated grid field on the nodes with mass
    vt = np.where(out["m"][:, None] > 0, rng.normal(size=(g.node_count, dim)), 0.0)
    dt = 1e-2
    xt = g.node_positions() + dt * vt
    r = oracle.g2p(g, s.x, s.F, vt, xt, transfer=RPIC)
    tg_n = oracle.grid_totals(g, out["m"], vt)
    tg_t = oracle.grid_totals(g, out["m"], vt, xt)
    S = float(np.sum(out["m"] * (np.linalg.norm(g.node_positions(), axis=1) + 1.0) * np.linalg.norm(vt, axis=1)))
    for tp1 in (oracle.particle_totals(s.x, r["v"], r["B"], s.m),
                oracle.particle_totals(r["x"], r["v"], r["B"], s.m)):
        np.testing.assert_allclose(tp1[:3], tg_n[:3], atol=1e-13 * S)
        np.testing.assert_allclose(_lcomp(tp1, dim), _lcomp(tg_n, dim), atol=1e-13 * S)
        np.testing.assert_allclose(_lcomp(tp1, dim), _lcomp(tg_t, dim), atol=1e-13 * S)
    # PIC keeps the linear momentum and loses angular momentum here
    p = oracle.g2p(g, s.x, s.F, vt, xt, transfer=PIC)
    tpic = oracle.particle_totals(s.x, p["v"], p["B"], s.m)
    np.testing.assert_allclose(tpic[:3], tg_n[:3], atol=1e-13 * S)
    assert float(np.abs(_lcomp(tpic, dim) - _lcomp(tg_n, dim)).max()) > 1e-4 * S


@pytest.mark.parametrize("dim,degree", CASES)
def test_pic_loses_sum_of_k_omega_on_rigid_rotation(dim, degree):
    """Grid in rigid rotation with the masses of a P2G: the PIC particles
    carry l^G - sum_p K_p omega with K_p = 2 m_p c dx^2 (about omega)."""
    rng = np.random.default_rng(16)
    s = scenes.random_particles(40, dim=dim, cells=8, degree=degree, seed=16)
    g = _grid(s)
    out = oracle.p2g(g, s.x, s.v, s.B, s.F, s.m, s.V)
    W, w = _rigid(dim, rng)
    vt, xt = _linear_field(g, np.zeros(dim), W, 0.0)
    vt = np.where(out["m"][:, None] > 0, vt, 0.0)
    lg = _lcomp(oracle.grid_totals(g, out["m"], vt), dim)
    p = oracle.g2p(g, s.x, s.F, vt, xt, transfer=PIC)
    lp = _lcomp(oracle.particle_totals(s.x, p["v"], p["B"], s.m), dim)
    loss = 2.0 * _dc(s) * float(s.m.sum()) * w
    np.testing.assert_allclose(lg - lp, loss, rtol=1e-12)
    r = oracle.g2p(g, s.x, s.F, vt, xt, transfer=RPIC)
    np.testing.assert_allclose(_lcomp(oracle.particle_totals(s.x, r["v"], r["B"], s.m), dim), lg, rtol=1e-12)


@pytest.mark.parametrize("dim,degree", CASES)
def test_whole_step_per_transfer(dim, degree):
    """Full steps with forces: RPIC conserves p and l like APIC; PIC
    conserves p only; all three give the same positions and F."""
    s = scenes.random_particles(50, dim=dim, cells=8, degree=degree, seed=17, b_sigma=0.05)
    g = _grid(s)
    dt = 2e-3
    res = {tr: oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, 1, s.mu, s.lam, dt=dt, transfer=tr)
           for tr in (APIC, RPIC, PIC)}
    for tr, out in res.items():
        B_in = {APIC: s.B, RPIC: 0.5 * (s.B - np.swapaxes(s.B, 1, 2)), PIC: np.zeros_like(s.B)}[tr]
        t0 = oracle.particle_totals(s.x, s.v, B_in, s.m)
        t1 = oracle.particle_totals(out["x_new"], out["v_new"], out["B_new"], s.m)
        tg = oracle.grid_totals(g, out["m"], out["vt"], out["xt"])
        S = float(np.sum(s.m * (np.linalg.norm(s.x, axis=1) * np.linalg.norm(s.v, axis=1) + 1.0)))
        np.testing.assert_allclose(t1[:3], t0[:3], atol=1e-13 * S)
        np.testing.assert_allclose(tg[:3], t0[:3], atol=1e-13 * S)
        if tr != PIC:
            np.testing.assert_allclose(_lcomp(t1, dim), _lcomp(t0, dim), atol=1e-13 * S)
        else:
            assert float(np.abs(_lcomp(t1, dim) - _lcomp(tg, dim)).max()) > 1e-9 * S
        assert not (tr == PIC and out["B_new"].any())
