"""Pins of the oracle's energy totals (Sec. 3.1: kinetic energy, read with
the factor 1/2 the paper's formula omits; Sec. 3.3: potential energy
Phi = sum_p V_p Psi(F_p)) against values fixed outside the oracle:

* a lone particle's 1/2 m |v|^2 written out by hand;
* the grid kinetic energy at the node of the worked example of Sec. 5.9,
  from the node mass and velocity the paper prints;
* a rigid body: 1/2 M |v_c|^2 + 1/2 omega^T I omega with I in closed form,
  for the particles and, after the transfer to grid (Sec. 3.2), for the
  grid, whose inertia is the particles' plus sum_p m_p (tr D_p I - D_p) with
  D_p = k dx^2 I (Sec. 5.6, k = 1/4 quadratic, 1/3 cubic);
* the potential: zero at rest, sum_p V_p Psi for a uniform stretch written
  out from the neo-Hookean formula, additivity over particles.
"""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "multilinear_example.json")


def test_lone_particle_kinetic_energy():
    x = np.array([[0.3, 0.7, 0.2]])
    v = np.array([[0.3, -0.4, 1.2]])
    B = np.array([[[0.5, 0.1, 0.0], [0.0, 0.2, 0.3], [0.4, 0.0, 0.1]]])
    m = np.array([2.5])
    t = oracle.particle_totals(x, v, B, m)
    # 1/2 * 2.5 * (0.09 + 0.16 + 1.44) = 2.1125, independent of x and B
    assert t[6] == pytest.approx(2.1125, rel=1e-15)
    assert t[7] == 2.5
    t2 = oracle.particle_totals(x + 5.0, v, 3 * B, m)
    assert t2[6] == t[6]


def test_grid_kinetic_energy_of_the_worked_example_of_sec_5_9():
    """Node (1,1) of the example carries mass (eps/2) m_p and velocity
    <1/(eps dx), 2/dx>; its kinetic energy is m_p (1/eps + 4 eps)/(4 dx^2)
    (printed with 1/dx; the fixture records the reading)."""
    ex = json.load(open(GOLDEN))
    assert ex["node"] == [1, 1]
    dx, mp = 0.25, 3.0
    g = oracle.Grid(2, 1, (4, 4), dx)
    node = 1 + 5 * 1
    for eps in (0.5, 1e-2, 1e-5):
        gm = np.zeros(g.node_count)
        gv = np.zeros((g.node_count, 2))
        gm[node] = 0.5 * eps * mp
        gv[node] = [1.0 / (eps * dx), 2.0 / dx]
        t = oracle.grid_totals(g, gm, gv)
        assert t[6] * dx * dx / mp == pytest.approx((1.0 / eps + 4.0 * eps) / 4.0, rel=1e-14)


def _octahedron(center, a, m):
    """Six particles at center +- a e_k, mass m each: inertia 4 m a^2 I about center."""
    x = np.repeat(np.asarray(center, float)[None], 6, axis=0)
    for k in range(3):
        x[2 * k, k] += a
        x[2 * k + 1, k] -= a
    return x, np.full(6, m)


def _lattice(center, h, n, m):
    """(2n+1)^3 particles at center + h (i, j, k), |i|,|j|,|k| <= n, mass m each."""
    r = np.arange(-n, n + 1) * h
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + np.asarray(center, float)
    return x, np.full(x.shape[0], m)


def _lattice_inertia(h, n, m):
    """Closed form: sum_i i^2 = n (n+1) (2n+1) / 3 over one axis, times the
    (2n+1)^2 points of the other two; I = 2 m (2n+1)^2 h^2 sum_i i^2 * I."""
    s2 = n * (n + 1) * (2 * n + 1) / 3.0
    return 2.0 * m * (2 * n + 1) ** 2 * h * h * s2


@pytest.mark.parametrize("body", ["octahedron", "lattice"])
def test_rigid_body_particle_kinetic_energy(body):
    rng = np.random.default_rng(7)
    c = np.array([0.5, 0.45, 0.55])
    if body == "octahedron":
        a, mm = 0.1, 0.7
        x, m = _octahedron(c, a, mm)
        inertia = 4.0 * mm * a * a
    else:
        h, n, mm = 0.02, 3, 0.05
        x, m = _lattice(c, h, n, mm)
        inertia = _lattice_inertia(h, n, mm)
    vc = rng.normal(size=3)
    w = rng.normal(size=3)
    v = vc + np.cross(w, x - c)
    t = oracle.particle_totals(x, v, None, m)
    M = float(m.sum())
    expect = 0.5 * M * vc @ vc + 0.5 * inertia * w @ w
    assert t[6] == pytest.approx(expect, rel=1e-13)


@pytest.mark.parametrize("degree,k", [(2, 0.25), (3, 1.0 / 3.0)])
def test_rigid_body_grid_kinetic_energy_after_transfer(degree, k):
    """APIC carries a rigid field exactly to the nodes (B_p = omega^* D_p),
    so the grid kinetic energy is 1/2 M |v_c|^2 + 1/2 omega^T I_grid omega
    with I_grid = (I_particles + 2 k dx^2 M) I about the centre of mass, and
    the round trip back to the particles returns their kinetic energy."""
    rng = np.random.default_rng(11)
    cells = 16
    dx = 1.0 / cells
    g = oracle.Grid(3, degree, (cells,) * 3, dx)
    c = np.array([0.5, 0.5, 0.5])
    h, n, mm = 0.7 * dx, 3, 0.02
    x, m = _lattice(c, h, n, mm)
    x = x + 1e-3 * dx * np.array([0.3, -0.2, 0.1])      # off the node lattice
    c = x.mean(axis=0)
    inertia_p = _lattice_inertia(h, n, mm)
    vc = rng.normal(size=3)
    w = rng.normal(size=3)
    W = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    v = vc + (x - c) @ W.T
    B = np.repeat((k * dx * dx * W)[None], x.shape[0], axis=0)
    F = np.repeat(np.eye(3)[None], x.shape[0], axis=0)
    M = float(m.sum())
    out = oracle.p2g(g, x, v, B, F, m, m)
    u = oracle.grid_update(g, out["m"], out["mv"], None, 0.0)
    tg = oracle.grid_totals(g, out["m"], u["v"])
    expect = 0.5 * M * vc @ vc + 0.5 * (inertia_p + 2.0 * k * dx * dx * M) * w @ w
    assert tg[6] == pytest.approx(expect, rel=1e-12)
    back = oracle.g2p(g, x, F, u["vt"], u["xt"])
    tp = oracle.particle_totals(x, back["v"], back["B"], m)
    assert tp[6] == pytest.approx(0.5 * M * vc @ vc + 0.5 * inertia_p * w @ w, rel=1e-12)


def test_potential_energy_closed_forms():
    """Phi = sum V_p Psi(F_p): zero at rest; for a uniform stretch
    F = diag(s1, s2, s3), Psi = mu/2 (sum s^2 - 3) - mu ln J + lam/2 (ln J)^2
    written out; additive over particles."""
    mu, lam = 3.0, 5.0
    F = np.repeat(np.eye(3)[None], 4, axis=0)
    V = np.array([0.1, 0.2, 0.3, 0.4])
    assert oracle.potential(F, V, mu, lam) == 0.0
    s = np.array([1.1, 0.9, 1.2])
    J = float(np.prod(s))
    psi = 0.5 * mu * (float(s @ s) - 3.0) - mu * np.log(J) + 0.5 * lam * np.log(J) ** 2
    Fs = np.repeat(np.diag(s)[None], 4, axis=0)
    assert oracle.potential(Fs, V, mu, lam) == pytest.approx(psi * V.sum(), rel=1e-14)
    mixed = Fs.copy()
    mixed[:2] = np.eye(3)
    assert oracle.potential(mixed, V, mu, lam) == pytest.approx(psi * V[2:].sum(), rel=1e-14)
