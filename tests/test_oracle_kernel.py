"""Pins of the oracle's interpolation weights (Sec. 3.5) against facts fixed
outside the oracle: the truncated-power definition of the cardinal B-spline,
textbook node values, the kernel identities of Sec. 3.5, the constant
inertia-like tensor D_p and the printed Gram-matrix constants of Sec. 5.6."""
import json
import os

import numpy as np
import pytest

import oracle
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gram_constants.json")


@pytest.mark.parametrize("degree", [2, 3])
def test_bspline_matches_truncated_power_definition(degree):
    for t in np.linspace(-2.6, 2.6, 1041):
        assert oracle.bspline(degree, t) == pytest.approx(bf.bspline_tp(degree, t), abs=1e-14)
        assert oracle.bspline_deriv(degree, t) == pytest.approx(bf.bspline_tp_deriv(degree, t), abs=1e-13)


def test_bspline_textbook_node_values():
    # quadratic B-spline sampled at the integers: 1/8, 3/4, 1/8; at the half
    # integers 1/2, 1/2 and zero at the support edge
    assert oracle.bspline(2, 0.0) == 0.75
    assert oracle.bspline(2, 1.0) == 0.125 and oracle.bspline(2, -1.0) == 0.125
    assert oracle.bspline(2, 0.5) == 0.5 and oracle.bspline(2, -0.5) == 0.5
    assert oracle.bspline(2, 1.5) == 0.0
    # cubic: 1/6, 2/3, 1/6, and 0 at +-2
    assert oracle.bspline(3, 0.0) == pytest.approx(2.0 / 3.0, abs=1e-16)
    assert oracle.bspline(3, 1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert oracle.bspline(3, -1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert oracle.bspline(3, 2.0) == 0.0


def _random_positions(rng, dim, cells, degree, n):
    h = 1.5 if degree == 2 else 2.0
    dx = 1.0 / cells
    return (h + rng.random((n, dim)) * (cells - 2 * h)) * dx


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("degree", [2, 3])
def test_kernel_identities(dim, degree):
    """Sec. 3.5: sum w = 1, sum w x_i = x_p, sum w (x_i - x_p) = 0,
    sum x_i grad w^T = I (hence sum grad w = 0)."""
    cells = 10
    g = oracle.Grid(dim, degree, (cells,) * dim, 1.0 / cells)
    xi_all = g.node_positions()
    rng = np.random.default_rng(7)
    for xp in _random_positions(rng, dim, cells, degree, 50):
        nodes, w, gw = oracle.weights(g, xp)
        xi = xi_all[nodes]
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        np.testing.assert_allclose(w @ xi, xp, atol=1e-15)
        np.testing.assert_allclose(w @ (xi - xp), 0.0, atol=1e-15)
        np.testing.assert_allclose(gw.sum(axis=0), 0.0, atol=1e-12)
        np.testing.assert_allclose(xi.T @ gw, np.eye(dim), atol=1e-12)


@pytest.mark.parametrize("degree", [2, 3])
def test_support_size_and_ties(degree):
    g = oracle.Grid(3, degree, (8, 8, 8), 1.0 / 8)
    nodes, w, _ = oracle.weights(g, [0.4, 0.41, 0.43])
    assert len(nodes) == (3 if degree == 2 else 4) ** 3
    assert np.all(w > 0)
    # a particle exactly on a half node (quadratic) / node (cubic): the two
    # nodes at the support edges carry exactly zero weight
    tie = 4.5 if degree == 2 else 4.0
    nodes, w, gw = oracle.weights(g, [tie / 8, 0.41, 0.43])
    assert len(nodes) == (4 if degree == 2 else 5) * (3 if degree == 2 else 4) ** 2
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    assert np.count_nonzero(w) == (2 if degree == 2 else 3) * (3 if degree == 2 else 4) ** 2


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("degree", [2, 3])
def test_gradient_is_derivative_wrt_particle_position(dim, degree):
    """grad w_ip = grad N(x_p - x_i): central differences in x_p."""
    cells = 8
    dx = 1.0 / cells
    g = oracle.Grid(dim, degree, (cells,) * dim, dx)
    rng = np.random.default_rng(11)
    h = 1e-7
    for xp in _random_positions(rng, dim, cells, degree, 10):
        nodes, w, gw = oracle.weights(g, xp)
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = h
            n1, w1, _ = oracle.weights(g, xp + e)
            n0, w0, _ = oracle.weights(g, xp - e)
            full1 = dict(zip(n1, w1))
            full0 = dict(zip(n0, w0))
            for k, node in enumerate(nodes):
                fd = (full1.get(node, 0.0) - full0.get(node, 0.0)) / (2 * h)
                assert gw[k, a] == pytest.approx(fd, abs=2e-6 / dx)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("degree", [2, 3])
def test_weights_match_brute_force_over_all_nodes(dim, degree):
    cells = 6
    dx = 1.0 / cells
    g = oracle.Grid(dim, degree, (cells,) * dim, dx)
    rng = np.random.default_rng(3)
    for xp in _random_positions(rng, dim, cells, degree, 5):
        idx, _, wb, dwb = bf.weight_all_nodes(degree, (cells,) * dim, dx, xp)
        lin = bf.ij_to_oracle(idx, (cells,) * dim)
        full_w = np.zeros(g.node_count)
        full_g = np.zeros((g.node_count, dim))
        full_w[lin] = wb
        full_g[lin] = dwb
        nodes, w, gw = oracle.weights(g, xp)
        mine_w = np.zeros(g.node_count)
        mine_g = np.zeros((g.node_count, dim))
        mine_w[nodes] = w
        mine_g[nodes] = gw
        np.testing.assert_allclose(mine_w, full_w, atol=1e-14)
        np.testing.assert_allclose(mine_g, full_g, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("degree,factor", [(2, 0.25), (3, 1.0 / 3.0)])
def test_D_is_constant_multiple_of_identity(dim, degree, factor):
    """D_p = (dx^2/4) I for quadratic and (dx^2/3) I for cubic B-splines,
    independent of the particle position (Sec. 5.6, 'Coefficient
    computations'; the same constant k enters the CFL rule of Sec. 4.3)."""
    cells = 12
    dx = 1.0 / cells
    s = np.random.default_rng(5)
    x = _random_positions(s, dim, cells, degree, 40)
    n = len(x)
    g = oracle.Grid(dim, degree, (cells,) * dim, dx)
    out = oracle.p2g(g, x, np.zeros((n, dim)), np.zeros((n, dim, dim)), np.tile(np.eye(dim), (n, 1, 1)),
                     np.ones(n), np.ones(n), want_D=True)
    for D in out["D"]:
        np.testing.assert_allclose(D, factor * dx * dx * np.eye(dim), rtol=1e-13, atol=1e-13 * dx * dx)


def _levi(a, b, c):
    return float(np.linalg.det(np.eye(3)[[a, b, c]]))


def _affine_basis(r):
    """The 12 basis vectors b_jpi of Sec. 5.6 at one node offset r = x_i - x_p."""
    e = np.eye(3)
    out = [e[j] for j in range(3)]
    for j in range(3):   # rotations: component l is sum_k eps_{j k l} r_k
        out.append(np.array([sum(_levi(j, k, l) * r[k] for k in range(3)) for l in range(3)]))
    for j in range(3):   # symmetric shears: |eps_{j k l}|
        out.append(np.array([sum(abs(_levi(j, k, l)) * r[k] for k in range(3)) for l in range(3)]))
    for j in range(3):   # diagonal stretches: e_j e_j^T r
        out.append(e[j] * r[j])
    return np.array(out)


@pytest.mark.parametrize("degree", [2, 3])
def test_gram_matrix_matches_printed_constants(degree):
    """Sec. 5.6: b_jp^T M b_ip is diagonal and constant with the printed
    entries (golden fixture, citation inside)."""
    golden = json.load(open(GOLDEN))
    key = "quadratic" if degree == 2 else "cubic"
    cells = 10
    dx = 1.0 / cells
    g = oracle.Grid(3, degree, (cells,) * 3, dx)
    xi_all = g.node_positions()
    mp = 1.7
    expect = np.diag(np.array(golden[key]["translation"] + [c * dx * dx for c in golden[key]["per_dx2"]]) * mp)
    rng = np.random.default_rng(9)
    for xp in _random_positions(rng, 3, cells, degree, 12):
        nodes, w, _ = oracle.weights(g, xp)
        G = np.zeros((12, 12))
        for k, node in enumerate(nodes):
            b = _affine_basis(xi_all[node] - xp)
            G += mp * w[k] * (b @ b.T)
        np.testing.assert_allclose(G, expect, atol=1e-13 * mp)


def test_particle_outside_support_domain_is_an_error():
    g = oracle.Grid(3, 2, (8, 8, 8), 1.0 / 8)
    with pytest.raises(oracle.OracleError):
        oracle.weights(g, [0.04, 0.5, 0.5])     # support reaches node -1
    nodes, w, _ = oracle.weights(g, [0.5 / 8, 0.5, 0.5])   # edge: node -1 has zero weight
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
