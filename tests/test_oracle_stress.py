"""Pins of the oracle's neo-Hookean energy density and stress (Sec. 3.1:
P = dPsi/dF), checked against calculus and continuum-mechanics facts rather
than against a retyped formula."""
import numpy as np
import pytest

import oracle

MU, LAM = 3.7, 5.1


def _rot(rng, d):
    q, r = np.linalg.qr(rng.normal(size=(d, d)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _rand_F(rng, d):
    return np.eye(d) + 0.3 * rng.normal(size=(d, d))


@pytest.mark.parametrize("d", [2, 3])
def test_rest_state_is_stress_and_energy_free(d):
    assert oracle.neo_hookean_psi(np.eye(d), MU, LAM) == 0.0
    np.testing.assert_array_equal(oracle.neo_hookean_P(np.eye(d), MU, LAM), np.zeros((d, d)))


@pytest.mark.parametrize("d", [2, 3])
def test_P_is_derivative_of_psi(d):
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(10):
        F = _rand_F(rng, d)
        if np.linalg.det(F) <= 0.2:
            continue
        P = oracle.neo_hookean_P(F, MU, LAM)
        for r in range(d):
            for c in range(d):
                E = np.zeros((d, d))
                E[r, c] = h
                fd = (oracle.neo_hookean_psi(F + E, MU, LAM) - oracle.neo_hookean_psi(F - E, MU, LAM)) / (2 * h)
                assert P[r, c] == pytest.approx(fd, rel=1e-6, abs=1e-7)


@pytest.mark.parametrize("d", [2, 3])
def test_frame_indifference_and_symmetric_kirchhoff_stress(d):
    """Psi(RF) = Psi(F), P(RF) = R P(F); P F^T symmetric -- the property the
    angular-momentum argument of Sec. 5.3 needs from an energy-derived force."""
    rng = np.random.default_rng(2)
    for _ in range(10):
        F = _rand_F(rng, d)
        if np.linalg.det(F) <= 0.2:
            continue
        R = _rot(rng, d)
        assert oracle.neo_hookean_psi(R @ F, MU, LAM) == pytest.approx(oracle.neo_hookean_psi(F, MU, LAM),
                                                                      rel=1e-12, abs=1e-13)
        np.testing.assert_allclose(oracle.neo_hookean_P(R @ F, MU, LAM), R @ oracle.neo_hookean_P(F, MU, LAM),
                                   atol=1e-12)
        tau = oracle.neo_hookean_P(F, MU, LAM) @ F.T
        np.testing.assert_allclose(tau, tau.T, atol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_small_strain_limit_is_linear_elasticity(d):
    """P(I + eps H) = eps (lambda tr(S) I + 2 mu S) + O(eps^2), S = sym(H)."""
    rng = np.random.default_rng(3)
    H = rng.normal(size=(d, d))
    S = 0.5 * (H + H.T)
    lin = LAM * np.trace(S) * np.eye(d) + 2 * MU * S
    for eps in (1e-3, 1e-4):
        P = oracle.neo_hookean_P(np.eye(d) + eps * H, MU, LAM)
        np.testing.assert_allclose(P / eps, lin, atol=20 * eps * (MU + LAM) * np.abs(H).max() ** 2)


def test_inverted_element_is_an_error():
    F = np.diag([1.0, 1.0, -1.0])
    with pytest.raises(oracle.OracleError):
        oracle.neo_hookean_P(F, MU, LAM)
    with pytest.raises(oracle.OracleError):
        oracle.neo_hookean_psi(F, MU, LAM)
