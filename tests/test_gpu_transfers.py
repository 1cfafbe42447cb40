"""RPIC and PIC transfers on the GPU (Sec. 2.1, Sec. 5.6) against the FP64
oracle, which forms the RPIC state from K_p^{-1} l_p while the kernels keep
the skew part of B.  Bars as for APIC: binary64 1e-12, binary32 1e-5 per
field per step (k chained steps: k times the bar)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1603_06188_amd import scenes
from tests.test_gpu_parity import TOL, compare_step, ogrid, rel

pytestmark = pytest.mark.gpu

RPIC, PIC = oracle.TRANSFER_RPIC, oracle.TRANSFER_PIC


def _b():
    from paper_1603_06188_amd import binding
    return binding


def _scene(dim, degree, precision, transfer, seed, n=None):
    """Neo-Hookean particles with a general (not skew) B, so that the
    transfer to grid has to drop part of it."""
    s = scenes.random_particles(n or (3000 if dim == 3 else 2000), dim=dim, cells=20, degree=degree, seed=seed,
                                precision=precision, f_sigma=0.05, b_sigma=0.05, vel_sigma=0.3, model=1)
    return dataclasses.replace(s, transfer=transfer)


@pytest.mark.parametrize("transfer", [RPIC, PIC])
@pytest.mark.parametrize("precision,compensated", [("fp64", False), ("fp32", True)])
@pytest.mark.parametrize("dim,degree", [(3, 2), (3, 3), (2, 2), (2, 3)])
def test_one_step_per_phase(dim, degree, precision, compensated, transfer):
    s = _scene(dim, degree, precision, transfer, seed=31)
    ds = _b().DeviceScene(s, compensated=compensated)
    _, got, _ = compare_step(s, ds, TOL[precision], label=f"transfer {transfer} {dim}d deg{degree} {precision}")
    if transfer == PIC:
        assert not got["B"].any()
    else:
        np.testing.assert_array_equal(got["B"], -np.swapaxes(got["B"], 1, 2))


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("transfer", [RPIC, PIC])
def test_steps_in_one_call_match_chained_oracle(transfer, fused):
    """Three binary32 steps in one apic_step call (the first two fused with
    the next transfer to grid when asked) against three chained oracle
    steps.  Particles drift about half a cell per step, so most change key
    and many change tile (the re-binning inside the call is exercised)."""
    b = _b()
    s = scenes.random_particles(5000, dim=3, cells=16, degree=2, seed=32, precision="fp32", margin=3.0,
                                vel_sigma=0.3, f_sigma=0.02, b_sigma=0.02, model=1)
    s = dataclasses.replace(s.with_state(v=s.v + np.array([6.0, 4.0, -4.0])), dt=5e-3, transfer=transfer)
    steps = 3
    ds = b.DeviceScene(s, compensated=True, fused=fused)
    ds.step(steps)
    got = ds.state()
    assert ds.flags() == 0
    g = ogrid(s)
    x, v, B, F = s.x, s.v, s.B, s.F
    moved = 0
    for _ in range(steps):
        r = oracle.step(g, x, v, B, F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band, transfer=transfer)
        moved += int(np.count_nonzero((np.floor(r["x_new"] / s.dx - 0.5) != np.floor(x / s.dx - 0.5)).any(axis=1)))
        x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
    assert moved > s.n
    tol = steps * 1e-5
    assert float(np.abs(got["x"] - x).max() / s.dx) <= tol
    for key, ref in (("v", v), ("B", B), ("F", F)):
        assert rel(got[key], ref) <= tol, (key, rel(got[key], ref))


@pytest.mark.parametrize("transfer", [oracle.TRANSFER_APIC, RPIC, PIC])
def test_stiff_steps_each_from_the_oracle_state(transfer):
    """A stiff scene near the explicit limit (wave speed x dt / dx ~ 0.4):
    after the first step some nodes are reached only by weights near 1e-9
    and carry velocities of order 1e3.  Each binary32 step starts from the
    oracle's state and meets the one-step bar; this holds because the
    velocity taken out of the G2P sums is that of the node nearest each
    particle (a corner node of the support can be such an outlier, and its
    rounding then dominated v at the 1e-4 level)."""
    b = _b()
    s = dataclasses.replace(_scene(3, 2, "fp32", transfer, seed=32, n=5000), dt=2e-3)
    ds = b.DeviceScene(s, compensated=True)
    for k in range(3):
        ref, _, _ = compare_step(s, ds, TOL["fp32"], label=f"transfer {transfer} step {k}")
        s = s.with_state(x=ref["x_new"], v=ref["v_new"], B=ref["B_new"], F=ref["F_new"])
        ds.upload(s)


def test_rotating_disk_round_trips_per_transfer():
    """The rotating disk of the transfer tests, ten P2G -> G2P round trips at
    dt = 0 in binary64: APIC and RPIC keep the angular momentum of the
    rotation, PIC loses sum_p K_p omega on the first trip and keeps losing;
    each GPU trip matches the oracle's."""
    b = _b()
    base = scenes.disk2d()
    g = ogrid(base)
    scale = float(np.sum(base.m * (np.linalg.norm(base.x, axis=1) * np.linalg.norm(base.v, axis=1))))
    l_end = {}
    for tr in (oracle.TRANSFER_APIC, RPIC, PIC):
        s = dataclasses.replace(base, transfer=tr)
        ds = b.DeviceScene(s)
        x, v, B, F = s.x, s.v, s.B, s.F
        l0 = oracle.particle_totals(x, v, B, s.m)[5]
        for k in range(10):
            ref = oracle.step(g, x, v, B, F, s.m, s.V, 0, dt=0.0, transfer=tr)
            ds.step(1)
            got = ds.state()
            for key, a, bb in (("v", got["v"], ref["v_new"]), ("B", got["B"], ref["B_new"])):
                assert rel(a, bb) <= 1e-12, (tr, k, key, rel(a, bb))
            x, v, B, F = ref["x_new"], ref["v_new"], ref["B_new"], ref["F_new"]
        l_end[tr] = ds.diagnostics(b.APIC_DIAG_PARTICLES)[5]
        if tr != PIC:
            assert abs(l_end[tr] - l0) <= 1e-12 * scale, (tr, l_end[tr], l0)
    assert l_end[PIC] < l_end[RPIC] - 1e-3 * abs(l_end[RPIC])


def test_rpic_conserves_angular_momentum_with_forces():
    """Binary64, neo-Hookean, no gravity or walls: over several RPIC steps
    the particle momenta (B term included) stay at their initial values to
    rounding, as for APIC (Sec. 5.1 transfers, Sec. 5.3 forces)."""
    b = _b()
    s = dataclasses.replace(_scene(3, 2, "fp64", RPIC, seed=33, n=4000), dt=2e-3)
    ds = b.DeviceScene(s)
    skew = 0.5 * (s.B - np.swapaxes(s.B, 1, 2))
    t0 = oracle.particle_totals(s.x, s.v, skew, s.m)
    ds.step(5)
    t1 = ds.diagnostics(b.APIC_DIAG_PARTICLES)
    assert ds.flags() == 0
    S = float(np.sum(s.m * (np.linalg.norm(s.x, axis=1) * np.linalg.norm(s.v, axis=1) + 1.0)))
    assert np.abs(t1[:6] - t0[:6]).max() <= 1e-13 * S, (t1[:6], t0[:6])
