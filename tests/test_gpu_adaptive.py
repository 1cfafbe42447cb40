"""Adaptive steps (APIC_OPT_ADAPTIVE_DT): every step of one apic_step call
takes dt_k = min(dt, nu dx / b_k) with b_k the CFL bound of Sec. 4.3 over the
state the step starts from, chosen on the device (the first step from a
pass over the particles, later ones from the bound the transfer to
particles folded in).  Checked against the oracle chained with
oracle.cfl_dt choosing each step's dt from its own state."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1603_06188_amd import scenes
from tests.test_gpu_parity import ogrid, rel

pytestmark = pytest.mark.gpu


def _b():
    from paper_1603_06188_amd import binding
    return binding


def _adaptive_chain(s, steps, cap, nu):
    g = ogrid(s)
    x, v, B, F = s.x, s.v, s.B, s.F
    dts = []
    for _ in range(steps):
        dt = min(cap, oracle.cfl_dt(s.dx, v, B, nu))
        r = oracle.step(g, x, v, B, F, s.m, s.V, s.model, s.mu, s.lam, dt, s.gravity, s.band, transfer=s.transfer)
        x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
        dts.append(dt)
    return x, v, B, F, dts


@pytest.mark.parametrize("precision,dim,degree", [("fp64", 3, 2), ("fp64", 3, 3), ("fp64", 2, 2), ("fp32", 3, 2)])
def test_adaptive_steps_match_oracle_chain(precision, dim, degree):
    """The CFL rule binds (cap 1e-2 is never reached): four steps of
    different dt, each the oracle's rule applied to its own state.  The 2D
    scene uses nu = 0.2: its random field smooths out after one step, and at
    nu = 0.4 the rule then allows steps past the elastic limit, where the
    oracle's chain inverts elements too (the rule of Sec. 4.3 bounds
    advection only)."""
    b = _b()
    s = scenes.random_particles(3000 if dim == 3 else 2000, dim=dim, cells=16, degree=degree, seed=41,
                                precision=precision, vel_sigma=0.5, f_sigma=0.02, b_sigma=0.01, model=1)
    nu, cap, steps = (0.4 if dim == 3 else 0.2), 1e-2, 4
    s = dataclasses.replace(s, dt=cap, cfl=nu)
    ds = b.DeviceScene(s, compensated=precision == "fp32", adaptive=True)
    ds.step(steps)
    got = ds.state()
    dt_last, t = ds.step_time()
    assert ds.flags() == 0
    x, v, B, F, dts = _adaptive_chain(s, steps, cap, nu)
    assert max(dts) < cap and len(set(dts)) == steps  # the rule chose every step's dt
    tol = 1e-11 if precision == "fp64" else steps * 1e-5
    assert abs(t - sum(dts)) <= tol * sum(dts), (t, sum(dts))
    assert abs(dt_last - dts[-1]) <= tol * dts[-1], (dt_last, dts[-1])
    assert float(np.abs(got["x"] - x).max() / s.dx) <= tol
    for key, ref in (("v", v), ("B", B), ("F", F)):
        assert rel(got[key], ref) <= tol, (key, rel(got[key], ref))


def test_cap_binds_and_time_accumulates_over_calls():
    """A slow scene: the cap is the step every time, the clock advances by
    exactly n * cap over two calls, and the state equals that of fixed
    steps of the same size."""
    b = _b()
    s = scenes.cube3d(cells=24, precision="fp64", steps=3)
    s = dataclasses.replace(s, cfl=0.5)
    ad = b.DeviceScene(s, adaptive=True)
    fx = b.DeviceScene(s)
    ad.step(2)
    ad.step(3)
    fx.step(5)
    dt_last, t = ad.step_time()
    assert dt_last == s.dt
    assert t == s.dt + s.dt + s.dt + s.dt + s.dt
    a, f = ad.state(), fx.state()
    for key in ("x", "v", "B", "F"):
        assert rel(a[key], f[key]) <= 1e-13, key
    assert ad.flags() == fx.flags() == 0


def test_bound_pass_and_folded_bound_agree_with_apic_cfl_dt():
    """After a call, the dt the first step of the next call takes (a binary64
    pass) equals apic_cfl_dt's; the dt a third step takes from the bound the
    second G2P folded in (binary32 here) agrees to binary32 rounding."""
    b = _b()
    s = scenes.random_particles(4000, dim=3, cells=16, degree=2, seed=42, precision="fp32", vel_sigma=0.5,
                                f_sigma=0.02, b_sigma=0.01, model=1)
    nu = 0.3
    s = dataclasses.replace(s, dt=1.0, cfl=nu)
    ds = b.DeviceScene(s, compensated=True, adaptive=True)
    ds.step(2)
    full = ds.cfl_dt(nu)          # full pass over the state after two steps
    ds.step(1)                    # first step of a call: its own full pass
    dt_first, _ = ds.step_time()
    assert dt_first == pytest.approx(full, rel=1e-15)
    ds2 = b.DeviceScene(s, compensated=True, adaptive=True)
    ds2.step(3)                   # third step: the bound folded into the second G2P
    dt_folded, _ = ds2.step_time()
    assert dt_folded == pytest.approx(full, rel=1e-6)  # two binary32 runs, mover order aside


def test_batched_adaptive_steps_match_each_scene_alone():
    """apic_step_batch with adaptive steps: every scene takes its own dt per
    step, as when it runs alone (binary64, three scenes of different size
    and speed), and the smallest matches the oracle chained with the rule."""
    b = _b()
    nu, cap, steps = 0.4, 1e-2, 3
    hosts = [dataclasses.replace(
        scenes.random_particles(n, dim=3, cells=c, degree=2, seed=70 + k, precision="fp64", vel_sigma=vs,
                                f_sigma=0.02, b_sigma=0.01, model=1), dt=cap, cfl=nu)
        for k, (n, c, vs) in enumerate(((1500, 12, 0.5), (6000, 20, 1.0), (900, 10, 0.3)))]
    batch = b.SceneBatch([b.DeviceScene(h, adaptive=True) for h in hosts])
    batch.step(steps)
    alone = [b.DeviceScene(h, adaptive=True) for h in hosts]
    for a in alone:
        a.step(steps)
    times = []
    for k, (d, a) in enumerate(zip(batch.scenes, alone)):
        assert d.flags() == 0 and a.flags() == 0, k
        (dl, t), (dla, ta) = d.step_time(), a.step_time()
        assert t == pytest.approx(ta, rel=1e-12) and dl == pytest.approx(dla, rel=1e-12), k
        times.append(t)
        got, ref = d.state(), a.state()
        for key in ("x", "v", "B", "F"):
            assert rel(got[key], ref[key]) <= 1e-12, (k, key)
    assert len(set(round(t, 12) for t in times)) == 3  # each scene took its own steps
    h = hosts[2]
    x, v, B, F, dts = _adaptive_chain(h, steps, cap, nu)
    assert max(dts) < cap
    got = batch.scenes[2].state()
    assert abs(times[2] - sum(dts)) <= 1e-11 * sum(dts)
    for key, ref in (("v", v), ("B", B), ("F", F)):
        assert rel(got[key], ref) <= 1e-11, (key, rel(got[key], ref))


def test_fused_option_is_off_with_adaptive_steps():
    """Asking for the fused transfer and adaptive steps together runs the
    adaptive, unfused path: the same dt and state as adaptive steps alone
    (binary32 quadratic 3D, where fusion would otherwise apply)."""
    b = _b()
    s = scenes.random_particles(4000, dim=3, cells=16, degree=2, seed=43, precision="fp32", vel_sigma=0.5,
                                f_sigma=0.02, b_sigma=0.01, model=1)
    s = dataclasses.replace(s, dt=1e-2, cfl=0.4)
    both = b.DeviceScene(s, compensated=True, fused=True, adaptive=True)
    alone = b.DeviceScene(s, compensated=True, adaptive=True)
    both.step(3)
    alone.step(3)
    assert both.flags() == alone.flags() == 0
    (d1, t1), (d2, t2) = both.step_time(), alone.step_time()
    assert t1 == pytest.approx(t2, rel=1e-6) and d1 == pytest.approx(d2, rel=1e-6)
    got, ref = both.state(), alone.state()
    for key in ("x", "v", "B", "F"):
        # same kernels; the order movers are summed in differs between the two
        # binary32 runs (B has seen 1.2e-6 after three steps)
        assert rel(got[key], ref[key]) <= 1e-5, key
