"""Several steps in one apic_step call with APIC_OPT_FUSED_TRANSFER, binary32
quadratic 3D: the transfer to particles of every step but the last is fused
with the next step's transfer to grid (the slabs of the new layout are formed from the values just written;
particles that changed key are added by a second pass).

Checked against the FP64 oracle chained over the same steps.  Tolerance: the
binary32 bar of one step is 1e-5 (relative to the field's largest value, or
cells for positions); a k-step chain compounds at most k of them to first
order, so the bar here is k * 1e-5.  The grid exported after the call is the
one the last step was computed from, i.e. the fused pass's slabs; it comes
from the state after k - 1 steps, so its bar is k * 1e-5 as well.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1603_06188_amd import scenes

pytestmark = pytest.mark.gpu


def _b():
    from paper_1603_06188_amd import binding
    return binding


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float(np.abs(b).max())
    return float(np.abs(a - b).max()) / den if den else float(np.abs(a).max())


def _chain(s, steps):
    g = oracle.Grid(s.dim, s.degree, s.cells, s.dx)
    x, v, B, F = s.x, s.v, s.B, s.F
    out = []
    for _ in range(steps):
        r = oracle.step(g, x, v, B, F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band, transfer=s.transfer)
        out.append((x, r))
        x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
    return out


def _fast_scene(seed, n=5000):
    """Neo-Hookean particles drifting ~0.5 cell per step: a large share
    changes key and many change tile every step."""
    s = scenes.random_particles(n, dim=3, cells=16, degree=2, seed=seed, precision="fp32", margin=3.0,
                                vel_sigma=0.3, f_sigma=0.02, b_sigma=0.02, model=1)
    drift = np.array([6.0, 4.0, -4.0])
    return dataclasses.replace(s.with_state(v=s.v + drift), dt=5e-3)


def _keys(x, dx):
    return np.floor(x / dx - 0.5).astype(np.int64)


@pytest.mark.parametrize("compensated", [False, True])
def test_fused_steps_match_chained_oracle(compensated):
    b = _b()
    s = _fast_scene(51)
    steps = 3
    ds = b.DeviceScene(s, compensated=compensated, fused=True)
    ds.step(steps)
    got = ds.state()
    assert ds.flags() == 0
    chain = _chain(s, steps)
    # the re-binning inside the fused pass is exercised: keys and tiles change
    key_moves = tile_moves = 0
    for x_in, r in chain:
        k0, k1 = _keys(x_in, s.dx), _keys(r["x_new"], s.dx)
        key_moves += int(np.count_nonzero((k0 != k1).any(axis=1)))
        tile_moves += int(np.count_nonzero((k0 // 4 != k1 // 4).any(axis=1)))
    assert key_moves > s.n // 2 and tile_moves > s.n // 10
    tol = steps * 1e-5
    last = chain[-1][1]
    assert float(np.abs(got["x"] - last["x_new"]).max() / s.dx) <= tol
    for key, ref in (("v", last["v_new"]), ("B", last["B_new"]), ("F", last["F_new"])):
        assert rel(got[key], ref) <= tol, (key, rel(got[key], ref))
    # the grid of the last step: the fused pass's slabs
    assert rel(ds.export(b.APIC_GRID_MASS), last["m"]) <= tol
    assert rel(ds.export(b.APIC_GRID_MOMENTUM), last["mv"] + s.dt * last["f"]) <= tol


def test_fused_and_per_call_steps_agree():
    """Three steps in one call (two fused) and three calls of one step (none
    fused) give the same state to the same bar."""
    b = _b()
    s = _fast_scene(52, n=3000)
    one = b.DeviceScene(s, compensated=True, fused=True)
    one.step(3)
    each = b.DeviceScene(s, compensated=True)
    for _ in range(3):
        each.step(1)
    a, c = one.state(), each.state()
    assert float(np.abs(a["x"] - c["x"]).max() / s.dx) <= 3e-5
    for key in ("v", "B", "F", "m"):
        assert rel(a[key], c[key]) <= 3e-5, key
    assert one.flags() == each.flags() == 0


def test_fused_full_size_two_steps():
    """The benchmark cube (128^3 grid, 2,097,152 particles, compensated):
    two steps in one call, the first fused, against two chained oracle
    steps; the grid of the second step comes from the fused pass."""
    b = _b()
    s = scenes.cube3d()
    ds = b.DeviceScene(s, compensated=True, fused=True)
    ds.step(2)
    got = ds.state()
    assert ds.flags() == 0
    chain = _chain(s, 2)
    last = chain[-1][1]
    assert float(np.abs(got["x"] - last["x_new"]).max() / s.dx) <= 2e-5
    for key, ref in (("v", last["v_new"]), ("B", last["B_new"]), ("F", last["F_new"])):
        assert rel(got[key], ref) <= 2e-5, (key, rel(got[key], ref))
    assert rel(ds.export(b.APIC_GRID_MASS), last["m"]) <= 2e-5
    assert rel(ds.export(b.APIC_GRID_MOMENTUM), last["mv"] + s.dt * last["f"]) <= 2e-5
