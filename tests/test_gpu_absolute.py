"""Positions held as plain binary32 coordinates (APIC_OPT_ABSOLUTE_POSITIONS),
the third precision mode of the two-sphere comparison: one step against the
FP64 oracle from the binary32-rounded coordinates, phase by phase.  The
transfers derive cell and offset from x (s = x / dx, c = floor(s),
o = s - c); with dx a power of two these offsets are exact, so the grid and
v, B, F are held to the binary32 bar of 1e-5; the stored coordinate is
rounded to half a unit in the last place of x.  Also: several steps through
apic_step against chained oracle steps, and the conversions to and from
absolute coordinates."""
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


def _rounded(s):
    return s.with_state(x=s.x.astype(np.float32).astype(np.float64))


def _x_bound(ref_x, ref_v, dt, dx, steps=1):
    half_ulp = np.spacing(np.float32(np.abs(ref_x).max())).astype(np.float64) / 2
    return steps * (half_ulp + dt * 1e-5 * float(np.abs(ref_v).max())) / dx * 1.01


@pytest.mark.parametrize("dim,degree", [(3, 2), (3, 3), (2, 2), (2, 3)])
def test_absolute_positions_one_step(dim, degree):
    b = _b()
    s = _rounded(scenes.random_particles(3000 if dim == 3 else 2000, dim=dim, cells=16, degree=degree, seed=23,
                                         precision="fp32", f_sigma=0.05, b_sigma=0.01, vel_sigma=0.3))
    g = oracle.Grid(s.dim, s.degree, s.cells, s.dx)
    ref = oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band)
    ds = b.DeviceScene(s, compensated=True, absolute=True)
    np.testing.assert_array_equal(ds.state()["x"], s.x)       # the planes hold the coordinates
    ds.p2g()
    errs = {"m": rel(ds.export(b.APIC_GRID_MASS), ref["m"]),
            "mv": rel(ds.export(b.APIC_GRID_MOMENTUM), ref["mv"] + s.dt * ref["f"])}
    ds.grid_update()
    ds.g2p()
    got = ds.state()
    assert ds.flags() == 0
    for k in ("v", "B", "F"):
        errs[k] = rel(got[k], ref[k + "_new"])
    print(dim, degree, errs, flush=True)
    for k, e in errs.items():
        assert e <= 1e-5, (k, e)
    xerr = float(np.abs(got["x"] - ref["x_new"]).max() / s.dx)
    assert xerr <= _x_bound(ref["x_new"], ref["v_new"], s.dt, s.dx), xerr
    # the stored coordinates are binary32 values
    assert np.array_equal(got["x"], got["x"].astype(np.float32).astype(np.float64))


def test_absolute_positions_steps_and_rebinning():
    """Four whole steps in one apic_step call with fast particles (many change
    key every step, so the re-binning sees absolute coordinates), against the
    oracle chained over the same steps from the binary32 state each step."""
    import dataclasses
    b = _b()
    s = scenes.random_particles(4000, dim=3, cells=16, degree=2, seed=33, margin=5.0, vel_sigma=0.3,
                                f_sigma=0.05, b_sigma=0.02, model=0, precision="fp32")
    s = _rounded(dataclasses.replace(s.with_state(v=s.v + np.array([1.5, 1.0, -1.0])), dt=2e-2))
    ds = b.DeviceScene(s, compensated=True, absolute=True)
    ds.step(4)
    got = ds.state()
    assert ds.flags() == 0
    g = oracle.Grid(s.dim, s.degree, s.cells, s.dx)
    x, v, B, F = s.x, s.v, s.B, s.F
    for _ in range(4):
        r = oracle.step(g, x, v, B, F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band)
        x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
    for k, a, ref in (("v", got["v"], v), ("B", got["B"], B), ("F", got["F"], F)):
        assert rel(a, ref) <= 4e-5, (k, rel(a, ref))
    assert float(np.abs(got["x"] - x).max() / s.dx) <= _x_bound(x, v, s.dt, s.dx, steps=4)


def test_absolute_positions_conversions():
    """apic_positions_from_absolute stores the binary32 coordinate; the
    conversion back returns it; the particle diagnostics use it."""
    import torch
    b = _b()
    s = _rounded(scenes.random_particles(500, dim=3, cells=16, degree=3, seed=5, precision="fp32"))
    ds = b.DeviceScene(s, absolute=True)
    # dim planes of the scene's plane stride (its capacity, whole 64-particle blocks)
    assert ds.capacity >= s.n and ds.capacity % 64 == 0
    x = torch.zeros((3, ds.capacity), dtype=torch.float64, device="cuda")
    x[:, :s.n] = torch.tensor(np.ascontiguousarray(s.x.T), dtype=torch.float64)
    back = torch.empty_like(x)
    b.apic_positions_to_absolute(ds.s, back.data_ptr())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(back[:, :s.n].cpu().numpy().T, s.x)
    b.apic_positions_from_absolute(ds.s, x.data_ptr())
    b.apic_sort(ds.s)
    np.testing.assert_array_equal(ds.state()["x"], s.x)
    t = oracle.particle_totals(s.x, s.v, s.B, s.m)
    np.testing.assert_allclose(ds.diagnostics(b.APIC_DIAG_PARTICLES), t, rtol=1e-12, atol=1e-12 * np.abs(t).max())
