"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Per field, per step: err = max_k |X_gpu - X_ref| / max_k |X_ref| (positions:
max displacement error in cell units).  Bars: binary64 mode 1e-12, binary32
mode 1e-5.  Both sides start from the same seeded input; the oracle never
sees a value the GPU produced.
"""
import numpy as np
import pytest

import oracle
from paper_1603_06188_amd import scenes

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _b():
    from paper_1603_06188_amd import binding
    return binding


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float(np.abs(b).max())
    if den == 0.0:
        return float(np.abs(a).max())
    return float(np.abs(a - b).max()) / den


def ogrid(s):
    return oracle.Grid(s.dim, s.degree, s.cells, s.dx)


def compare_step(s, ds, tol, check_grid=True, label=""):
    """Run one GPU step phase by phase and compare every phase with the oracle."""
    b = _b()
    g = ogrid(s)
    ref = oracle.step(g, s.x, s.v, s.B, s.F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band, transfer=s.transfer)
    errs = {}
    # kinetic energy of the input state (Sec. 3.1): the same numbers on both sides
    ke = oracle.particle_totals(s.x, s.v, s.B, s.m)[6]
    errs["KE_in"] = rel(ds.diagnostics(b.APIC_DIAG_PARTICLES)[6], ke)
    ds.p2g()
    if check_grid:
        m = ds.export(b.APIC_GRID_MASS)
        mv = ds.export(b.APIC_GRID_MOMENTUM)
        errs["m"] = rel(m, ref["m"])
        errs["mv"] = rel(mv, ref["mv"] + s.dt * ref["f"])
    ds.grid_update()
    if check_grid:
        vt = ds.export(b.APIC_GRID_VELOCITY)
        # grid velocity weighted by mass: vt is ill-conditioned where m_i -> 0
        # and those nodes carry weight ~0 in every particle update
        errs["m*vt"] = rel(vt * ref["m"][:, None], ref["vt"] * ref["m"][:, None])
    ds.g2p()
    got = ds.state()
    errs["x_cells"] = float(np.abs(got["x"] - ref["x_new"]).max() / s.dx)
    errs["v"] = rel(got["v"], ref["v_new"])
    errs["B"] = rel(got["B"], ref["B_new"])
    errs["F"] = rel(got["F"], ref["F_new"])
    bad = {k: e for k, e in errs.items() if not e <= tol}
    assert not bad, f"{label} errors above {tol}: {errs}"
    assert ds.flags() == 0
    return ref, got, errs


@pytest.mark.parametrize("precision,compensated", [("fp64", False), ("fp32", False), ("fp32", True)])
@pytest.mark.parametrize("dim,degree", [(3, 2), (3, 3), (2, 2), (2, 3)])
def test_one_step_random_particles(dim, degree, precision, compensated):
    s = scenes.random_particles(3000 if dim == 3 else 2000, dim=dim, cells=20, degree=degree, seed=21,
                                precision=precision, f_sigma=0.05, b_sigma=0.01, vel_sigma=0.3)
    ds = _b().DeviceScene(s, compensated=compensated)
    compare_step(s, ds, TOL[precision], label=f"{dim}d deg{degree} {precision}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cube_steps_against_oracle(precision):
    """Small version of the elastic cube (gravity, sticky floor), several
    steps, each compared from the same input state."""
    s = scenes.cube3d(cells=24, precision=precision, steps=3)
    ds = _b().DeviceScene(s, compensated=True)
    for k in range(3):
        ref, got, errs = compare_step(s, ds, TOL[precision], label=f"step {k}")
        # next step starts from the oracle's state on both sides
        s = s.with_state(x=ref["x_new"], v=ref["v_new"], B=ref["B_new"], F=ref["F_new"])
        ds.upload(s)


@pytest.mark.parametrize("dim,degree", [(3, 2), (3, 3), (2, 2)])
def test_apic_step_matches_chained_oracle_steps(dim, degree):
    """Several whole steps through apic_step (particles re-binned by every
    G2P, state alternating between the caller's planes and the workspace)
    against the oracle chained over the same steps, in binary64.  Fast
    particles make many change their base node every step."""
    import dataclasses
    b = _b()
    s = scenes.random_particles(4000 if dim == 3 else 3000, dim=dim, cells=16, degree=degree, seed=31,
                                margin=5.0, vel_sigma=0.3, f_sigma=0.05, b_sigma=0.02, model=0)
    drift = np.array([1.5, 1.0, -1.0])[:dim]
    s = dataclasses.replace(s.with_state(v=s.v + drift), dt=2e-2)   # ~0.5 cell per step
    steps = 6
    ds = b.DeviceScene(s)
    ds.step(steps)
    got = ds.state()
    g = ogrid(s)
    x, v, B, F = s.x, s.v, s.B, s.F
    moved_keys = 0
    for _ in range(steps):
        r = oracle.step(g, x, v, B, F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band, transfer=s.transfer)
        moved_keys += int(np.count_nonzero(np.floor(r["x_new"] / s.dx - (0.5 if degree == 2 else 0.0))
                                            != np.floor(x / s.dx - (0.5 if degree == 2 else 0.0))))
        x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
    assert moved_keys > s.n // 10          # the re-binning path is exercised
    assert ds.flags() == 0
    assert float(np.abs(got["x"] - x).max() / s.dx) <= 1e-11
    for key, a, ref in (("v", got["v"], v), ("B", got["B"], B), ("F", got["F"], F)):
        assert rel(a, ref) <= 1e-11, (key, rel(a, ref))
    raw = ds.state(raw=True)
    if dim == 3:
        tile, local = _base_keys(raw["cell"], raw["off"], s.cells, degree)
        check_binned_layout(tile, local)


@pytest.mark.parametrize("degree,precision", [(2, "fp64"), (3, "fp64"), (2, "fp32")])
def test_particles_leaving_the_grid_are_carried_and_the_rest_match(degree, precision):
    """A cluster moving 0.6 cells per step toward the -x face leaves the
    grid during the second step: from then on it sits in the dead region,
    carried unchanged (its state is the oracle's after the step that took it
    out), OUT_OF_DOMAIN is raised, and every other particle matches the
    oracle chained over the steps without the cluster once it is gone.
    Binary32 (quadratic: the steps before the last are fused with the next
    transfer to grid): bar 1e-5 per step, 4e-5 over the four steps."""
    import dataclasses
    b = _b()
    cells, dt = 16, 1e-2
    dx = 1.0 / cells
    bulk = scenes.random_particles(1500, dim=3, cells=cells, degree=degree, seed=41, margin=5.0,
                                   vel_sigma=0.2, f_sigma=0.02, b_sigma=0.01, model=0, precision=precision)
    rng = np.random.default_rng(42)
    start = 1.55 if degree == 2 else 2.05      # first cell whose support is inside
    xc = np.column_stack([(start + 0.1 * rng.random(40)) * dx,
                          (6.0 + 4.0 * rng.random((40, 2))) * dx])
    x = np.vstack([bulk.x, xc])
    v = np.vstack([bulk.v, np.tile([-0.6 * dx / dt, 0.0, 0.0], (40, 1))])
    B = np.concatenate([bulk.B, np.zeros((40, 3, 3))])
    F = np.concatenate([bulk.F, np.tile(np.eye(3), (40, 1, 1))])
    m = np.concatenate([bulk.m, np.ones(40)])
    s = dataclasses.replace(bulk, m=m, v=v, B=B, F=F, dt=dt).with_state(x=x)
    steps = 4
    ds = b.DeviceScene(s)
    ds.step(steps)
    got = ds.state()
    g = ogrid(s)
    cluster = np.arange(bulk.n, s.n)
    live = np.ones(s.n, bool)
    X, V, Bm, Fm = s.x.copy(), s.v.copy(), s.B.copy(), s.F.copy()
    left_at = None
    for k in range(steps):
        idx = np.flatnonzero(live)
        r = oracle.step(g, X[idx], V[idx], Bm[idx], Fm[idx], s.m[idx], s.V[idx], s.model, s.mu, s.lam, s.dt,
                        s.gravity, s.band)
        X[idx], V[idx], Bm[idx], Fm[idx] = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
        # supports that no longer fit: base node below 0 along x
        base = np.floor(X[:, 0] / dx - (0.5 if degree == 2 else 1.0))
        gone = live & (base < 0)
        if gone.any() and left_at is None:
            left_at = k
        live &= ~gone
    assert left_at is not None and 0 < left_at < steps - 1
    assert not live[cluster].any() and live[:bulk.n].all()
    assert ds.flags() & b.APIC_FLAG_OUT_OF_DOMAIN
    tol = 1e-11 if precision == "fp64" else steps * 1e-5
    for key, a, ref in (("x", got["x"], X), ("v", got["v"], V), ("B", got["B"], Bm), ("F", got["F"], Fm)):
        assert rel(a, ref) <= tol, (key, rel(a, ref))


def test_disk2d_fp64_ten_round_trips():
    """The rotating-disk transfer test: 10 P2G -> normalize -> G2P round
    trips at dt = 0 in binary64; per-transfer momenta conserved."""
    b = _b()
    s = scenes.disk2d()
    ds = b.DeviceScene(s)
    g = ogrid(s)
    x, v, B, F = s.x, s.v, s.B, s.F
    scale = float(np.sum(s.m * (np.linalg.norm(s.x, axis=1) * np.linalg.norm(s.v, axis=1))))
    for k in range(10):
        ref = oracle.step(g, x, v, B, F, s.m, s.V, 0, dt=0.0)
        t_p = oracle.particle_totals(x, v, B, s.m)
        ds.p2g()
        gd = ds.diagnostics(b.APIC_DIAG_GRID)
        pd = ds.diagnostics(b.APIC_DIAG_PARTICLES)
        ds.grid_update()
        ds.g2p()
        got = ds.state()
        pd1 = ds.diagnostics(b.APIC_DIAG_PARTICLES)
        for key, a, bb in (("v", got["v"], ref["v_new"]), ("B", got["B"], ref["B_new"])):
            assert rel(a, bb) <= 1e-12, (k, key, rel(a, bb))
        assert np.abs(got["x"] - s.x).max() == 0.0
        # kinetic energy (Sec. 3.1): particles before, grid, particles after
        t_g = oracle.grid_totals(g, ref["m"], ref["v"])
        t_p1 = oracle.particle_totals(ref["x_new"], ref["v_new"], ref["B_new"], s.m)
        assert pd[6] == pytest.approx(t_p[6], rel=1e-13), k
        assert gd[6] == pytest.approx(t_g[6], rel=1e-12), k
        assert pd1[6] == pytest.approx(t_p1[6], rel=1e-12), k
        # conservation per transfer (Sec. 5.2, 5.3): particles -> grid -> particles
        for t in (gd, pd1):
            assert np.abs(t[:2] - t_p[:2]).max() <= 1e-12 * scale
            assert abs(t[5] - t_p[5]) <= 1e-12 * scale
        assert np.abs(pd[:2] - t_p[:2]).max() <= 1e-14 * scale
        x, v, B, F = ref["x_new"], ref["v_new"], ref["B_new"], ref["F_new"]


def _base_keys(cell, off, cells, degree):
    """Tile id and local index (0..63) of each particle's base node."""
    base = np.where(off < 0.5, cell - 1, cell) if degree == 2 else cell - 1
    TN = [(c + 1 + 3) // 4 for c in cells]
    tile = (base[:, 0] >> 2) + TN[0] * ((base[:, 1] >> 2) + TN[1] * (base[:, 2] >> 2))
    local = (base[:, 0] & 3) + 4 * (base[:, 1] & 3) + 16 * (base[:, 2] & 3)
    return tile, local


def check_binned_layout(tile, local):
    """Particles of a tile are contiguous and level-major: every level lists
    distinct base nodes in increasing order, and the nodes of level j+1 are
    a subset of those of level j."""
    starts = np.flatnonzero(np.r_[True, tile[1:] != tile[:-1]])
    ends = np.r_[starts[1:], len(tile)]
    assert len(np.unique(tile[starts])) == len(starts), "a tile appears in two runs"
    for s0, e0 in zip(starts, ends):
        seq = local[s0:e0]
        cuts = np.flatnonzero(np.r_[True, seq[1:] <= seq[:-1]])
        levels = [seq[a:b] for a, b in zip(cuts, np.r_[cuts[1:], len(seq)])]
        for lo, hi in zip(levels, levels[1:]):
            assert set(hi.tolist()) <= set(lo.tolist())


def test_sort_bins_particles_level_major_by_base_node():
    b = _b()
    s = scenes.cube3d(cells=24, precision="fp32", steps=1)
    rng = np.random.default_rng(0)
    s = s.subset(rng.permutation(s.n))
    ds = b.DeviceScene(s)
    ds.sort()
    raw = ds.state(raw=True)
    # a permutation of the input rows, each row intact
    assert np.array_equal(np.sort(raw["id"]), np.arange(s.n))
    for k in ("cell", "off", "v", "B", "F", "m"):
        ref = {"cell": s.cell, "off": s.off, "v": s.v, "B": s.B, "F": s.F, "m": s.m}[k]
        assert np.array_equal(raw[k], ref[raw["id"]]), k
    tile, local = _base_keys(raw["cell"], raw["off"], s.cells, s.degree)
    check_binned_layout(tile, local)
    # every step keeps the particles binned
    ds.step(3)
    raw = ds.state(raw=True)
    tile, local = _base_keys(raw["cell"], raw["off"], s.cells, s.degree)
    check_binned_layout(tile, local)
    assert ds.flags() == 0


def test_empty_scene():
    b = _b()
    s = scenes.cube3d(cells=8, precision="fp32").subset(np.arange(0))
    ds = b.DeviceScene(s)
    ds.sort()
    ds.step(2)
    assert np.all(ds.export(b.APIC_GRID_MASS) == 0)
    assert ds.flags() == 0


@pytest.mark.parametrize("degree,transfer", [(2, 1), (1, 0), (3, 2)])
def test_empty_scene_adaptive_and_variants(degree, transfer):
    """No particles with adaptive steps (the bound is 0, so every step takes
    the cap), an RPIC or PIC transfer, or the multilinear kernel: the steps
    run, the clock advances by the cap and nothing is flagged."""
    import dataclasses
    b = _b()
    s = scenes.cube3d(cells=8, precision="fp32", degree=degree).subset(np.arange(0))
    s = dataclasses.replace(s, transfer=transfer, cfl=0.5)
    ds = b.DeviceScene(s, adaptive=True)
    ds.step(3)
    dt_last, t = ds.step_time()
    assert dt_last == s.dt and t == s.dt + s.dt + s.dt
    assert np.all(ds.export(b.APIC_GRID_MASS) == 0)
    assert ds.flags() == 0
    assert ds.cfl_dt(0.5) == np.inf


def test_lone_particle_is_stable_on_gpu():
    """Sec. 5.4 on the GPU: v and B unchanged, x moves by dt v."""
    b = _b()
    rng = np.random.default_rng(4)
    v = rng.normal(size=3)
    B = 0.01 * rng.normal(size=(3, 3))
    s = scenes.single_particle([0.41, 0.52, 0.47], v, B, dim=3, cells=8, dt=1e-2)
    ds = b.DeviceScene(s)
    ds.step(1)
    got = ds.state()
    np.testing.assert_allclose(got["v"][0], v, atol=1e-14)
    np.testing.assert_allclose(got["B"][0], B, atol=1e-15)
    np.testing.assert_allclose(got["x"][0], s.x[0] + 1e-2 * v, atol=1e-15)


def test_bad_particles_are_flagged_and_skipped():
    b = _b()
    s = scenes.random_particles(50, dim=3, cells=10, degree=2, seed=5)
    s.cell[0] = [0, 5, 5]          # support leaves the grid
    s.off[0] = [0.2, 0.5, 0.5]
    s.v[1, 0] = np.nan             # non-finite
    ds = b.DeviceScene(s)
    ds.p2g()
    assert ds.flags() & b.APIC_FLAG_OUT_OF_DOMAIN
    assert ds.flags() & b.APIC_FLAG_NONFINITE
    good = s.subset(np.arange(2, s.n))
    ref = oracle.p2g(ogrid(good), good.x, good.v, good.B, good.F, good.m, good.V, 1, good.mu, good.lam)
    assert rel(ds.export(b.APIC_GRID_MASS), ref["m"]) <= 1e-12


def test_invalid_arguments_are_rejected():
    b = _b()
    s = scenes.random_particles(10, dim=3, cells=8)
    ds = b.DeviceScene(s)
    ds.s.prm.dt = -1.0
    with pytest.raises(b.ApicError):
        ds.p2g()
    ds.s.prm.dt = 0.0
    ds.s.workspace_bytes = 16
    with pytest.raises(b.ApicError):
        ds.p2g()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cfl_dt_matches_oracle(precision):
    """apic_cfl_dt (Sec. 4.3) against the oracle's rule on the same particle
    state, before and after a step; the binary32 state is promoted exactly,
    so both sides reduce the same numbers in binary64."""
    b = _b()
    s = scenes.random_particles(5000, dim=3, cells=16, degree=2, seed=61, precision=precision, b_sigma=0.05,
                                vel_sigma=0.4, model=0)
    ds = b.DeviceScene(s)
    assert ds.cfl_dt(0.5) == pytest.approx(oracle.cfl_dt(s.dx, s.v, s.B, nu=0.5), rel=1e-14)
    ds.step(1)
    got = ds.state()
    v, B = np.ascontiguousarray(got["v"]), np.ascontiguousarray(got["B"])
    assert ds.cfl_dt() == pytest.approx(oracle.cfl_dt(s.dx, v, B), rel=1e-14)
    with pytest.raises(b.ApicError):
        ds.cfl_dt(0.0)
    rest = b.DeviceScene(s.with_state(v=0 * s.v, B=0 * s.B))
    assert rest.cfl_dt() == float("inf")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_energy_diagnostics_match_oracle(precision):
    """APIC_DIAG_ENERGY on the small elastic cube: kinetic energy (Sec. 3.1)
    and neo-Hookean potential Phi = sum V_p Psi(F_p) (Sec. 3.3) of the input
    state (both sides reduce the same numbers in binary64: 1e-12), then of
    the state after one step against the oracle's step (binary64: 1e-11;
    binary32: the first-order effect of the 1e-5 per-field bar on T and on
    Phi through P:dF).  The sticky band and gravity are on."""
    b = _b()
    s = scenes.cube3d(cells=24, precision=precision, steps=1)
    rng = np.random.default_rng(9)
    F = s.F + 0.02 * rng.normal(size=s.F.shape)            # stressed: Phi > 0
    if precision == "fp32":
        F = F.astype(np.float32).astype(np.float64)
    s = s.with_state(F=F)
    ds = b.DeviceScene(s)
    e0 = ds.diagnostics(b.APIC_DIAG_ENERGY)
    T0 = oracle.particle_totals(s.x, s.v, s.B, s.m)[6]
    P0 = oracle.potential(s.F, s.V, s.mu, s.lam)
    assert P0 > 0.0
    assert e0[0] == pytest.approx(T0, rel=1e-12)
    assert e0[1] == pytest.approx(P0, rel=1e-12)
    assert e0[2] == pytest.approx(T0 + P0, rel=1e-12)
    assert e0[7] == pytest.approx(float(s.m.sum()), rel=1e-13)
    ref = oracle.step(ogrid(s), s.x, s.v, s.B, s.F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band)
    ds.step(1)
    assert ds.flags() == 0
    e1 = ds.diagnostics(b.APIC_DIAG_ENERGY)
    T1 = oracle.particle_totals(ref["x_new"], ref["v_new"], ref["B_new"], s.m)[6]
    P1 = oracle.potential(ref["F_new"], s.V, s.mu, s.lam)
    if precision == "fp64":
        tol_t, tol_p = 1e-11 * T1, 1e-11 * P1
    else:
        vn = np.linalg.norm(ref["v_new"], axis=1)
        tol_t = 2 * TOL["fp32"] * float(np.abs(ref["v_new"]).max()) * float(np.sum(s.m * vn)) * np.sqrt(3)
        Pn = np.array([np.linalg.norm(oracle.neo_hookean_P(Fp, s.mu, s.lam)) for Fp in ref["F_new"]])
        tol_p = 2 * TOL["fp32"] * float(np.abs(ref["F_new"]).max()) * float(np.sum(s.V * Pn)) * 3
    assert abs(e1[0] - T1) <= tol_t, (e1[0], T1, tol_t)
    assert abs(e1[1] - P1) <= tol_p, (e1[1], P1, tol_p)
    # no model: no potential
    s0 = dataclasses_replace(s, model=0)
    ds0 = b.DeviceScene(s0)
    assert ds0.diagnostics(b.APIC_DIAG_ENERGY)[1] == 0.0


def dataclasses_replace(s, **kw):
    import dataclasses
    return dataclasses.replace(s, **kw)
