"""Record lists of a layout when a whole tile empties in one step.

The key pass claims a tile's record in the new layout when it starts the
tile, so a tile all of whose particles leave it is listed without particles
in the next layout, and the steps after walk it as an empty tile (zero slab,
no particles).  A cluster that moves rigidly by 0.6 cells per step from the
last key layer of one tile into the next empties its tile in the first step;
binary64 steps through one apic_step call are compared with the oracle
chained over the same steps (bar 1e-11, as for the other chained steps).
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1603_06188_amd import scenes

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max()) / max(float(np.abs(b).max()), 1e-300)


def _base(x, dx):
    return np.floor(x / dx - 0.5).astype(np.int64)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 4e-5)])
def test_tile_emptied_in_one_step_is_walked_empty(precision, tol):
    from paper_1603_06188_amd import binding as b

    cells, dt = 16, 1e-2
    dx = 1.0 / cells
    rng = np.random.default_rng(11)
    # cluster A: base node 7 along x (the last key layer of the tile of base
    # nodes 4..7), x/dx in [7.95, 8.45); +0.6 cells takes all of it to base 8
    na = 240
    xa = np.stack([rng.uniform(7.95, 8.45, na), rng.uniform(5.0, 7.0, na), rng.uniform(5.0, 7.0, na)], 1) * dx
    va = np.tile([0.6 * dx / dt, 0.0, 0.0], (na, 1))
    # cluster B: slow particles in other tiles, away from A's supports
    nb = 360
    xb = np.stack([rng.uniform(11.0, 13.5, nb), rng.uniform(3.0, 12.0, nb), rng.uniform(3.0, 12.0, nb)], 1) * dx
    vb = rng.normal(0.0, 0.05, (nb, 3))
    tmpl = scenes.random_particles(na + nb, dim=3, cells=cells, degree=2, seed=3, model=0, dt=dt,
                                   precision=precision)
    s = tmpl.with_state(x=np.concatenate([xa, xb]), v=np.concatenate([va, vb]),
                        B=np.zeros((na + nb, 3, 3)))
    s = dataclasses.replace(s, dt=dt)
    steps = 3

    g = oracle.Grid(s.dim, s.degree, s.cells, s.dx)
    x, v, B, F = s.x, s.v, s.B, s.F
    for k in range(steps):
        r = oracle.step(g, x, v, B, F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band,
                        transfer=s.transfer)
        if k == 0:
            before = _base(x[:na], dx) // 4
            after = _base(r["x_new"][:na], dx) // 4
            # every particle of A starts in one tile and leaves it in this step
            assert len({tuple(t) for t in before}) == 1
            assert np.all(after[:, 0] == before[0, 0] + 1) and np.all(after[:, 1:] == before[:, 1:])
        x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]

    ds = b.DeviceScene(s)
    ds.step(steps)
    got = ds.state()
    assert ds.flags() == 0
    assert float(np.abs(got["x"] - x).max() / dx) <= tol
    for key, a, ref in (("v", got["v"], v), ("B", got["B"], B), ("F", got["F"], F)):
        assert _rel(a, ref) <= tol, (key, _rel(a, ref))
