"""Grids at the largest sizes the packed cell index allows: 1024 cells along
an axis in 3D (10 bits per axis), 65535 in 2D (16 bits), with the particles
in the last cells of that axis, moving toward its end until the quadratic
supports of some of them reach its last node.  Steps through one
apic_step call are compared with the oracle chained over the same steps
(binary64 bar 1e-11, binary32 4e-5 over the steps, as for the other chained
steps).

The oracle takes absolute binary64 coordinates, which at x/dx ~ 65534 round
at ~1.5e-11 cells and would put its own error above the binary64 bar.  It runs
instead in a frame moved by a whole number of cells along the long axis, on a
grid of 16 cells there that ends where the large grid ends: with no sticky band
and no gravity the step depends on the positions only through x_p - x_i on the
node lattice (Sec. 3.2-3.5), so the move changes nothing but that rounding.
The device's cell + offset state is moved back by the same number of cells
before the comparison."""
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


def _scene(dim, cells, precision, n=400, seed=21):
    dx = 1.0 / 8
    rng = np.random.default_rng(seed)
    lo = np.array([cells[0] - 6.0] + [2.0] * (dim - 1))
    hi = np.array([cells[0] - 1.1] + [6.0] * (dim - 1))
    x = (lo + rng.random((n, dim)) * (hi - lo)) * dx
    dt = 1e-2
    v = rng.normal(0.0, 0.03, (n, dim)) * dx / dt
    v[:, 0] += 0.1 * dx / dt  # toward the end of the long axis, 0.1 cells per step
    tmpl = scenes.random_particles(n, dim=dim, cells=8, degree=2, seed=seed, model=1, dt=dt, precision=precision)
    tmpl = dataclasses.replace(tmpl, cells=tuple(cells), dx=dx)
    s = tmpl.with_state(x=x, v=v)
    return dataclasses.replace(s, dt=dt)


SHORT = 16  # cells of the oracle's grid along the long axis


@pytest.mark.parametrize("dim,cells", [(3, (1024, 8, 8)), (2, (65535, 8))])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 4e-5)])
def test_particles_in_the_last_cells_of_the_largest_grid(dim, cells, precision, tol):
    from paper_1603_06188_amd import binding as b

    s = _scene(dim, cells, precision)
    shift = np.zeros(dim, dtype=np.int64)
    shift[0] = cells[0] - SHORT
    steps = 3
    g = oracle.Grid(s.dim, s.degree, (SHORT,) + tuple(cells[1:]), s.dx)
    x = (s.cell.astype(np.int64) - shift + s.off) * s.dx
    v, B, F = s.v, s.B, s.F
    for _ in range(steps):
        r = oracle.step(g, x, v, B, F, s.m, s.V, s.model, s.mu, s.lam, s.dt, s.gravity, s.band,
                        transfer=s.transfer)
        x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
    # the supports of some particles reach the last node of the long axis
    base = np.floor(x[:, 0] / s.dx - 0.5).astype(np.int64)
    assert int((base + s.degree == SHORT).sum()) > 0 and int(base.max()) + s.degree <= SHORT

    ds = b.DeviceScene(s)
    ds.step(steps)
    got = ds.state()
    assert ds.flags() == 0
    xg = (got["cell"] - shift + got["off"]) * s.dx
    assert float(np.abs(xg - x).max() / s.dx) <= tol
    for key, a, ref in (("v", got["v"], v), ("B", got["B"], B), ("F", got["F"], F)):
        assert _rel(a, ref) <= tol, (key, _rel(a, ref))
