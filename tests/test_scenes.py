"""Seeded generators: counts, ranges and exactness of the cell + offset split."""
import numpy as np
import pytest

from paper_1603_06188_amd import scenes


def test_disk2d_shape_and_count():
    s = scenes.disk2d()
    exp = scenes.expected_count_disk()
    assert abs(s.n - exp) < 4 * np.sqrt(exp)
    assert np.all(np.sum((s.x - 0.5) ** 2, axis=1) < 0.3 ** 2)
    assert s.m.sum() == pytest.approx(1.0, rel=1e-12)
    assert np.all(s.B == 0) and np.all(s.F == np.eye(2))
    # deterministic for a fixed seed
    assert scenes.disk2d().n == s.n and np.array_equal(scenes.disk2d().v, s.v)


def test_cube3d_count_and_layout():
    s = scenes.cube3d(cells=32)
    assert s.n == (16 ** 3) * 8
    assert s.x.min() >= 0.25 and s.x.max() < 0.75
    # cell + offset split is exact and offsets are binary32 values in [0, 1)
    assert np.all((s.off >= 0) & (s.off < 1))
    assert np.array_equal(s.off.astype(np.float32).astype(np.float64), s.off)
    assert np.array_equal(np.floor(s.x / s.dx).astype(np.int32), s.cell)
    assert s.V[0] == pytest.approx(s.dx ** 3 / 8)


def test_cube3d_full_size_count():
    # 64^3 cells of the 128^3 grid, 8 per cell
    s = scenes.cube3d()
    assert s.n == 2_097_152


def test_spheres3d_small():
    s = scenes.spheres3d(cells=64)
    exp = 2 * 4.0 / 3.0 * np.pi * 0.2 ** 3 * 64 ** 3 * 8
    assert abs(s.n - exp) < 4 * np.sqrt(exp)
    left = s.x[:, 0] < 0.5
    assert np.allclose(s.v[left, 0].mean(), 1.0, atol=0.05)
    assert np.allclose(s.v[~left, 0].mean(), -1.0, atol=0.05)
