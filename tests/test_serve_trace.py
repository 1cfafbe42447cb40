"""Arrival traces of the serving replay (host logic, no GPU)."""
import numpy as np


def test_poisson_trace_statistics():
    from paper_1603_06188_amd import serve
    tr = serve.poisson_trace(rate=200.0, duration=20.0, pool_size=8, seed=1)
    gaps = np.diff([0.0] + [r.arrival for r in tr])
    assert abs(len(tr) / 20.0 - 200.0) < 200.0 * 0.05
    assert abs(gaps.mean() - 1 / 200.0) < 0.05 / 200.0 * 20
    steps = np.array([r.steps for r in tr])
    assert steps.min() >= 50 and steps.max() <= 500 and abs(steps.mean() - 275) < 10
