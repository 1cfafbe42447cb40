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


def test_admission_respects_order_count_and_memory_budget():
    from collections import deque
    from paper_1603_06188_amd import serve
    fp = {0: 40, 1: 30, 2: 100, 3: 10}
    reqs = [serve.Request(rid=k, arrival=0.1 * k, pool_index=k % 4, steps=50) for k in range(8)]
    pending = deque(reqs)
    # at t = 0.25 three have arrived; 40 + 30 fit in 80, the third (100) waits: the head is not overtaken
    got, used = serve.admit(pending, 0.25, 0, 0, fp.get, max_active=10, budget=80)
    assert [r.rid for r in got] == [0, 1] and used == 70 and pending[0].rid == 2
    # nothing resident: a request larger than the budget is admitted alone
    got, used = serve.admit(pending, 0.25, 0, 0, fp.get, max_active=10, budget=80)
    assert [r.rid for r in got] == [2] and used == 100
    # the count cap binds before the budget
    got, used = serve.admit(pending, 10.0, 1, 10, fp.get, max_active=3, budget=10 ** 6)
    assert [r.rid for r in got] == [3, 4] and used == 10 + 10 + 40
    # not yet arrived: nothing admitted
    got, used = serve.admit(pending, 0.45, 0, 0, fp.get, max_active=10, budget=10 ** 6)
    assert got == [] and used == 0


def test_scene_footprint_covers_planes_and_workspace():
    from paper_1603_06188_amd import binding as b, scenes
    s = scenes.body3d(7, n_target=5000)
    fp = b.scene_footprint_bytes(s, compensated=True, with_id=False)
    ws = b.apic_workspace_bytes(b.grid_desc(s, compensated=True), s.n)
    assert fp >= ws + s.n * (25 * 4 + 4)
