"""Host logic of the serving replay (arrival traces, admission, the server
loops against a fake device): no GPU."""
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


class _FakeScene:
    def __init__(self, n):
        self.n = n
        self.s = object()
        self.steps = 0

    def step(self, k):
        self.steps += k


class _FakePool:
    """Pool interface of serve.Pool without device memory."""
    sizes = [1000, 5000, 20000]

    def __len__(self):
        return len(self.sizes)

    def footprint(self, k):
        return self.sizes[k] * 200

    def particles(self, k):
        return self.sizes[k]

    def instantiate(self, k):
        return _FakeScene(self.sizes[k])


def test_server_loops_on_a_fake_device(monkeypatch):
    """Every request is admitted, advanced by exactly its steps and retired;
    the batch loop never holds more than max_active scenes or steps past a
    request's remaining count."""
    import torch
    from paper_1603_06188_amd import serve
    calls = []
    resident = {}

    def fake_step_batch(scenes, n_steps, ptr, nbytes, stream=None):
        calls.append((len(scenes), n_steps))
        for sc in scenes:
            resident[id(sc)] = resident.get(id(sc), 0) + n_steps

    monkeypatch.setattr(serve.b, "apic_step_batch", fake_step_batch)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a: None)
    trace = serve.poisson_trace(rate=2000.0, duration=0.02, pool_size=3, seed=3, steps_lo=20, steps_hi=45)
    assert len(trace) > 10
    pool = _FakePool()
    srv = serve.BatchServer(pool, quantum=10, max_active=4, device="cpu", mem_budget=6_000_000, keep_scenes=True)
    st = srv.run(trace)
    assert len(st.latencies) == len(trace) and (st.latencies >= 0).all()
    assert st.particle_updates == sum(pool.sizes[r.pool_index] * r.steps for r in trace)
    assert all(1 <= n <= 4 and 1 <= q <= 10 for n, q in calls)
    assert sorted(resident.values()) == sorted(r.steps for r in trace)
    seq = serve.SequentialServer(pool, keep_scenes=True).run(
        [serve.Request(rid=r.rid, arrival=r.arrival, pool_index=r.pool_index, steps=r.steps) for r in trace])
    assert len(seq.latencies) == len(trace) and seq.particle_updates == st.particle_updates
