"""Batched steps (apic_step_batch): one launch per phase for many scenes.

Each scene of a batch must evolve as it does alone: the same kernels run on
its own memory.  Checked against the per-scene path and against the FP64
oracle chained over the steps.
"""
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


def _bodies(precision, sizes=(1200, 5000, 20000, 3000, 800), seed=100):
    return [scenes.body3d(seed + k, n_target=t, precision=precision) for k, t in enumerate(sizes)]


def _close(ga, gb, tol, label):
    for key in ("x", "v", "B", "F", "m"):
        e = rel(ga[key], gb[key])
        assert e <= tol, (label, key, e)


# The same kernels on the same data: a layout is a function of the one
# before it (movers ranked by their old place, not by counter order), so a
# scene in a batch and the same scene alone give the same bits.
@pytest.mark.parametrize("precision,steps,tol", [("fp64", 4, 0.0), ("fp32", 4, 0.0)])
def test_batch_matches_each_scene_alone(precision, steps, tol):
    b = _b()
    hosts = _bodies(precision)
    alone = [b.DeviceScene(h) for h in hosts]
    for d in alone:
        d.step(steps)
    batch = b.SceneBatch([b.DeviceScene(h) for h in hosts])
    batch.step(steps)
    for k, (d0, d1) in enumerate(zip(alone, batch.scenes)):
        _close(d1.state(), d0.state(), tol, f"scene {k}")
        assert d1.flags() == d0.flags() == 0


def test_batch_matches_chained_oracle_fp64():
    b = _b()
    hosts = _bodies("fp64", sizes=(1500, 700, 2500), seed=200)
    batch = b.SceneBatch([b.DeviceScene(h) for h in hosts])
    steps = 3
    batch.step(steps)
    for k, (h, d) in enumerate(zip(hosts, batch.scenes)):
        g = oracle.Grid(h.dim, h.degree, h.cells, h.dx)
        x, v, B, F = h.x, h.v, h.B, h.F
        for _ in range(steps):
            r = oracle.step(g, x, v, B, F, h.m, h.V, h.model, h.mu, h.lam, h.dt, h.gravity, h.band, transfer=h.transfer)
            x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
        got = d.state()
        assert float(np.abs(got["x"] - x).max() / h.dx) <= 1e-11, k
        for key, ref in (("v", v), ("B", B), ("F", F)):
            assert rel(got[key], ref) <= 1e-11, (k, key, rel(got[key], ref))


def test_batched_and_per_scene_calls_interleave():
    """batch 2 steps, per-scene 3 steps, batch 1 step == 6 steps alone."""
    b = _b()
    hosts = _bodies("fp64", sizes=(900, 4000, 1600), seed=300)
    alone = [b.DeviceScene(h) for h in hosts]
    for d in alone:
        d.step(6)
    batch = b.SceneBatch([b.DeviceScene(h) for h in hosts])
    batch.step(2)
    batch.step_each(3)
    batch.step(1)
    for k, (d0, d1) in enumerate(zip(alone, batch.scenes)):
        _close(d1.state(), d0.state(), 1e-12, f"scene {k}")


def test_batch_edge_cases():
    """An empty scene, a scene already binned next to fresh ones, zero steps,
    and a batch of one."""
    b = _b()
    hosts = _bodies("fp64", sizes=(1000, 2000), seed=400)
    empty = hosts[0].subset(np.arange(0))
    ds = [b.DeviceScene(h) for h in (hosts[0], empty, hosts[1])]
    ds[2].sort()
    batch = b.SceneBatch(ds)
    batch.step(0)
    batch.step(3)
    assert ds[1].n == 0 and np.all(ds[1].export(b.APIC_GRID_MASS) == 0)
    ref = [b.DeviceScene(h) for h in (hosts[0], hosts[1])]
    for d in ref:
        d.step(3)
    _close(ds[0].state(), ref[0].state(), 1e-12, "scene 0")
    _close(ds[2].state(), ref[1].state(), 1e-12, "scene 2")
    one = b.SceneBatch([b.DeviceScene(hosts[1])])
    one.step(3)
    _close(one.scenes[0].state(), ref[1].state(), 1e-12, "batch of one")


def test_batch_rejects_bad_arguments():
    b = _b()
    h32 = scenes.body3d(500, n_target=800, precision="fp32")
    h64 = scenes.body3d(501, n_target=800, precision="fp64")
    d32, d64 = b.DeviceScene(h32), b.DeviceScene(h64)
    with pytest.raises(b.ApicError):
        b.SceneBatch([d32, d64]).step(1)
    with pytest.raises(b.ApicError):
        b.SceneBatch([d32, d32]).step(1)
    batch = b.SceneBatch([d32])
    with pytest.raises(b.ApicError):
        b.apic_step_batch([d32.s], 1, batch.bptr, 16)
    with pytest.raises(b.ApicError):
        b.apic_step_batch([d32.s], 1, batch.bptr + 8, batch.bbytes)


def test_batch_fp32_one_step_matches_oracle():
    """Binary32 bodies (rigid velocity and spin, compensated): one batched
    step against the FP64 oracle per body, within the binary32 bar of 1e-5
    per field (positions in cell units)."""
    b = _b()
    hosts = _bodies("fp32", sizes=(1500, 6000, 800), seed=500)
    batch = b.SceneBatch([b.DeviceScene(h, compensated=True) for h in hosts])
    batch.step(1)
    for k, (h, d) in enumerate(zip(hosts, batch.scenes)):
        g = oracle.Grid(h.dim, h.degree, h.cells, h.dx)
        r = oracle.step(g, h.x, h.v, h.B, h.F, h.m, h.V, h.model, h.mu, h.lam, h.dt, h.gravity, h.band, transfer=h.transfer)
        got = d.state()
        assert d.flags() == 0
        assert float(np.abs(got["x"] - r["x_new"]).max() / h.dx) <= 1e-5, k
        for key in ("v", "B", "F"):
            assert rel(got[key], r[key + "_new"]) <= 1e-5, (k, key, rel(got[key], r[key + "_new"]))


def test_every_launch_plan_gives_the_same_bits():
    """Each launch plan of apic_step_batch (blocks per scene share, one block
    per work item or a persistent launch taking items from a device queue)
    runs the same work items, so four batched steps under every plan equal
    the scenes stepped alone bit for bit."""
    b = _b()
    hosts = _bodies("fp32", sizes=(1200, 5000, 20000, 3000, 800), seed=600)
    alone = [b.DeviceScene(h, compensated=True) for h in hosts]
    for d in alone:
        d.step(4)
    want = [d.state() for d in alone]
    try:
        for p in range(b.apic_batch_plan_count()):
            b.apic_batch_set_plan(p)
            batch = b.SceneBatch([b.DeviceScene(h, compensated=True) for h in hosts])
            batch.step(4)
            for k, d in enumerate(batch.scenes):
                _close(d.state(), want[k], 0.0, f"plan {p} scene {k}")
                assert d.flags() == 0
    finally:
        b.apic_batch_set_plan(-1)


@pytest.mark.parametrize("plan", [0, 3])
def test_graph_replays_equal_direct_launches(plan):
    """APIC_OPT_BATCH_GRAPH: the call's step sequence is captured once and
    replayed by the later calls.  Three calls, with per-scene steps (eager
    launches) between them, give on every replay the bits of the same calls
    launched directly."""
    b = _b()
    hosts = _bodies("fp32", sizes=(900, 4000, 1600, 12000), seed=700)
    direct = b.SceneBatch([b.DeviceScene(h, compensated=True) for h in hosts])
    graph = b.SceneBatch([b.DeviceScene(h, compensated=True, batch_graph=True) for h in hosts])
    try:
        b.apic_batch_set_plan(plan)
        for call in range(3):
            direct.step(2)
            graph.step(2)
            for k, (dd, dg) in enumerate(zip(direct.scenes, graph.scenes)):
                _close(dg.state(), dd.state(), 0.0, f"call {call} scene {k}")
                assert dg.flags() == 0
            direct.step_each(1)
            graph.step_each(1)
    finally:
        b.apic_batch_set_plan(-1)
    for k, (dd, dg) in enumerate(zip(direct.scenes, graph.scenes)):
        _close(dg.state(), dd.state(), 0.0, f"end scene {k}")


def test_tuner_times_every_plan_then_keeps_the_fastest():
    """With no plan forced, the first calls of a batch time each plan (twice)
    and later calls use the one with the least time per particle-step."""
    b = _b()
    b.apic_batch_set_plan(-1)
    hosts = _bodies("fp64", sizes=(3000, 700, 1500, 2200, 900, 1300, 600), seed=800)
    batch = b.SceneBatch([b.DeviceScene(h) for h in hosts])
    count = b.apic_batch_plan_count()
    for _ in range(2 * count + 1):
        batch.step(1)
    plan, ns = batch.tuning()
    print("tuned plan", plan, ns, flush=True)
    assert 0 <= plan < count
    assert all(np.isfinite(v) and v > 0 for v in ns)
    assert ns[plan] == min(ns)
    for d in batch.scenes:
        assert d.flags() == 0
