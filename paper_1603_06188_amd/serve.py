"""Serving many simulation requests on one GPU.

A request is a scene (a body on its own grid) and a number of explicit APIC
steps to run; its latency is the wall time from its arrival to the moment
its last step has completed on the device.  Two servers replay the same
arrival trace:

* ``BatchServer`` keeps every admitted request resident and advances all of
  them together, ``quantum`` steps per ``apic_step_batch`` call (one kernel
  launch per phase for all of them); requests join and leave between quanta.
  Arrived requests are admitted in arrival order while their device
  footprint (particle planes + workspace) fits the memory budget next to the
  requests already resident.
* ``SequentialServer`` solves one request at a time to completion with
  ``apic_step`` on that scene alone, first come first served.

Request bodies come from a pool of synthetic scenes generated once
(``request_pool``); each request copies its pool entry from pinned host
memory into its own device buffers on admission, so requests never share
state.  All numbers are produced by the library's kernels; this module only
schedules calls.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import List, Optional

import numpy as np
import torch

from . import binding as b
from . import scenes


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float         # seconds after the start of the trace
    pool_index: int
    steps: int
    # filled by a server
    start: float = math.nan
    finish: float = math.nan
    scene: Optional[b.DeviceScene] = None
    left: int = 0

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def request_pool(count: int = 32, seed: int = 5, n_lo: float = 1e4, n_hi: float = 1e6,
                 precision: str = "fp32") -> List[scenes.Scene]:
    """Bodies with N log-uniform in [n_lo, n_hi] (grid, material, gravity and
    dt as in the batched workload)."""
    return [scenes.body3d(seed + k, n_lo=n_lo, n_hi=n_hi, precision=precision) for k in range(count)]


def poisson_trace(rate: float, duration: float, pool_size: int, seed: int = 6, steps_lo: int = 50,
                  steps_hi: int = 500) -> List[Request]:
    """Arrivals of a Poisson process of `rate` requests/s over `duration` s;
    each request picks a pool entry uniformly and U{steps_lo..steps_hi} steps."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        out.append(Request(rid=len(out), arrival=t, pool_index=int(rng.integers(pool_size)),
                           steps=int(rng.integers(steps_lo, steps_hi + 1))))
    return out


class Pool:
    """Pool scenes packed once in pinned host memory; every request gets its
    own device copy (particles and workspace) on admission."""

    def __init__(self, pool, compensated: bool = True, device: str = "cuda", with_id: bool = False):
        self.with_id = with_id
        self.templates = []
        self.footprints = []
        for s in pool:
            dtype = torch.float32 if s.precision == "fp32" else torch.float64
            f, cell = b.DeviceScene.pack(s, dtype)
            self.templates.append((s, (f.pin_memory(), cell.pin_memory())))
            self.footprints.append(b.scene_footprint_bytes(s, compensated=compensated, with_id=with_id))
        self.compensated = compensated
        self.device = device

    def __len__(self):
        return len(self.templates)

    def instantiate(self, k: int) -> b.DeviceScene:
        s, packed = self.templates[k]
        return b.DeviceScene(s, device=self.device, compensated=self.compensated, with_id=self.with_id,
                             packed=packed)

    def particles(self, k: int) -> int:
        return self.templates[k][0].n

    def footprint(self, k: int) -> int:
        """Device bytes a request on pool entry k holds while resident."""
        return self.footprints[k]


@dataclasses.dataclass
class ServeStats:
    latencies: np.ndarray
    wall: float
    particle_updates: float

    @property
    def throughput(self) -> float:
        return self.particle_updates / self.wall

    def percentile(self, q: float) -> float:
        return float(np.percentile(self.latencies, q)) if self.latencies.size else math.nan


def _wait_until(t0: float, t: float) -> None:
    dt = t - (time.perf_counter() - t0)
    if dt > 0:
        time.sleep(dt)


def admit(pending, now: float, n_active: int, used: int, footprint, max_active: int, budget: int):
    """Admission of the batch server: pops from the head of `pending` (in
    arrival order) the requests that have arrived by `now`, while the number
    of resident requests stays within `max_active` and their footprints
    (`footprint(pool_index)` bytes each) within `budget`.  The head is never
    overtaken; a request larger than the whole budget is admitted alone when
    nothing else is resident.  Returns (admitted requests, bytes in use)."""
    out = []
    while pending and pending[0].arrival <= now and n_active + len(out) < max_active:
        fp = footprint(pending[0].pool_index)
        if used + fp > budget and n_active + len(out) > 0:
            break
        out.append(pending.popleft())
        used += fp
    return out, used


class BatchServer:
    def __init__(self, pool, quantum: int = 10, max_active: int = 256, compensated: bool = True,
                 device: str = "cuda", keep_scenes: bool = False, mem_budget: Optional[int] = None):
        self.pool = pool if hasattr(pool, "instantiate") else Pool(pool, compensated, device)
        self.quantum = int(quantum)
        self.max_active = int(max_active)
        # device memory for resident requests: by default 80 % of what is free now
        self.mem_budget = int(mem_budget if mem_budget is not None else 0.8 * torch.cuda.mem_get_info()[0])
        self.keep = keep_scenes
        self.bbytes = b.apic_batch_workspace_bytes(self.max_active)
        self.bws = torch.empty(self.bbytes + 256, dtype=torch.uint8, device=device)
        self.bptr = (self.bws.data_ptr() + 255) // 256 * 256

    def run(self, trace: List[Request]) -> ServeStats:
        pending = deque(sorted(trace, key=lambda r: r.arrival))
        active: List[Request] = []
        done: List[Request] = []
        work = 0.0
        used = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            admitted, used = admit(pending, now, len(active), used, self.pool.footprint, self.max_active,
                                   self.mem_budget)
            for r in admitted:
                r.scene = self.pool.instantiate(r.pool_index)
                r.left = r.steps
                r.start = now
                active.append(r)
            if not active:
                _wait_until(t0, pending[0].arrival)
                continue
            q = min(self.quantum, min(r.left for r in active))
            b.apic_step_batch([r.scene.s for r in active], q, self.bptr, self.bbytes)
            torch.cuda.synchronize()
            now = time.perf_counter() - t0
            still = []
            for r in active:
                r.left -= q
                work += r.scene.n * q
                if r.left == 0:
                    r.finish = now
                    used -= self.pool.footprint(r.pool_index)
                    if not self.keep:
                        r.scene = None
                    done.append(r)
                else:
                    still.append(r)
            active = still
        wall = time.perf_counter() - t0
        return ServeStats(np.array([r.latency for r in done]), wall, work)


class SequentialServer:
    def __init__(self, pool, compensated: bool = True, device: str = "cuda", keep_scenes: bool = False):
        self.pool = pool if hasattr(pool, "instantiate") else Pool(pool, compensated, device)
        self.keep = keep_scenes

    def run(self, trace: List[Request]) -> ServeStats:
        queue = deque(sorted(trace, key=lambda r: r.arrival))
        done: List[Request] = []
        work = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while queue:
            r = queue.popleft()
            _wait_until(t0, r.arrival)
            r.start = time.perf_counter() - t0
            r.scene = self.pool.instantiate(r.pool_index)
            r.scene.step(r.steps)
            torch.cuda.synchronize()
            r.finish = time.perf_counter() - t0
            work += r.scene.n * r.steps
            if not self.keep:
                r.scene = None
            done.append(r)
        wall = time.perf_counter() - t0
        return ServeStats(np.array([r.latency for r in done]), wall, work)


def saturated_rate(pool, steps: int = 50, copies: int = 2, quantum: int = 10) -> float:
    """Closed-loop capacity of the batch server, in particle-updates/s: every
    pool entry `copies` times admitted at t = 0 and run for `steps` steps."""
    trace = [Request(rid=k, arrival=0.0, pool_index=k % len(pool), steps=steps) for k in range(copies * len(pool))]
    stats = BatchServer(pool, quantum=quantum).run(trace)
    return stats.throughput
