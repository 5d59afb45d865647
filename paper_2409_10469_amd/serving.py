"""Batched-serving driver: a seeded Poisson stream of MPPI requests with mixed tasks,
admitted into a Batch by its HBM budget, each living a fixed number of control steps.

The batch itself (allocation, tile queues, graph launch, update and plant tails) is in
libmppi.so; this module only generates requests, keeps the FIFO of those waiting for
memory, and records per-step latency with HIP events on the batch's stream.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding as B
from . import workloads as W
from .timing import DeviceEvent

# per-task controller settings (flat walking, heightfield walking, box climbing, box pushing)
TASKS = {
    "flat_walk": dict(workload=W.FLAT_WALK, dt=0.02, nk=4, sigma=0.3, lam=0.1),
    "heightfield_walk": dict(workload=W.TERRAIN_WALK, dt=0.01, nk=6, sigma=0.25, lam=0.05),
    "box_climb": dict(workload=W.BOX_CLIMB, dt=0.01, nk=6, sigma=0.25, lam=0.05),
    "box_push": dict(workload=W.BOX_PUSH, dt=0.01, nk=8, sigma=0.25, lam=0.05),
}
K_RANGE = (256, 4096)
H_RANGE = (20, 80)


def draw_request(rng, rid):
    task = list(TASKS)[rng.integers(len(TASKS))]
    K = int(round(math.exp(rng.uniform(math.log(K_RANGE[0]), math.log(K_RANGE[1])))))
    H = int(rng.integers(H_RANGE[0], H_RANGE[1] + 1))
    return dict(id=rid, task=task, K=K, H=H, seed=int(rng.integers(1 << 30)))


class ServingSim:
    def __init__(self, seed=0, n_target=256, budget_bytes=64 << 20, lifetime=200, arith="fp64", max_instances=512):
        import torch
        self.rng = np.random.default_rng(seed)
        self.age_rng = np.random.default_rng([seed, 1])  # ages of the prefilled instances
        self.lifetime = lifetime
        self.rate = n_target / lifetime
        self.arith = arith
        self.stream = torch.cuda.Stream()
        self.batch = B.Batch(max_instances=max_instances, budget_bytes=budget_bytes, max_horizon=H_RANGE[1],
                             max_hf_cells=W.HF_N * W.HF_N, arith=arith, stream=self.stream)
        self.slots, self.models = {}, {}
        for name, t in TASKS.items():
            m = B.Model(W.model_dict(t["workload"], 0))
            self.models[name] = m
            self.slots[name] = self.batch.add_model(m)
        self.pending = []      # FIFO of (request, arrival step)
        self.live = {}         # instance id -> (request, admitted step)
        self.step_no = 0
        self.next_rid = 0
        self.queue_delay = []  # steps between arrival and admission
        self.refused = 0

    def _params(self, req):
        t = TASKS[req["task"]]
        return W.params_dict(t["workload"], req["seed"], K=req["K"], H=req["H"], nk=t["nk"], dt=t["dt"],
                             sigma=t["sigma"], lam=t["lam"], instance=req["id"] & 0xFFFFFFFF, arith=self.arith)

    def _try_admit(self):
        while self.pending:
            req, t_arr = self.pending[0]
            t = TASKS[req["task"]]
            x0 = W.initial_state(req["seed"], t["workload"]["scene"])
            iid = self.batch.admit(self.slots[req["task"]], self._params(req), x0, W.stance_knots(t["nk"]))
            if iid is None:
                self.refused += 1
                return
            self.pending.pop(0)
            self.live[iid] = (req, self.step_no)
            self.queue_delay.append(self.step_no - t_arr)

    def arrive(self, n):
        for _ in range(n):
            self.pending.append((draw_request(self.rng, self.next_rid), self.step_no))
            self.next_rid += 1

    def prefill(self, n):
        """n requests as a snapshot of the steady state: the admitted ones get ages drawn
        uniformly from [0, lifetime), so their departures spread over one lifetime
        instead of coinciding while the Poisson arrivals continue."""
        before = set(self.live)
        self.arrive(n)
        self._try_admit()
        for iid in sorted(set(self.live) - before):
            req, t0 = self.live[iid]
            self.live[iid] = (req, t0 - int(self.age_rng.integers(self.lifetime)))

    def host_tick(self):
        """Departures, Poisson arrivals and admissions before a control step."""
        for iid, (req, t0) in list(self.live.items()):
            if self.step_no - t0 >= self.lifetime:
                self.batch.remove(iid)
                del self.live[iid]
        self.arrive(int(self.rng.poisson(self.rate)))
        self._try_admit()

    def work(self):
        """Rollout-steps of the next control step and its algorithmic flops."""
        from .roofline import flops_per_rollout_step
        rs, fl = 0, 0.0
        for req, _ in self.live.values():
            t = TASKS[req["task"]]
            n = req["K"] * req["H"]
            rs += n
            fl += n * flops_per_rollout_step(t["workload"]["scene"], t["nk"])
        return rs, fl

    def run(self, steps, warmup=3, autotune=True):
        import torch
        tune = None
        for _ in range(warmup):
            self.host_tick()
            with torch.cuda.stream(self.stream):
                self.batch.step()
            self.step_no += 1
        if autotune:
            self.stream.synchronize()
            tune = self.batch.autotune(steps=1) + (self.batch.tuning()[2],)
        self.stream.synchronize()
        lat, host_ms, work, flops, live = [], [], 0, 0.0, []
        evs = [(DeviceEvent(), DeviceEvent()) for _ in range(steps)]
        t0 = time.perf_counter()
        for i in range(steps):
            h0 = time.perf_counter()
            self.host_tick()
            host_ms.append((time.perf_counter() - h0) * 1e3)
            rs, fl = self.work()
            work += rs
            flops += fl
            live.append(len(self.live))
            evs[i][0].record(self.stream)
            self.batch.step()
            evs[i][1].record(self.stream)
            self.step_no += 1
        self.stream.synchronize()
        elapsed = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(b) for a, b in evs])
        return dict(elapsed=elapsed, latency_ms=lat, host_ms=np.array(host_ms), rollout_steps=work, flops=flops,
                    live=np.array(live), queue_delay=np.array(self.queue_delay), refused=self.refused, tune=tune,
                    stats=self.batch.stats())
