"""Served stream of simulation runs with continuous batching.

Requests (a run description, a step count and an arrival time) are admitted
while the device has room: the sum of the active runs' exact arena sizes
(`footprint_bytes`) stays under a cap, and the number of active runs under a
slot limit.  Admitted runs stay resident on the device until they finish.
All active runs advance together in ticks: one batch (grouped launches, one
captured graph per batched step) advances each run by up to `tick_steps`
steps.  Sweep tile shapes come from the batch-level tuner, run once when
the batch first holds `tune_min` runs; later admissions of the same
precision class take the tuned shape.  Between ticks finished runs are read back and released, and arrived
requests are admitted, so new work joins while other runs are mid-flight.
The batch is rebuilt only when its membership changed.

Each result is what the run gives alone: a member's arithmetic does not
depend on the other members of its batch.

Only argument marshalling and scheduling live here; every step of every run
runs in the HIP library.
"""
from __future__ import annotations

import dataclasses
import time
from concurrent.futures import ThreadPoolExecutor
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    desc: dict              # run descriptor (workloads.Workload.descriptor())
    bunch: Callable         # () -> (xyz, u, q_macro), drawn on admission
    n_particles: int
    steps: int
    keep_fields: Sequence[str] = ()


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    nodes: int
    particles: int
    power: np.ndarray       # lab-frame power through the diagnostic plane, per step
    bunching: float
    fields: Dict[str, np.ndarray]

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    def __init__(self, req: Request, eng, admitted: float, footprint: int):
        self.req = req
        self.eng = eng
        self.admitted = admitted
        self.footprint = footprint
        self.done = 0


class Server:
    """Continuous-batching runner on one device.

    cap_bytes: admission limit on the sum of active arena sizes.
    max_active: slot limit (runs per batch).
    tick_steps: steps per tick (the granularity of admission and retirement).
        A multiple of the runs' sort interval keeps every member's sorts on
        the same steps (members join at tick boundaries), so the batch
        replays its step without the sort passes on the other steps.
    autotune: pick each run's sweep tile shape with the library's autotuner
        (runs timed alone), until the batch-level tuner has chosen a shape
        for the run's precision class.
    tune_min: batch size at which the batch-level shape tuner runs (once);
        0 disables it.
    prepare_workers: host threads that draw the bunches of arrived requests
        while the device works on a tick (0: drawn at admission).
    """

    def __init__(self, cap_bytes: float = 250e9, max_active: int = 64, tick_steps: int = 48,
                 autotune: bool = True, device: str = "cuda:0", clock: Optional[Callable[[], float]] = None,
                 backend=None, tune_min: int = 16, prepare_workers: int = 2):
        if backend is None:
            from . import engine as backend
        self.backend = backend  # provides Engine, Batch, footprint_bytes
        self.cap = float(cap_bytes)
        self.max_active = int(max_active)
        self.tick_steps = int(tick_steps)
        self.autotune = autotune
        self.tune_min = int(tune_min)
        self.prepare_workers = int(prepare_workers)
        self.class_shape: Dict[tuple, int] = {}  # (precision, compensated) -> tuned sweep shape
        self.device = device
        self.clock = clock or time.perf_counter
        # counts, and host seconds spent admitting (bunch, arena, load),
        # building batches, in ticks (device work and the wait for it) and
        # retiring
        self.stats = {"ticks": 0, "rebuilds": 0, "peak_active": 0, "peak_bytes": 0,
                      "t_admit_s": 0.0, "t_rebuild_s": 0.0, "t_tick_s": 0.0, "t_retire_s": 0.0}

    def _admit(self, req: Request, now: float, ready=None):
        xyz, u, q = ready.result() if ready is not None else req.bunch()
        eng = self.backend.Engine(req.desc, max_particles=len(xyz), device=self.device)
        eng.load_bunch(xyz, u, q)
        shape = self.class_shape.get(self._class(req))
        if shape is not None:
            eng.set_sweep_shape(shape)
        elif self.autotune:
            eng.autotune_sweep(2)
        return _Active(req, eng, now, eng.footprint)

    @staticmethod
    def _class(req: Request) -> tuple:
        return (req.desc.get("field_precision"), req.desc.get("compensated"))

    def _retire(self, a: _Active, now: float) -> Result:
        e = a.eng
        res = Result(rid=a.req.rid, arrival=a.req.arrival, admitted=a.admitted, finished=now,
                     steps=a.req.steps, nodes=int(np.prod(e.shape)), particles=int(e.np),
                     power=e.power_history(a.req.steps), bunching=e.bunching(),
                     fields={f: e.read_field(f) for f in a.req.keep_fields})
        e.close()
        return res

    def run(self, requests: Sequence[Request], realtime: bool = True) -> List[Result]:
        """Serve `requests` (in arrival order).  With realtime, a request is
        admissible only once the wall clock since the start has passed its
        arrival time; otherwise all are available at once."""
        Batch, footprint_bytes = self.backend.Batch, self.backend.footprint_bytes
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        qi = 0
        active: List[_Active] = []
        results: List[Result] = []
        batch = None
        used = 0
        # bunches of arrived requests drawn on host threads while a tick runs
        # (the device wait releases the interpreter); at most max_active ahead
        pool = ThreadPoolExecutor(self.prepare_workers) if self.prepare_workers > 0 else None
        ready: Dict[int, object] = {}

        def prepare(now: float):
            if pool is None:
                return
            for r in pending[qi:qi + self.max_active]:
                if realtime and r.arrival > now:
                    break
                if r.rid not in ready:
                    ready[r.rid] = pool.submit(r.bunch)

        t0 = self.clock()
        while qi < len(pending) or active:
            now = self.clock() - t0
            # admit arrived requests in order while slots and memory allow
            changed = False
            while qi < len(pending) and len(active) < self.max_active:
                r = pending[qi]
                if realtime and r.arrival > now:
                    break
                fp = footprint_bytes(r.desc, r.n_particles)
                if fp > self.cap:
                    raise ValueError(f"request {r.rid} needs {fp} bytes, above the cap {self.cap:.0f}")
                if used + fp > self.cap:
                    break  # wait for a run to finish
                if batch is not None:
                    batch.close()
                    batch = None
                ta = self.clock()
                active.append(self._admit(r, now, ready.pop(r.rid, None)))
                self.stats["t_admit_s"] += self.clock() - ta
                used += fp
                qi += 1
                changed = True
            if not active:
                if qi < len(pending):
                    wait = pending[qi].arrival - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.02))
                continue
            self.stats["peak_active"] = max(self.stats["peak_active"], len(active))
            self.stats["peak_bytes"] = max(self.stats["peak_bytes"], used)
            if batch is None or changed:
                tb = self.clock()
                batch = Batch([a.eng for a in active])
                self.stats["rebuilds"] += 1
                if self.tune_min > 0 and not self.class_shape and len(active) >= self.tune_min:
                    shapes = batch.autotune_sweep(2)
                    for a, sh in zip(active, shapes):
                        self.class_shape[self._class(a.req)] = int(sh)
                    self.stats["tuned_shapes"] = dict((str(k), v) for k, v in self.class_shape.items())
                self.stats["t_rebuild_s"] += self.clock() - tb
            n = [min(self.tick_steps, a.req.steps - a.done) for a in active]
            tt = self.clock()
            batch.run(n)
            prepare(self.clock() - t0)
            batch.sync()
            self.stats["t_tick_s"] += self.clock() - tt
            self.stats["ticks"] += 1
            for a, k in zip(active, n):
                a.done += k
            now = self.clock() - t0
            fin = [a for a in active if a.done >= a.req.steps]
            if fin:
                tr = self.clock()
                batch.close()
                batch = None
                for a in fin:
                    results.append(self._retire(a, now))
                    used -= a.footprint
                self.stats["t_retire_s"] += self.clock() - tr
                active = [a for a in active if a.done < a.req.steps]
        if batch is not None:
            batch.close()
        if pool is not None:
            pool.shutdown(wait=True)
        return results


def request_from_workload(rid: int, arrival: float, w, steps: Optional[int] = None,
                          keep_fields: Sequence[str] = ()) -> Request:
    """A request running workload `w` (workloads.Workload) for `steps` (its own by default)."""
    from . import workloads as W
    return Request(rid=rid, arrival=float(arrival), desc=w.descriptor(), bunch=lambda w=w: W.make_bunch(w),
                   n_particles=int(w.n_particles), steps=int(w.steps if steps is None else steps),
                   keep_fields=tuple(keep_fields))


def summarize(results: Sequence[Result], wall: float, warmup: int = 0) -> dict:
    rs = sorted(results, key=lambda r: r.rid)[warmup:]
    lat = np.array([r.latency for r in rs]) if rs else np.zeros(1)
    cells = float(sum(r.nodes * r.steps for r in results))
    psteps = float(sum(r.particles * r.steps for r in results))
    return {"requests": len(results), "measured": len(rs), "wall_s": wall,
            "cell_updates_per_s": cells / wall, "particle_steps_per_s": psteps / wall,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(np.mean(lat))}
