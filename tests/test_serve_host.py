"""Host logic of the continuous-batching server, on the CPU with a fake
device backend: admission by footprint and slots, every request run for
exactly its steps, runs joining and leaving between ticks, and results that
do not depend on what else was in the batch."""
import numpy as np
import pytest

from paper_2009_13645_amd.serve import Request, Server, summarize


class FakeEngine:
    live = 0
    peak = 0

    def __init__(self, desc, max_particles, device=None):
        self.desc = desc
        self.shape = (desc["nz"], desc["ny"], desc["nx"])
        self.footprint = desc["fp"]
        self.steps = 0
        self.np = max_particles
        self.batched = False
        FakeEngine.live += 1
        FakeEngine.peak = max(FakeEngine.peak, FakeEngine.live)

    def load_bunch(self, xyz, u, q):
        self.seed = float(np.sum(xyz))

    def autotune_sweep(self, iters):
        self.shape_id = 0
        return 0

    def set_sweep_shape(self, shape):
        self.shape_id = shape

    def power_history(self, n):
        # a deterministic function of the run's own inputs and step count
        return self.seed + np.arange(min(n, self.steps), dtype=float)

    def bunching(self):
        return self.seed * 1e-3 + self.steps

    def read_field(self, name):
        return np.full(self.shape, self.seed + self.steps)

    def close(self):
        assert not self.batched
        FakeEngine.live -= 1


class FakeBatch:
    open_batches = 0

    def __init__(self, engines):
        self.engines = engines
        for e in engines:
            assert not e.batched
            e.batched = True
        FakeBatch.open_batches += 1
        assert FakeBatch.open_batches == 1

    def autotune_sweep(self, iters):
        for e in self.engines:
            e.shape_id = 7
        return [7] * len(self.engines)

    def run(self, steps):
        for e, n in zip(self.engines, steps):
            assert n >= 0
            e.steps += n

    def sync(self):
        pass

    def close(self):
        for e in self.engines:
            e.batched = False
        FakeBatch.open_batches -= 1


class Backend:
    Engine = FakeEngine
    Batch = FakeBatch

    @staticmethod
    def footprint_bytes(desc, n):
        return desc["fp"]


def req(rid, arrival, steps, fp, nxyz=(8, 8, 8)):
    d = {"nx": nxyz[0], "ny": nxyz[1], "nz": nxyz[2], "fp": fp}
    xyz = np.full((5, 3), float(rid))
    return Request(rid=rid, arrival=arrival, desc=d, bunch=lambda: (xyz, xyz, -1.0), n_particles=5,
                   steps=steps, keep_fields=("Ex",))


class Clock:
    """Simulated time: each call advances by dt."""

    def __init__(self, dt=0.01):
        self.t = 0.0
        self.dt = dt

    def __call__(self):
        self.t += self.dt
        return self.t


def run(reqs, **kw):
    FakeEngine.live = FakeEngine.peak = 0
    srv = Server(backend=Backend, autotune=True, clock=Clock(), **kw)
    res = srv.run(reqs)
    assert FakeEngine.live == 0 and FakeBatch.open_batches == 0
    return srv, res


def test_every_request_runs_exactly_its_steps_and_is_released():
    reqs = [req(i, 0.05 * i, steps=10 + 7 * i, fp=100) for i in range(12)]
    srv, res = run(reqs, tick_steps=4, max_active=5)
    assert sorted(r.rid for r in res) == list(range(12))
    for r in res:
        assert r.steps == 10 + 7 * r.rid
        assert len(r.power) == r.steps
        assert r.finished >= r.admitted >= r.arrival
    assert FakeEngine.peak <= 5
    assert srv.stats["peak_active"] <= 5


def test_admission_respects_the_footprint_cap():
    reqs = [req(i, 0.0, steps=20, fp=300) for i in range(6)]
    srv, res = run(reqs, tick_steps=5, cap_bytes=1000)
    assert srv.stats["peak_bytes"] <= 1000
    assert FakeEngine.peak == 3
    assert len(res) == 6


def test_request_larger_than_the_cap_is_refused():
    with pytest.raises(ValueError):
        run([req(0, 0.0, steps=5, fp=2000)], cap_bytes=1000)


def test_result_alone_equals_result_in_the_mix():
    mix = [req(i, 0.02 * i, steps=5 + 3 * i, fp=10) for i in range(9)]
    _, res_mix = run(mix, tick_steps=4, max_active=4)
    for target in (0, 4, 8):
        _, alone = run([req(target, 0.0, steps=5 + 3 * target, fp=10)], tick_steps=4)
        a = alone[0]
        m = next(r for r in res_mix if r.rid == target)
        assert np.array_equal(a.power, m.power)
        assert a.bunching == m.bunching
        assert np.array_equal(a.fields["Ex"], m.fields["Ex"])


def test_summary_counts_work_and_latency_percentiles():
    reqs = [req(i, 0.01 * i, steps=8, fp=10, nxyz=(4, 5, 6)) for i in range(10)]
    _, res = run(reqs, tick_steps=8)
    s = summarize(res, wall=2.0, warmup=2)
    assert s["requests"] == 10 and s["measured"] == 8
    assert s["cell_updates_per_s"] == pytest.approx(10 * 120 * 8 / 2.0)
    assert s["particle_steps_per_s"] == pytest.approx(10 * 5 * 8 / 2.0)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_batch_tuner_runs_once_and_later_admissions_take_its_shape():
    shapes = []
    orig = FakeEngine.close

    def close(self):
        shapes.append(self.shape_id)
        orig(self)
    FakeEngine.close = close
    try:
        reqs = [req(i, 0.02 * i, steps=30, fp=10, nxyz=(8, 8, 8)) for i in range(10)]
        srv, res = run(reqs, tick_steps=5, max_active=4, tune_min=3)
    finally:
        FakeEngine.close = orig
    assert len(res) == 10
    assert srv.stats.get("tuned_shapes")
    # every run admitted after the tuning took the tuned shape without its own autotune
    assert shapes.count(7) >= 7
