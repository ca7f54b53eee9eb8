"""Batched runs (grouped launches, one graph per batched step) on the GPU.

A batch must give each member the result it gets when stepped alone: the
step arithmetic of a run does not depend on the other members, and only
the order of floating-point atomic additions in the deposit may differ (as
between two solo runs).  Members of different grids, particle counts,
precisions and sweep shapes are mixed, with different step counts, over
two batch calls.  Batched FP64 members are also held to the oracle.
"""
import numpy as np
import pytest
import torch  # noqa: F401

from oracle.oracle import Oracle
from paper_2009_13645_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["Ax", "Ay", "Az", "F", "Jx", "Jy", "Jz", "Q", "Ex", "Ey", "Ez", "Bx", "By", "Bz"]


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def members():
    """Six uneven runs of the batched-scan recipe, particles scaled down,
    precision and compensation set so every kernel variant appears."""
    runs = W.config4_runs(6, base_seed=4000, scale=0.03)
    kinds = [(64, 0), (32, 0), (32, 1), (64, 0), (32, 0), (64, 0)]
    for w, (p, c) in zip(runs, kinds):
        w.field_precision, w.compensated = p, c
    return runs


def make(w, tune=False):
    from paper_2009_13645_amd.engine import Engine
    d = w.descriptor()
    xyz, u, q = W.make_bunch(w)
    e = Engine(d, max_particles=len(xyz))
    e.load_bunch(xyz, u, q)
    if tune:
        e.autotune_sweep(3)
    return e, d, (xyz, u, q)


def tol(w):
    return 1e-11 if w.field_precision == 64 else 1e-5


def test_batch_equals_solo_runs_over_two_calls():
    from paper_2009_13645_amd.engine import Batch
    runs = members()
    calls = [[30, 0, 20, 45, 5, 12], [10, 25, 20, 0, 40, 12]]
    total = [a + b for a, b in zip(*calls)]
    for w in runs:
        print(f"[batch] member {w.name} np={w.n_particles} prec={w.field_precision} comp={w.compensated}",
              flush=True)
    # FP64 members run autotuned shapes in the batch and the scalar sweep
    # solo (FP64 rounding makes the two agree far below the bar); FP32
    # members use the same default shape on both sides, so only the order
    # of the deposit's atomic additions differs
    batched = [make(w, tune=(w.field_precision == 64)) for w in runs]
    b = Batch([e for e, _, _ in batched])
    for c in calls:
        b.run(c)
    b.sync()
    for (e, d, _), w, n in zip(batched, runs, total):
        s, _, _ = make(w)
        if w.field_precision == 64:
            s.set_sweep_shape(0)
        s.step(n)
        worst = {f: rel_l2(e.read_field(f), s.read_field(f)) for f in FIELDS}
        xb, ub, cb, pb = e.read_particles()
        xs, us, cs, ps = s.read_particles()
        worst["u"] = rel_l2(ub, us)
        print(f"[batch] {w.name} steps={n}:", {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
        assert e.constants()["steps"] == n
        for k, v in worst.items():
            assert v < tol(w), (w.name, k, v)
        if w.field_precision == 64:
            assert int(np.sum(cb != cs)) == 0
            assert int(np.sum(pb != ps)) == 0
        s.close()
    b.close()
    # members are ordinary runs again
    batched[0][0].step(1)


@pytest.mark.parametrize("prec", [64, 32])
def test_single_precision_batch_equals_solo_runs(prec):
    """A batch whose members all have one precision (one of the step graph's
    two precision branches is empty), over the steps after which no member
    sorts (the sort-free graph) and a sort step."""
    from paper_2009_13645_amd.engine import Batch
    runs = W.config4_runs(2, base_seed=4100, scale=0.03)
    for w in runs:
        w.field_precision, w.compensated = prec, 0
    n = 20  # the recipe sorts after every 16th push
    batched = [make(w) for w in runs]
    b = Batch([e for e, _, _ in batched])
    b.run([n, n])
    b.sync()
    for (e, d, _), w in zip(batched, runs):
        s, _, _ = make(w)
        s.step(n)
        worst = {f: rel_l2(e.read_field(f), s.read_field(f)) for f in FIELDS}
        print(f"[batch] single precision FP{prec} {w.name}:", {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
        for k, v in worst.items():
            assert v < tol(w), (w.name, k, v)
        xb, ub, cb, pb = e.read_particles()
        xs, us, cs, ps = s.read_particles()
        assert rel_l2(ub, us) < tol(w)
        if prec == 64:
            assert int(np.sum(cb != cs)) == 0 and int(np.sum(pb != ps)) == 0
        s.close()
    b.close()


def test_batched_fp64_members_match_the_oracle():
    from paper_2009_13645_amd.engine import Batch
    runs = [w for w in members() if w.field_precision == 64][:2]
    for w in runs:
        w.n_particles = min(w.n_particles, 3000)
    engs = [make(w) for w in runs]
    b = Batch([e for e, _, _ in engs])
    steps = [40, 25]
    b.run(steps)
    b.sync()
    for (e, d, (xyz, u, q)), w, n in zip(engs, runs, steps):
        o = Oracle(d)
        o.load_bunch(xyz, u, q)
        o.step(n)
        worst = {f: rel_l2(e.read_field(f), o.field(f)) for f in FIELDS}
        xg, ug, cg, pg = e.read_particles()
        xo, uo, co, po = o.particles()
        worst["u"] = rel_l2(ug, uo)
        print(f"[batch-oracle] {w.name} steps={n}:", {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
        for k, v in worst.items():
            assert v < 1e-10, (w.name, k, v)
        assert int(np.sum(cg != co)) == 0
        assert int(np.sum(pg != po)) == 0
        o.close()
    b.close()


def test_autotune_is_cached_and_valid():
    from paper_2009_13645_amd.engine import Engine
    w = members()[1]
    e1, _, _ = make(w)
    s1 = e1.autotune_sweep(3)
    e2, _, _ = make(w)
    s2 = e2.autotune_sweep(3)
    assert 0 <= s1 < Engine.sweep_shape_count()
    assert s1 == s2


def test_batch_autotune_keeps_state_and_results():
    """The batch-level shape tuner leaves every member's state untouched and
    the tuned batch still gives each member its solo result."""
    from paper_2009_13645_amd.engine import Batch, Engine
    runs = members()
    batched = [make(w) for w in runs]
    b = Batch([e for e, _, _ in batched])
    b.run(10)
    b.sync()
    names = ["Ax", "Ay", "Az", "F", "Jx", "Jy", "Jz", "Q"]
    before = [{f: e.read_field(f) for f in names} for e, _, _ in batched]
    parts = [e.read_particles() for e, _, _ in batched]
    shapes = b.autotune_sweep(2)
    print(f"[batch-tune] shapes {shapes}", flush=True)
    assert all(0 <= s < Engine.sweep_shape_count() for s in shapes)
    # one shape per (precision, compensation) class
    by_cls = {}
    for w, s in zip(runs, shapes):
        by_cls.setdefault((w.field_precision, w.compensated), set()).add(s)
    assert all(len(v) == 1 for v in by_cls.values()), by_cls
    for (e, _, _), snap, pa in zip(batched, before, parts):
        for f in names:
            assert np.array_equal(e.read_field(f), snap[f]), f
        for x, y in zip(e.read_particles(), pa):
            assert np.array_equal(x, y)
    b.run(15)
    b.sync()
    for (e, d, _), w, sh in zip(batched, runs, shapes):
        s, _, _ = make(w)
        s.set_sweep_shape(sh)
        s.step(25)
        worst = {f: rel_l2(e.read_field(f), s.read_field(f)) for f in FIELDS}
        print(f"[batch-tune] {w.name}:", {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
        for k, v in worst.items():
            assert v < tol(w), (w.name, k, v)
        s.close()
    b.close()
