"""Oracle parity of the batched scan.

All runs of the batched-scan recipe (64 undulator runs; grids, gamma, K
and precision as drawn) are stepped as one GPU batch, then each member is
compared with the FP64 CPU oracle run alone on the same inputs:
- every field, relative L2;
- momenta, relative L2;
- cells and sort order, mismatch counts.

Particle counts are scaled by `--scale` (default 0.05) and the step count
is 200.  The oracle's per-particle loop sets the CPU time, so the scale
bounds it.  The grids are the recipe's own.

Bars: 1e-10 (FP64 runs) and 2e-4 (FP32 runs) relative L2.  Cells and sort
order must match exactly for FP64 runs.

With --served N it checks the served stream instead: N requests of the
served-stream recipe (reduced particle counts, 120..200 steps) go through
the continuous-batching server, at most 8 at once, so requests are admitted
and retired while others run; each result (fields kept at the end, the
per-step power history, the bunching factor) is compared with the oracle
run alone.  Bars: the field bars above; power history 1e-9 (FP64) and 1e-3
(FP32) of the run's largest power; bunching factor 1e-9 (FP64) and 2e-3
(FP32) relative.

Test-support script: it runs the oracle, and pytest does not collect it.
    python tests/batch_parity.py OUT.md [--runs 64 --steps 200 --scale 0.05]
    python tests/batch_parity.py OUT.md --served 32 [--scale 0.05]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

FIELDS = ["Ax", "Ay", "Az", "F", "Jx", "Jy", "Jz", "Q", "Ex", "Ey", "Ez", "Bx", "By", "Bz"]


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--runs", type=int, default=64)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--scale", type=float, default=0.05)
    ap.add_argument("--served", type=int, default=0, help="check N served-stream requests instead")
    a = ap.parse_args()
    if a.served > 0:
        return served(a)

    import torch
    from oracle.oracle import Oracle, threads
    from paper_2009_13645_amd import workloads as W
    from paper_2009_13645_amd.engine import Batch, Engine

    runs = W.config4_runs(a.runs, scale=a.scale)
    engs, inputs = [], []
    for w in runs:
        d = w.descriptor()
        xyz, u, q = W.make_bunch(w)
        e = Engine(d, max_particles=len(xyz))
        e.load_bunch(xyz, u, q)
        shape = e.autotune_sweep(2)
        engs.append(e)
        inputs.append((d, xyz, u, q, shape))
    b = Batch(engs)
    t0 = time.perf_counter()
    b.run(a.steps)
    b.sync()
    t_gpu = time.perf_counter() - t0
    print(f"batch-parity: {len(runs)} runs x {a.steps} steps on the GPU in {t_gpu:.2f} s", flush=True)

    rows = []
    t_ora = 0.0
    for i, (w, e, (d, xyz, u, q, shape)) in enumerate(zip(runs, engs, inputs)):
        o = Oracle(d)
        o.load_bunch(xyz, u, q)
        t0 = time.perf_counter()
        o.step(a.steps)
        t_ora += time.perf_counter() - t0
        worst_f, worst_name = 0.0, ""
        for f in FIELDS:
            r = rel_l2(e.read_field(f), o.field(f))
            if r > worst_f:
                worst_f, worst_name = r, f
        xg, ug, cg, pg = e.read_particles()
        xo, uo, co, po = o.particles()
        ru = rel_l2(ug, uo)
        mc = int(np.sum(cg != co))
        mp = int(np.sum(pg != po))
        bar = 1e-10 if w.field_precision == 64 else 2e-4
        ok = worst_f < bar and ru < bar and (w.field_precision == 32 or (mc == 0 and mp == 0))
        rows.append((w.name, w.field_precision, len(xyz), shape, worst_name, worst_f, ru, mc, mp, ok))
        o.close()
        print(f"batch-parity: {i:2d} {w.name} fp{w.field_precision} np={len(xyz)} shape={shape} "
              f"worst field {worst_name} {worst_f:.2e} u {ru:.2e} cells {mc} perm {mp} {'ok' if ok else 'FAIL'}",
              flush=True)
    b.close()

    n_ok = sum(r[-1] for r in rows)
    with open(a.out, "w") as f:
        f.write("# Oracle parity of the batched scan\n\n")
        f.write(f"Command (from the repository root): `python3 tests/batch_parity.py <out.md> --runs {a.runs} "
                f"--steps {a.steps} --scale {a.scale}`\n\n")
        f.write(f"{len(runs)} runs of the batched-scan recipe were stepped {a.steps} steps as one GPU batch, "
                f"with grouped launches and tiles from the autotuner ({t_gpu:.2f} s).\n"
                f"Each run was compared with the FP64 oracle run alone on the host "
                f"({threads()} threads, {t_ora:.0f} s).\n"
                f"Particle counts were scaled by {a.scale}.\n"
                f"Bars: 1e-10 (FP64 runs) and 2e-4 (FP32 runs) relative L2; for FP64 runs, "
                f"cells and sort order must match exactly.\n\n")
        f.write(f"**{n_ok} of {len(rows)} runs within the bars.**\n\n")
        f.write("| run | fields | particles | sweep shape | worst field | rel L2 | rel L2 u | cell mismatches "
                "| order mismatches | ok |\n|---|---:|---:|---:|---|---:|---:|---:|---:|---|\n")
        for r in rows:
            f.write(f"| {r[0]} | FP{r[1]} | {r[2]} | {r[3]} | {r[4]} | {r[5]:.2e} | {r[6]:.2e} | {r[7]} | {r[8]} "
                    f"| {'yes' if r[9] else 'NO'} |\n")
    print(f"batch-parity: {n_ok}/{len(rows)} within the bars", flush=True)
    return 0 if n_ok == len(rows) else 1


KEEP = ("Ax", "Az", "F", "Jz", "Ex", "Ey", "Ez", "By")


def served(a):
    from oracle.oracle import Oracle, threads
    from paper_2009_13645_amd import workloads as W
    from paper_2009_13645_amd.serve import Server, request_from_workload

    reqs = []
    for i, (t, w) in enumerate(W.config5_requests(n_req=a.served, scale=a.scale)):
        steps = 120 + (i * 24) % 88  # 120..200: members leave on different ticks
        reqs.append((request_from_workload(i, 0.0, w, steps=steps, keep_fields=KEEP), w))
    srv = Server(cap_bytes=250e9, max_active=8, tick_steps=48)
    t0 = time.perf_counter()
    try:
        res = {r.rid: r for r in srv.run([r for r, _ in reqs], realtime=False)}
    except Exception:
        print(f"served-parity: the server stopped after {srv.stats}", flush=True)
        raise
    t_gpu = time.perf_counter() - t0
    print(f"served-parity: {len(reqs)} requests through the server in {t_gpu:.2f} s, "
          f"{srv.stats['ticks']} ticks, {srv.stats['rebuilds']} batch rebuilds", flush=True)

    rows = []
    t_ora = 0.0
    for req, w in reqs:
        d = w.descriptor()
        xyz, u, q = W.make_bunch(w)
        o = Oracle(d)
        o.load_bunch(xyz, u, q)
        pw = []
        t0 = time.perf_counter()
        for _ in range(req.steps):
            o.step(1)
            pw.append(o.radiated_power())
        t_ora += time.perf_counter() - t0
        r = res.pop(req.rid)
        worst_f, worst_name = 0.0, ""
        for f in KEEP:
            e = rel_l2(r.fields[f], o.field(f))
            if e > worst_f:
                worst_f, worst_name = e, f
        pw = np.array(pw)
        perr = float(np.max(np.abs(r.power - pw)) / max(np.max(np.abs(pw)), 1e-300))
        bo = o.bunching()
        berr = abs(r.bunching - bo) / max(abs(bo), 1e-300)
        fp64 = w.field_precision == 64
        ok = (worst_f < (1e-10 if fp64 else 2e-4) and len(r.power) == req.steps
              and perr < (1e-9 if fp64 else 1e-3) and berr < (1e-9 if fp64 else 2e-3))
        rows.append((w.name, w.field_precision, len(xyz), req.steps, worst_name, worst_f, perr, berr, ok))
        o.close()
        print(f"served-parity: {req.rid:2d} {w.name} fp{w.field_precision} np={len(xyz)} steps={req.steps} "
              f"worst field {worst_name} {worst_f:.2e} power {perr:.2e} bunching {berr:.2e} "
              f"{'ok' if ok else 'FAIL'}", flush=True)

    n_ok = sum(r[-1] for r in rows)
    with open(a.out, "w") as f:
        f.write("# Oracle parity of the served stream\n\n")
        f.write(f"Command (from the repository root): `python3 tests/batch_parity.py <out.md> --served {a.served} "
                f"--scale {a.scale}`\n\n")
        f.write(f"{len(reqs)} requests of the served-stream recipe (grids, gamma, K and precision as drawn; "
                f"120..200 steps) went through the continuous-batching server, at most 8 at once, in "
                f"{srv.stats['ticks']} ticks of 48 steps with {srv.stats['rebuilds']} batch rebuilds "
                f"({t_gpu:.2f} s), so requests were admitted and retired while others ran.\n"
                f"Each result was compared with the FP64 oracle run alone on the host "
                f"({threads()} threads, {t_ora:.0f} s).\n"
                f"Particle counts were scaled by {a.scale}.\n"
                f"Bars: fields 1e-10 (FP64 runs) and 2e-4 (FP32 runs) relative L2 over {', '.join(KEEP)}; "
                f"power history 1e-9 / 1e-3 of the largest power; bunching factor 1e-9 / 2e-3 relative.\n\n")
        f.write(f"**{n_ok} of {len(rows)} requests within the bars.**\n\n")
        f.write("| request | fields | particles | steps | worst field | rel L2 | power | bunching | ok |\n"
                "|---|---:|---:|---:|---|---:|---:|---:|---|\n")
        for r in rows:
            f.write(f"| {r[0]} | FP{r[1]} | {r[2]} | {r[3]} | {r[4]} | {r[5]:.2e} | {r[6]:.2e} | {r[7]:.2e} "
                    f"| {'yes' if r[8] else 'NO'} |\n")
    print(f"served-parity: {n_ok}/{len(rows)} within the bars", flush=True)
    return 0 if n_ok == len(rows) else 1


if __name__ == "__main__":
    sys.exit(main())
