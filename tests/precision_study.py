"""Precision study on the FEL amplifier (128x128x1024 nodes, 2^21 e-).

Three GPU runs of the same seeded inputs:
- FP32 fields with two-sum compensated FP32 deposition;
- FP64 everywhere;
- plain FP32 (for contrast).

Each is compared with the FP64 CPU oracle every `every` steps up to
`steps`:
- the relative L2 error of |E|^2 on sampled node planes;
- the relative error of the bunching factor;
- the relative error of the lab-frame power through the diagnostic plane;
- the relative error of the grid total of |E|^2.

The sampled planes are every 128th z plane (k = 64, 192, ..., 960), the
full 128 x 128 nodes of each.

Test-support script (it runs the oracle).  pytest does not collect it.
Modes:
    python tests/precision_study.py oracle OUT.npz [--steps 4000 --every 500]
    python tests/precision_study.py gpu OUT.npz [--steps 4000 --every 500]
    python tests/precision_study.py compare ORACLE.npz GPU.npz OUT.md
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

PLANES = list(range(64, 1024, 128))
VARIANTS = [("fp32_compensated", 32, 1), ("fp64", 64, 0), ("fp32_plain", 32, 0)]


def e2(get):
    """|E|^2 per node from a field reader get(name) -> [nz][ny][nx]."""
    ex, ey, ez = get("Ex"), get("Ey"), get("Ez")
    return ex * ex + ey * ey + ez * ez


def sample(get, power, bunching):
    f = e2(get)
    return {"e2_planes": f[PLANES].copy(), "e2_total": float(np.sum(f)),
            "power": float(power()), "bunching": float(bunching())}


def checkpoints(steps, every):
    return list(range(0, steps + 1, every))


def run_oracle(out, steps, every):
    from oracle.oracle import Oracle, threads
    from paper_2009_13645_amd import workloads as W
    w = W.config2(field_precision=64)
    d = w.descriptor()
    xyz, u, q = W.make_bunch(w)
    o = Oracle(d)
    o.load_bunch(xyz, u, q)
    rec = {}
    done = 0
    t0 = time.time()
    for c in checkpoints(steps, every):
        if c > done:
            o.step(c - done)
            done = c
        s = sample(o.field, o.radiated_power, o.bunching)
        for k, v in s.items():
            rec.setdefault(k, []).append(v)
        print(f"precision: oracle step {c} b={s['bunching']:.6e} P={s['power']:.6e} "
              f"({time.time() - t0:.0f} s, {threads()} threads)", flush=True)
        np.savez(out, steps=np.array(checkpoints(steps, every)[:len(rec['power'])]),
                 **{k: np.array(v) for k, v in rec.items()})
    o.close()


def run_gpu(out, steps, every):
    import torch
    from paper_2009_13645_amd import workloads as W
    from paper_2009_13645_amd.engine import Engine
    res = {}
    for name, prec, comp in VARIANTS:
        w = W.config2(field_precision=prec, compensated=comp)
        d = w.descriptor()
        xyz, u, q = W.make_bunch(w)
        e = Engine(d, max_particles=len(xyz))
        e.load_bunch(xyz, u, q)
        done = 0
        t0 = time.time()
        for c in checkpoints(steps, every):
            if c > done:
                e.step(c - done)
                done = c
            s = sample(lambda n: e.read_field(n), e.radiated_power, e.bunching)
            for k, v in s.items():
                res.setdefault(f"{name}/{k}", []).append(v)
            print(f"precision: {name} step {c} b={s['bunching']:.6e} P={s['power']:.6e} "
                  f"({time.time() - t0:.1f} s)", flush=True)
        e.close()
        del e
        torch.cuda.empty_cache()
    np.savez(out, steps=np.array(checkpoints(steps, every)), **{k: np.array(v) for k, v in res.items()})


def rel(a, b):
    return float(abs(a - b) / abs(b)) if b != 0 else float(abs(a))


def compare(f_oracle, f_gpu, out_md):
    o = np.load(f_oracle)
    g = np.load(f_gpu)
    n = min(len(o["steps"]), len(g["steps"]))
    lines = ["# Precision study: FEL amplifier (128x128x1024 nodes, 2^21 e-) against the FP64 oracle", "",
             "Commands (from the repository root):", "",
             "    python3 tests/precision_study.py oracle <oracle.npz> --steps 4000 --every 500   (host cores)",
             "    python3 tests/precision_study.py gpu <gpu.npz> --steps 4000 --every 500        (MI355X)",
             "    python3 tests/precision_study.py compare <oracle.npz> <gpu.npz> profiles/precision_study.md",
             "",
             "|E|^2 error: relative L2 over the full 128x128 nodes of the planes k = "
             + ", ".join(map(str, PLANES)) + ". b: bunching factor; P: lab-frame power through the "
             "diagnostic plane; sum: grid total of |E|^2. All errors are relative to the oracle.", ""]
    for name, _, _ in VARIANTS:
        lines += [f"## {name}", "", "| step | rel-L2 \\|E\\|^2 | rel err b | rel err P | rel err sum \\|E\\|^2 |",
                  "|---:|---:|---:|---:|---:|"]
        for i in range(n):
            eo = o["e2_planes"][i]
            eg = g[f"{name}/e2_planes"][i]
            nrm = np.linalg.norm(eo)
            l2 = float(np.linalg.norm(eg - eo) / nrm) if nrm > 0 else float(np.linalg.norm(eg))
            lines.append(f"| {int(o['steps'][i])} | {l2:.3e} | {rel(g[f'{name}/bunching'][i], o['bunching'][i]):.3e} | "
                         f"{rel(g[f'{name}/power'][i], o['power'][i]):.3e} | "
                         f"{rel(g[f'{name}/e2_total'][i], o['e2_total'][i]):.3e} |")
        lines.append("")
    lines += ["## Oracle values", "", "| step | b | P (W) | sum \\|E\\|^2 |", "|---:|---:|---:|---:|"]
    for i in range(n):
        lines.append(f"| {int(o['steps'][i])} | {o['bunching'][i]:.6e} | {o['power'][i]:.6e} | {o['e2_total'][i]:.6e} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["oracle", "gpu", "compare"])
    ap.add_argument("files", nargs="+")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--every", type=int, default=500)
    a = ap.parse_args()
    if a.mode == "oracle":
        run_oracle(a.files[0], a.steps, a.every)
    elif a.mode == "gpu":
        run_gpu(a.files[0], a.steps, a.every)
    else:
        compare(a.files[0], a.files[1], a.files[2])


if __name__ == "__main__":
    main()
