"""HBM traffic of the field sweep from hardware counters (rocprofv3 --pmc).

Two steps, each under its own profiler run:

  rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_f> -- python3 <repo>/paper_2009_13645_amd/counters.py run
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir_w> -- python3 <repo>/paper_2009_13645_amd/counters.py run
  python3 <repo>/paper_2009_13645_amd/counters.py summarize <dir_f> <dir_w>

and for the particle kernel (push + gather + deposit), four runs, one per
counter set (FETCH_SIZE; WRITE_SIZE TCC_ATOMIC_sum; eight SQ counters of
instruction mix, LDS and waits; the FP64 instruction mix and VALU activity),
then

  python3 <repo>/paper_2009_13645_amd/counters.py push <dir_1> <dir_2> <dir_3> <dir_4>

and for the kernel time of a benchmark run, one kernel trace, then

  python3 <repo>/paper_2009_13645_amd/counters.py kstats <dir> <n_steps>

which writes profiles/bench_fel_amplifier_fp32_kernel_stats.md: kernel
time over the run's last n_steps FP32 steps (the bench's timed steps and
its per-stage profile) beside the profiler's whole-process statistics;
and for the batched scan, one kernel trace of
`bench.py --workload batched-scan`, then

  python3 <repo>/paper_2009_13645_amd/counters.py bstats <dir>

which writes profiles/bench_batched_scan_kernel_stats.md: kernel time of
the grouped launches from the batch's first push on (the timed scan).

and for the manual's Example 1, from bench.py's output lines and power
histories,

  python3 <repo>/paper_2009_13645_amd/counters.py ex1 <example1.json> <hist.npz> [<convergence.json> <conv_hist.npz>]

which writes profiles/example1_gain_curve.md (and example1_convergence.md).

`run` executes the benchmark workload (FEL amplifier, FP32) until the
whole bunch is inside the undulator and 20 steps more, as the benchmark
times it, then 10 launches of the sweep alone, then a plain device-to-device
copy of a known size (torch's copy kernel) used to calibrate what the
counters read per byte.  `summarize` writes profiles/sweep_traffic.json
(bytes per sweep launch, tagged with the hash of the sweep's source file)
and profiles/sweep_traffic.md.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 256 * 1024 * 1024


def run():
    sys.path.insert(0, ROOT)
    import torch
    from paper_2009_13645_amd import workloads as W
    from paper_2009_13645_amd.engine import Engine
    w = W.config2(field_precision=32, compensated=0)
    d = w.descriptor()
    d["sort_every"] = 16  # as the benchmark runs it
    xyz, u, q = W.make_bunch(w)
    e = Engine(d, max_particles=len(xyz))
    e.load_bunch(xyz, u, q)
    e.step(w.steps_bunch_inside() + 20)
    torch.cuda.synchronize()
    e.time_sweep(-1, 10)
    torch.cuda.synchronize()
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("counters: run done", flush=True)


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    # the newest file: a folder reused by several runs keeps the older ones
    with open(max(files, key=os.path.getmtime)) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows, name_part, counter):
    vals = {}
    for r in rows:
        if name_part not in r.get("Kernel_Name", "") or r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return list(vals.values())


def summarize(dir_f, dir_w):
    rf, rw = _rows(dir_f), _rows(dir_w)
    sweep_f = _per_dispatch(rf, "Sweep", "FETCH_SIZE")
    sweep_w = _per_dispatch(rw, "Sweep", "WRITE_SIZE")
    # torch's device-to-device copy_ runs as the runtime's copyBuffer kernel
    copy_f = _per_dispatch(rf, "copyBuffer", "FETCH_SIZE")
    copy_w = _per_dispatch(rw, "copyBuffer", "WRITE_SIZE")
    # counters are in KiB per dispatch; calibrate on the copy (reads and
    # writes COPY_BYTES each); skip the first (cold) launches
    cf = COPY_BYTES / (1024.0 * max(copy_f[-3:]))
    cw = COPY_BYTES / (1024.0 * max(copy_w[-3:]))
    sf = sorted(sweep_f[-10:])[len(sweep_f[-10:]) // 2] * 1024.0 * cf
    sw = sorted(sweep_w[-10:])[len(sweep_w[-10:]) // 2] * 1024.0 * cw
    src = os.path.join(ROOT, "paper_2009_13645_amd", "csrc", "k_fdtd.hip")
    rec = {
        "kernel": "SweepVec (NSFD sweep, FP32, 128x128x1024 nodes, 4 potentials)",
        "fetch_bytes_per_launch": sf, "write_bytes_per_launch": sw, "bytes_per_launch": sf + sw,
        "copy_calibration": {"fetch_factor": cf, "write_factor": cw, "copy_bytes": COPY_BYTES},
        "source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_f> -- python3 <repo>/paper_2009_13645_amd/counters.py run",
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir_w> -- python3 <repo>/paper_2009_13645_amd/counters.py run",
            "python3 <repo>/paper_2009_13645_amd/counters.py summarize <dir_f> <dir_w>",
        ],
    }
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "sweep_traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)
    with open(os.path.join(ROOT, "profiles", "sweep_traffic.md"), "w") as f:
        f.write("# HBM traffic of the NSFD sweep (FEL amplifier, FP32, 128x128x1024)\n\n")
        for c in rec["commands"]:
            f.write(f"    {c}\n")
        f.write(f"\nFETCH_SIZE per launch: {sf/1e6:.1f} MB (copy calibration x{cf:.3f})\n")
        f.write(f"WRITE_SIZE per launch: {sw/1e6:.1f} MB (copy calibration x{cw:.3f})\n")
        f.write(f"Total: {(sf+sw)/1e6:.1f} MB per launch\n")
    print(json.dumps(rec))


def _median(v):
    v = sorted(v)
    return v[len(v) // 2] if v else float("nan")


def summarize_push(dirs):
    """Per-launch counters of the benchmark's particle kernel, the median of
    its last 10 dispatches in each run; bytes calibrated on the device copy
    as for the sweep."""
    rows = [_rows(d) for d in dirs]
    name = "PushDeposit<float, false, 0"
    vals = {}
    calib = {}
    for rr in rows:
        counters = sorted({r["Counter_Name"] for r in rr})
        for c in counters:
            v = _per_dispatch(rr, name, c)
            if v:
                vals[c] = _median(v[-10:])
            cp = _per_dispatch(rr, "copyBuffer", c)
            if cp and c in ("FETCH_SIZE", "WRITE_SIZE"):
                calib[c] = COPY_BYTES / (1024.0 * max(cp[-3:]))
    fetch = vals.get("FETCH_SIZE", float("nan")) * 1024.0 * calib.get("FETCH_SIZE", float("nan"))
    write = vals.get("WRITE_SIZE", float("nan")) * 1024.0 * calib.get("WRITE_SIZE", float("nan"))
    waves = vals.get("SQ_WAVES", float("nan"))
    f64 = 64.0 * (2.0 * vals.get("SQ_INSTS_VALU_FMA_F64", 0.0) + vals.get("SQ_INSTS_VALU_MUL_F64", 0.0)
                  + vals.get("SQ_INSTS_VALU_ADD_F64", 0.0) + vals.get("SQ_INSTS_VALU_TRANS_F64", 0.0))
    srcs = [os.path.join(ROOT, "paper_2009_13645_amd", "csrc", f) for f in ("k_particles.hip", "particle_dev.hpp")]
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(f, "rb").read())
    rec = {
        "kernel": "PushDeposit<float, false, 0> with the Mur edge workgroups at the end of its launch (gather + helical undulator + Boris + deposit; FEL amplifier, "
                  "2^21 e-, FP32 fields)",
        "counters_per_launch": vals,
        "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
        "fp64_flops_per_launch": f64,
        "per_wave": {k: vals[k] / waves for k in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM",
                                                   "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64",
                                                   "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_TRANS_F64")
                     if k in vals and waves == waves and waves > 0},
        "copy_calibration": calib,
        "source_sha256": h.hexdigest(),
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_1> -- python3 <repo>/paper_2009_13645_amd/counters.py run",
            "rocprofv3 --pmc WRITE_SIZE TCC_ATOMIC_sum --output-format csv -d <dir_2> -- python3 "
            "<repo>/paper_2009_13645_amd/counters.py run",
            "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE "
            "SQ_WAIT_INST_ANY SQ_WAVE_CYCLES SQ_BUSY_CYCLES --output-format csv -d <dir_3> -- python3 "
            "<repo>/paper_2009_13645_amd/counters.py run",
            "rocprofv3 --pmc SQ_ACTIVE_INST_VALU SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_ADD_F64 "
            "SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VMEM GRBM_GUI_ACTIVE --output-format csv -d <dir_4> -- python3 "
            "<repo>/paper_2009_13645_amd/counters.py run",
            "python3 <repo>/paper_2009_13645_amd/counters.py push <dir_1> <dir_2> <dir_3> <dir_4>",
        ],
    }
    with open(os.path.join(ROOT, "profiles", "push_counters.json"), "w") as f:
        json.dump(rec, f, indent=1)
    with open(os.path.join(ROOT, "profiles", "push_counters.md"), "w") as f:
        f.write("# Hardware counters of the particle kernel (FEL amplifier, FP32 fields, 2^21 e-)\n\n")
        for c in rec["commands"]:
            f.write(f"    {c}\n")
        f.write("\nMedian of the last 10 launches, per launch:\n\n| counter | value |\n|---|---:|\n")
        for k in sorted(vals):
            f.write(f"| {k} | {vals[k]:.4g} |\n")
        f.write(f"\nFETCH {fetch / 1e6:.1f} MB, WRITE {write / 1e6:.1f} MB per launch (copy-calibrated); "
                f"FP64 flops {f64 / 1e9:.2f} G per launch.\n")
    print(json.dumps(rec))


def kstats(trace_dir, n_steps):
    """Kernel time over the last n_steps steps of the FEL amplifier in a
    kernel trace of bench.py: the window opens at the n_steps-th last
    dispatch of the FP32 sweep and holds every dispatch from there on."""
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_trace.csv under {trace_dir}")
    with open(max(files, key=os.path.getmtime)) as f:
        rows = list(csv.DictReader(f))
    sweeps = sorted((r for r in rows if "SweepVec<float" in r["Kernel_Name"]), key=lambda r: int(r["Start_Timestamp"]))
    if len(sweeps) < n_steps:
        raise SystemExit(f"only {len(sweeps)} FP32 sweeps in the trace")
    t_open = int(sweeps[-n_steps]["Start_Timestamp"])
    win = {}
    for r in rows:
        if int(r["Start_Timestamp"]) < t_open:
            continue
        v = win.setdefault(r["Kernel_Name"], [0, 0.0])
        v[0] += 1
        v[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
    tot = sum(v[1] for v in win.values())
    L = ["# Kernel time of the benchmark's timed steps (FEL amplifier, FP32 fields, 128x128x1024 nodes, "
         "2^21 e-, whole bunch inside the undulator)", "",
         "Commands (from the repository root):", "",
         "    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o bench -- python3 -u bench.py "
         "--no-cpu-baseline --latency-runs 2",
         f"    python3 paper_2009_13645_amd/counters.py kstats <dir> {n_steps}", "",
         f"Window: every dispatch from the {n_steps}-th last FP32 sweep on (the bench's {n_steps // 2} graph-replayed "
         f"timed steps, then as many steps launched one by one with events between the stages).", "",
         "| kernel | calls | average us | share |", "|---|---:|---:|---:|"]
    for name, (n, t) in sorted(win.items(), key=lambda kv: -kv[1][1])[:14]:
        L.append(f"| `{name[:90].replace('|', '/')}` | {n} | {t / n:.1f} | {100 * t / tot:.1f}% |")
    L.append("")
    L.append(f"Kernel time in the window: {tot / 1e3:.2f} ms over {n_steps} steps, {tot / n_steps:.1f} us per step.")
    st = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if st:
        with open(max(st, key=os.path.getmtime)) as f:
            srows = sorted(csv.DictReader(f), key=lambda r: -float(r["TotalDurationNs"]))
        stot = sum(float(r["TotalDurationNs"]) for r in srows)
        L += ["", "The profiler's own statistics over the whole process (all legs of the bench: the FP32 steps "
              "from the load, the FP64 run, the latency runs):", "",
              "| kernel | calls | average us | share |", "|---|---:|---:|---:|"]
        for r in srows[:14]:
            L.append(f"| `{r['Name'][:90].replace('|', '/')}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{100 * float(r['TotalDurationNs']) / stot:.1f}% |")
    with open(os.path.join(ROOT, "profiles", "bench_fel_amplifier_fp32_kernel_stats.md"), "w") as f:
        f.write("\n".join(L) + "\n")
    print("\n".join(L))


def bstats(trace_dir):
    """Kernel time of the batched scan in a kernel trace of bench.py
    --workload batched-scan: every dispatch from the first grouped push on
    (the batch-level sweep tuner before it launches sweeps and boundaries
    only; the runs stepped alone come before the batch is created)."""
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_trace.csv under {trace_dir}")
    with open(max(files, key=os.path.getmtime)) as f:
        rows = list(csv.DictReader(f))
    pushes = [int(r["Start_Timestamp"]) for r in rows
              if "k_group" in r["Kernel_Name"] and "PushDeposit" in r["Kernel_Name"]]
    if not pushes:
        raise SystemExit("no grouped push in the trace")
    t_open = min(pushes)
    win, t_end = {}, t_open
    for r in rows:
        t0 = int(r["Start_Timestamp"])
        if t0 < t_open:
            continue
        t_end = max(t_end, int(r["End_Timestamp"]))
        v = win.setdefault(r["Kernel_Name"], [0, 0.0])
        v[0] += 1
        v[1] += (int(r["End_Timestamp"]) - t0) * 1e-3
    tot = sum(v[1] for v in win.values())
    span = (t_end - t_open) * 1e-3
    n_push = sum(v[0] for k, v in win.items() if "PushDeposit" in k)
    L = ["# Kernel time of the batched scan (64 uneven runs as one batch, grouped launches in captured graphs)", "",
         "Commands (from the repository root):", "",
         "    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o bscan -- python3 -u bench.py "
         "--workload batched-scan",
         "    python3 paper_2009_13645_amd/counters.py bstats <dir>", "",
         "Window: every dispatch from the batch's first grouped push to the end of the scan. Grouped launches "
         "are split by kernel variant (precision, compensation, sweep shape), so one batched step holds one "
         "launch per variant and stage; the FP64 and FP32 members run as two graph branches, so their kernels "
         "overlap and the shares are of summed kernel time, not of wall time.", "",
         "| kernel | calls | average us | share |", "|---|---:|---:|---:|"]
    groups = {}
    for name, (n, t) in sorted(win.items(), key=lambda kv: -kv[1][1]):
        if len(L) < 40:
            L.append(f"| `{name[:110].replace('|', '/')}` | {n} | {t / n:.1f} | {100 * t / tot:.1f}% |")
        low = name.lower()
        for stage, keys in (("sweep", ("sweep",)), ("push and deposit", ("pushdeposit",)), ("Mur", ("mur",)),
                            ("vertex fields", ("vertex",)), ("power", ("power",)),
                            ("sort", ("radix", "digit", "sort")), ("box reduction", ("box",)),
                            ("bookkeeping", ("book",))):
            if any(k in low for k in keys):
                groups[stage] = groups.get(stage, 0.0) + t
                break
        else:
            groups["other"] = groups.get("other", 0.0) + t
    L += ["", f"Summed kernel time {tot / 1e3:.1f} ms; first grouped push to last kernel end {span / 1e3:.1f} ms "
              f"({n_push} grouped push launches).", "",
          "| stage | summed kernel time ms | share |", "|---|---:|---:|"]
    for k, t in sorted(groups.items(), key=lambda kv: -kv[1]):
        L.append(f"| {k} | {t / 1e3:.1f} | {100 * t / tot:.1f}% |")
    with open(os.path.join(ROOT, "profiles", "bench_batched_scan_kernel_stats.md"), "w") as f:
        f.write("\n".join(L) + "\n")
    print("\n".join(L))


def ex1(j_path, h_path, c_path=None, cz_path=None):
    """Example 1 summaries from bench.py's JSON lines and power histories:
    profiles/example1_gain_curve.md (the three 8 m runs, gain-length fits,
    yardsticks, the oracle prefix parity, the power table) and, given the
    convergence run's line and histories, profiles/example1_convergence.md."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    j = json.loads(open(j_path).read().strip().splitlines()[-1])
    h = np.load(h_path)
    g0 = float(h["gamma0"]); b0 = float(h["beta0"])
    names = ("NSFD", "FD", "NSFD box")
    fits = {}
    for n in names:
        dt = float(h["dt_" + n]); fits[n] = bench._gain_fit(h[n], dt, g0, b0, 0.03 / (g0 * b0) / (299792458.0 * dt))
    y = j["yardsticks"]; par = j["oracle_prefix_parity"]
    L = ["# Example 1 (infrared FEL) on the GPU: gain curves", "",
         "Commands (from the repository root):", "", "    python3 bench.py --workload example1 --ex1-history <hist.npz> > <example1.json>",
         "    python3 paper_2009_13645_amd/counters.py ex1 <example1.json> <hist.npz>", "",
         "64 x 64 x 2800 nodes (lab mesh 50 x 50 x 0.1 um, boosted dz = gamma0 x 0.1 um), 131072 macro-electrons generated on the device (Halton quiet start, uniform 100.5 um along z with tapers, b_f = 0.01 at the bunching wavenumber, energy spread 1e-4), 29.5 pC, planar K = 1.417, 3 cm period, gamma = 100.41, Mur-2, no space charge, FP64 fields and particles, 16000 field steps (8 m). Power: lab-frame Poynting flux through the plane 110 um (lab) ahead of the bunch centre, averaged over one radiation period, against z = gamma0 beta0 c t.", "",
         "Transverse profile: 'Gaussian' follows the job file (the manual: MITHRA's transverse distributions are always Gaussian and sigma-position is their rms, 260 um; the job's 4-sigma truncation and 3.2 mm mesh fit this); 'box' is the uniform 260 x 260 um box whose N / volume is the table's 2.72e13 cm^-3.", "",
         "| | NSFD, Gaussian | FD, Gaussian | NSFD, box |", "|---|---:|---:|---:|"]
    def row(t, f): L.append(f"| {t} | " + " | ".join(f(n) for n in names) + " |")
    row("ms per step", lambda n: f"{j['runs'][n]['ms_per_step']:.3f}")
    row("gain length, steepest 0.4 m (m)", lambda n: f"{fits[n]['gain_length_m']:.3f} (z {fits[n]['steepest_window']['z_m'][0]:.2f}-{fits[n]['steepest_window']['z_m'][1]:.2f})")
    row("first power maximum (MW at m)", lambda n: f"{fits[n]['p_first_peak_W']/1e6:.2f} at {fits[n]['z_first_peak_m']:.2f}")
    row("largest power in 8 m (MW at m)", lambda n: f"{fits[n]['p_max_W']/1e6:.2f} at {fits[n]['z_max_m']:.2f}")
    row("bunching factor at 8 m", lambda n: f"{j['runs'][n]['bunching_end']:.3f}")
    row("lab gamma, start -> 8 m", lambda n: f"{j['runs'][n]['lab_gamma_start']:.3f} -> {j['runs'][n]['lab_gamma_end']:.3f}")
    xg = y["xie_3d"]; xb = y["xie_3d_box"]
    dz = 100 * (fits['FD']['z_first_peak_m'] - fits['NSFD']['z_first_peak_m'])
    L += ["", "Yardsticks:", "",
          f"- the manual: MITHRA 0.22 m and \"2.6 GW\"; its table: 1-D gain length 0.224 m from rho = 0.006, with the electron density N / (sigma_x sigma_y L) = 2.72e13 cm^-3 (2 pi above the Gaussian beam's peak density), and \"2.7 GW\" printed for rho P_beam, which is 0.006 x {y['p_beam_W']/1e9:.2f} GW = {y['manual_rho_times_p_beam_W']/1e6:.1f} MW;",
          f"- Xie's 3-D fit (a_w = K/sqrt 2): Gaussian beam, on-axis density: rho_1D = {xg['rho_1d']:.4f}, gain length {xg['gain_length_3d_m']:.3f} m, saturation {xg['p_sat_3d_W']/1e6:.1f} MW; box beam: rho_1D = {xb['rho_1d']:.4f}, {xb['gain_length_3d_m']:.3f} m, {xb['p_sat_3d_W']/1e6:.1f} MW.", "",
          f"With the job file's beam the gain length is {fits['NSFD']['gain_length_m']:.2f} m, {100*(fits['NSFD']['gain_length_m']/xg['gain_length_3d_m']-1):+.0f}% against Xie's estimate for that beam and {fits['NSFD']['gain_length_m']/0.22:.1f}x the manual's 0.22 m; with the table's box density it is {fits['NSFD box']['gain_length_m']:.3f} m ({100*(fits['NSFD box']['gain_length_m']/0.22-1):+.0f}% against 0.22 m). NSFD and FD agree: FD {100*(fits['FD']['gain_length_m']/fits['NSFD']['gain_length_m']-1):+.0f}% in gain length, first maximum {abs(dz):.0f} cm {'later' if dz > 0 else 'earlier'}.", "",
          f"Oracle prefix parity (the Gaussian NSFD run, same device-generated bunch, {par['steps']} steps, FP64; each component against the norm of its vector field): positions {par['bunch_max_dz_cells']:.1e} cells; A {max(par[k] for k in par if k.startswith('rel_l2_A')):.1e}, J {max(par[k] for k in par if k.startswith('rel_l2_J')):.1e}, rho {par['rel_l2_Q']:.1e}, E {max(par[k] for k in par if k.startswith('rel_l2_E')):.1e}, B {max(par[k] for k in par if k.startswith('rel_l2_B')):.1e}, momenta {par['rel_l2_u']:.1e} (relative L2).", "",
          "Power (MW, one-period average):", "", "| z (m) | NSFD, Gaussian | FD, Gaussian | NSFD, box |", "|---:|---:|---:|---:|"]
    for zz in np.arange(0.5, 8.01, 0.5):
        vals = [np.interp(zz, np.array(fits[n]["curve_z_m"]), np.array(fits[n]["curve_P_W"])) / 1e6 for n in names]
        L.append(f"| {zz:.1f} | " + " | ".join(f"{v:.4g}" for v in vals) + " |")
    open(os.path.join(ROOT, "profiles", "example1_gain_curve.md"), "w").write("\n".join(L) + "\n")
    # convergence
    if c_path:
        c = json.loads(open(c_path).read().strip().splitlines()[-1])
        cz = np.load(cz_path)
        M = ["# Example 1 convergence study on the GPU (the manual's error of eq. errorDefinition)", "",
             "Commands (from the repository root):", "", "    python3 bench.py --workload example1-convergence --ex1-history <conv_hist.npz> > <convergence.json>",
             "    python3 paper_2009_13645_amd/counters.py ex1 <example1.json> <hist.npz> <convergence.json> <conv_hist.npz>", "",
             "Each row runs Example 1 (the job file's Gaussian beam, NSFD, Mur-2, FP64, device-generated bunch with b_f = 0.01, sorted every push) to 5.5 m of undulator with one numerical parameter changed from the job file's value. error = integral of |P - P_0| over integral of P_0 along the 5 m undulator, P_0 being the finer run's power (one-period average at the plane 110 um ahead of the bunch centre). The last row compares two space-charge runs. Gain length: steepest 0.4 m of ln P after the entrance transient.", "",
             "| run | nodes | particles | n_sub | ms/step | gain length (m) | first power maximum (MW at m) | error against the job's values |",
             "|---|---|---:|---:|---:|---:|---:|---:|"]
        for k, v in c["runs"].items():
            if k == "space charge, l_z 380 um":
                errs = f"{c['error']['space charge, l_z 380 um vs space charge']:.3f} (against the space-charge run)"
            else:
                e = c["error"].get(k); errs = "reference" if e is None else f"{e:.3f}"
            key = k.replace(" ", "_").replace("/", "over")
            z = cz[key + "_z"]; P = cz[key + "_P"]
            lp = np.log(np.maximum(P, 1e-300)); dz_ = z[1] - z[0]; m = int(round(0.4 / dz_))
            ipk = int(np.argmax(P[: np.searchsorted(z, 5.4)]))
            st = np.nonzero(P[:ipk] > 1e-3 * P[ipk])[0]; a0 = int(st[0]) if len(st) else 0
            best = 0.0
            for a in range(a0, max(ipk - m, a0), max(m // 8, 1)):
                best = max(best, np.polyfit(z[a:a + m], lp[a:a + m], 1)[0])
            lg = 1 / best if best > 0 else float("nan")
            M.append(f"| {k} | {'x'.join(map(str, v['nodes']))} | {v['particles']} | {v['n_sub']} | {v['ms_per_step']:.3f} | {lg:.3f} | {P[ipk]/1e6:.2f} at {z[ipk]:.2f} | {errs} |")
        open(os.path.join(ROOT, "profiles", "example1_convergence.md"), "w").write("\n".join(M) + "\n")
        print("\n".join(M))
    print("\n".join(L[:26]))


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "run":
        run()
    elif len(sys.argv) >= 6 and sys.argv[1] == "push":
        summarize_push(sys.argv[2:6])
    elif len(sys.argv) >= 4 and sys.argv[1] == "ex1":
        ex1(*sys.argv[2:6])
    elif len(sys.argv) >= 3 and sys.argv[1] == "bstats":
        bstats(sys.argv[2])
    elif len(sys.argv) >= 4 and sys.argv[1] == "kstats":
        kstats(sys.argv[2], int(sys.argv[3]))
    elif len(sys.argv) >= 4 and sys.argv[1] == "summarize":
        summarize(sys.argv[2], sys.argv[3])
    else:
        print(__doc__)
        sys.exit(1)
