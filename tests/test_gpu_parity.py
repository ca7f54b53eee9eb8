"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars (fixed in the run contract): fields and momenta within 1e-10 relative
L2 at FP64 and 2e-4 at FP32 after 200 steps; cell indices and sort order
bit-exact on identical FP64 positions.
"""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (the first import is slow on a fresh box: keep it out of timed tests)

from oracle.oracle import Oracle
from paper_2009_13645_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["Ax", "Ay", "Az", "F", "Jx", "Jy", "Jz", "Q", "Ex", "Ey", "Ez", "Bx", "By", "Bz"]


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def engine(d, n):
    import torch
    from paper_2009_13645_amd.engine import Engine
    assert torch.cuda.is_available()
    return Engine(d, max_particles=n)


def run_both(w, steps, d_over=None, n=None, seed=None):
    d = w.descriptor()
    if d_over:
        d.update(d_over)
    xyz, u, q = W.make_bunch(w, n=n, seed=seed)
    print(f"[parity] {w.name} {d['nx']}x{d['ny']}x{d['nz']} np={len(xyz)} steps={steps} "
          f"prec={d['field_precision']} comp={d['compensated']}", flush=True)
    o = Oracle(d)
    o.load_bunch(xyz, u, q)
    g = engine(d, len(xyz))
    g.load_bunch(xyz, u, q)
    if steps:
        o.step(steps)
        g.step(steps)
    return d, o, g


def compare(d, o, g, tol, fields=FIELDS, ptol=None):
    worst = {}
    for f in fields:
        a = g.read_field(f)
        b = o.field(f)
        worst[f] = rel_l2(a, b)
    xg, ug, cg, pg = g.read_particles()
    xo, uo, co, po = o.particles()
    h = np.array([d["dx"], d["dy"], d["dz"]])
    worst["r(cells)"] = float(np.sqrt(np.mean(np.sum(((xg - xo) / h) ** 2, axis=1))))
    worst["u"] = rel_l2(ug, uo)
    print("[parity] errors:", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    for f in fields:
        assert worst[f] < tol, (f, worst[f])
    assert worst["u"] < (ptol or tol)
    assert worst["r(cells)"] < (ptol or tol) * 10
    return cg, co, pg, po


def test_config1_fp64_parity_200_steps():
    w = W.config1()
    d, o, g = run_both(w, 200)
    cg, co, pg, po = compare(d, o, g, 1e-10)
    mism = int(np.sum(cg != co)) + int(np.sum(pg != po))
    print("[parity] cell/perm mismatches after 200 steps:", mism, flush=True)
    assert mism == 0
    # diagnostics
    assert g.radiated_power() == pytest.approx(o.radiated_power(), rel=1e-9, abs=1e-30)
    assert g.bunching() == pytest.approx(o.bunching(), rel=1e-10)


@pytest.mark.parametrize("which,every,steps", [("tiny", 3, 200), ("tiny", 3, 202), ("small", 4, 41),
                                                ("small", 4, 43), ("small", 8, 47), ("small", 16, 49)])
def test_sort_every_few_steps_matches_the_oracle(which, every, steps):
    """Sorting after every few pushes only (the order kept in between) on
    both sides: fields, momenta, cells and the order itself, ending after a
    push with and without a sort; the one-workgroup and the multi-block
    sort paths."""
    w = W.config1() if which == "tiny" else W.config2_small(field_precision=64)
    d, o, g = run_both(w, steps, d_over=dict(sort_every=every))
    cg, co, pg, po = compare(d, o, g, 1e-10)
    mism = int(np.sum(cg != co)) + int(np.sum(pg != po))
    print(f"[parity] sort every {every}: cell/perm mismatches after {steps} steps:", mism, flush=True)
    assert mism == 0
    assert g.bunching() == pytest.approx(o.bunching(), rel=1e-10)


@pytest.mark.parametrize("which", ["tiny", "small"])
def test_power_history_matches_oracle_each_step(which):
    """The power recorded inside each step (partial sums in the vertex-field
    launch; the tiny run's one-workgroup sort adds them, a separate kernel
    otherwise) against the oracle's plane power after the same step."""
    if which == "tiny":
        w, steps = W.config1(), 24            # 4096 e-: one-workgroup sort ends the step
    else:
        w, steps = W.config2_small(field_precision=64), 12  # 20000 e-: multi-block sort
    d = w.descriptor()
    xyz, u, q = W.make_bunch(w)
    o = Oracle(d)
    o.load_bunch(xyz, u, q)
    g = engine(d, len(xyz))
    g.load_bunch(xyz, u, q)
    want, asked = [], []
    for _ in range(steps):
        o.step(1)
        g.step(1)
        want.append(o.radiated_power())
        asked.append(g.radiated_power())  # the on-request path, same fields
    hist = g.power_history(steps)
    print(f"[parity] power history {which}: {steps} steps, last {hist[-1]:.6e} W", flush=True)
    assert len(hist) == steps
    assert np.all(np.isfinite(hist))
    np.testing.assert_allclose(hist, np.array(asked), rtol=1e-12, atol=0.0)
    scale = max(np.max(np.abs(want)), 1e-300)
    np.testing.assert_allclose(hist, np.array(want), rtol=1e-9, atol=1e-9 * scale)
    o.close()
    g.close()


@pytest.mark.parametrize("comp", [0, 1])
def test_config1_fp32_parity_200_steps(comp):
    w = W.config1()
    w.field_precision = 32
    w.compensated = comp
    d, o, g = run_both(w, 200)
    compare(d, o, g, 2e-4, ptol=2e-4)


@pytest.mark.parametrize("prec", [64, 32])
def test_every_sweep_tile_shape_matches_oracle(prec):
    """All sweep kernels (scalar tiles and 16-byte vector tiles) on a ragged
    grid whose x length allows vectors: 60 steps against the oracle."""
    from paper_2009_13645_amd.engine import Engine
    w = W.Workload(name="shapes", nx=40, ny=27, nz=45, gamma=120.0, K=1.2, lambda_u=0.03,
                   n_periods=30, n_particles=1500, sigma_cells=(3.0, 2.0, 2.0), seed=8,
                   field_precision=prec, tile=(8, 4, 8))
    d = w.descriptor()
    xyz, u, q = W.make_bunch(w)
    o = Oracle(d)
    o.load_bunch(xyz, u, q)
    o.step(60)
    ref = {f: o.field(f) for f in ("Ax", "Az", "F", "Jz", "Q")}
    uo = o.particles()[1]
    tol = 1e-10 if prec == 64 else 2e-4
    for shape in range(Engine.sweep_shape_count()):
        g = engine(d, len(xyz))
        g.set_sweep_shape(shape)
        g.load_bunch(xyz, u, q)
        g.step(60)
        errs = {f: rel_l2(g.read_field(f), ref[f]) for f in ref}
        errs["u"] = rel_l2(g.read_particles()[1], uo)
        print(f"[parity] shape {shape}:", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
        assert max(errs.values()) < tol, (shape, errs)
        g.close()


def test_sort_and_cells_bit_exact_on_identical_positions():
    """Keys from the loaded FP64 positions: tie-heavy, ragged tiles, inactive."""
    w = W.Workload(name="sort", nx=37, ny=29, nz=53, gamma=100.0, K=1.0, lambda_u=0.03,
                   n_periods=40, n_particles=50000, tile=(5, 3, 7))
    d = w.descriptor()
    rng = np.random.default_rng(12)
    n = 50000
    g = np.stack([rng.uniform(-1, d["nx"], n), rng.uniform(-1, d["ny"], n),
                  rng.uniform(-1, d["nz"], n)], axis=1)
    g[: n // 4] = np.floor(g[: n // 4]) + 0.5  # many particles at identical points
    g[n // 4: n // 2] = np.round(g[n // 4: n // 2])  # exactly on cell faces
    xyz = np.stack([d["x0"] + g[:, 0] * d["dx"], d["y0"] + g[:, 1] * d["dy"],
                    d["z0"] + g[:, 2] * d["dz"]], axis=1)
    u = np.zeros((n, 3))
    for tile in [(5, 3, 7), (8, 8, 8), (36, 28, 52), (1, 1, 1)]:
        d["tile"] = tile
        o = Oracle(d)
        o.load_bunch(xyz, u, 0.0)
        e = engine(d, n)
        e.load_bunch(xyz, u, 0.0)
        _, _, cg, pg = e.read_particles()
        _, _, co, po = o.particles()
        assert np.array_equal(cg, co), tile
        assert np.array_equal(pg, po), tile


@pytest.mark.parametrize("variant", [
    dict(name="ragged-helical", nx=23, ny=19, nz=41, und_type=1, K=1.4, gamma=150.0, order=2, sc=1, nsub=1),
    dict(name="mur1-nosc-nsub3", nx=20, ny=26, nz=35, und_type=0, K=0.8, gamma=80.0, order=1, sc=0, nsub=3),
    dict(name="tiny-6", nx=8, ny=8, nz=10, und_type=0, K=1.0, gamma=60.0, order=2, sc=1, nsub=1),
    dict(name="polarised-30deg", nx=24, ny=24, nz=48, und_type=0, K=1.2, gamma=120.0, order=2, sc=1, nsub=2,
         pol=30.0),
])
def test_edge_case_geometries_fp64(variant):
    v = variant
    w = W.Workload(name=v["name"], nx=v["nx"], ny=v["ny"], nz=v["nz"], gamma=v["gamma"], K=v["K"],
                   lambda_u=0.03, n_periods=20, und_type=v["und_type"], n_sub=v["nsub"],
                   truncation_order=v["order"], space_charge=v["sc"], n_particles=700,
                   sigma_cells=(v["nx"] / 12, v["ny"] / 12, v["nz"] / 24), seed=21,
                   pol_angle_deg=v.get("pol", 0.0), tile=(4, 4, 4))
    steps = 60
    d, o, g = run_both(w, steps)
    compare(d, o, g, 1e-10)


def test_empty_active_region_and_single_particle():
    """All particles outside the active region: no deposit, external push only."""
    w = W.config1()
    d = w.descriptor()
    xyz = np.array([[d["x0"] + 0.2 * d["dx"], 0.0, d["z0"] + 10 * d["dz"]]])
    u = np.array([[0.0, 0.0, 0.3]])
    o = Oracle(d)
    o.load_bunch(xyz, u, -1e-15)
    g = engine(d, 1)
    g.load_bunch(xyz, u, -1e-15)
    o.step(20)
    g.step(20)
    xg, ug, cg, pg = g.read_particles()
    xo, uo, co, po = o.particles()
    assert cg[0] == -1 and co[0] == -1
    np.testing.assert_allclose(ug, uo, rtol=1e-12, atol=1e-14)
    assert np.max(np.abs(g.read_field("Q"))) == 0.0


@pytest.mark.parametrize("prec,comp,tol", [(64, 0, 1e-10), (32, 1, 1e-5)])
def test_continuity_and_charge_on_gpu_full_size_config2(prec, comp, tol):
    """Full-size FEL-amplifier geometry (128x128x1024 nodes, 2^21 e-): discrete
    continuity of the GPU's own J and rho and the total charge hold at any
    size.  FP32 + compensation is the benchmark's configuration."""
    w = W.config2(field_precision=prec, compensated=comp)
    d = w.descriptor()
    xyz, u, q = W.make_bunch(w)
    g = engine(d, len(xyz))
    g.load_bunch(xyz, u, q)
    g.step(3)
    rho0 = g.read_field("Q")
    g.step(1)
    rho1 = g.read_field("Q")
    J = [g.read_field(n) for n in ("Jx", "Jy", "Jz")]
    dt = g.constants()["dt"]
    div = np.zeros_like(rho1)
    for arr, ax, h in ((J[0], 2, d["dx"]), (J[1], 1, d["dy"]), (J[2], 0, d["dz"])):
        div += (arr - np.roll(arr, 1, axis=ax)) / h
    res = (rho1 - rho0) / dt + div
    scale = np.max(np.abs(rho1)) / dt
    print(f"[parity] cfg2 prec={prec} continuity residual / scale:",
          float(np.max(np.abs(res)) / scale), flush=True)
    assert np.max(np.abs(res)) < tol * scale
    _, _, cell, perm = g.read_particles()
    V = d["dx"] * d["dy"] * d["dz"]
    assert np.sum(rho1) * V == pytest.approx(q * np.sum(cell >= 0), rel=max(tol, 1e-9) * 10)
    assert np.array_equal(np.sort(perm), np.arange(len(xyz)))


def test_full_size_config2_against_oracle_few_steps():
    """Full-size FEL amplifier, FP64: two steps on both sides, all fields,
    particles, cells and sort order compared (the oracle runs on the host
    cores in seconds at this length)."""
    w = W.config2(field_precision=64)
    d, o, g = run_both(w, 2)
    cg, co, pg, po = compare(d, o, g, 1e-10)
    assert int(np.sum(cg != co)) == 0
    assert int(np.sum(pg != po)) == 0


def _block_boxes(d, xyz, tile, per):
    """Node boxes of consecutive groups of `per` particles in the sort order
    (tile-major cell key, ties by id), from the cells at load; the deposit
    box of the first push is this box grown by at most one cell."""
    n = np.array([d["nx"], d["ny"], d["nz"]])
    o = np.array([d["x0"], d["y0"], d["z0"]])
    h = np.array([d["dx"], d["dy"], d["dz"]])
    c = np.floor((xyz - o) / h).astype(np.int64)
    act = np.all((c >= 1) & (c <= n - 3), axis=1)
    T = np.array(tile)
    nt = (n - 1 + T - 1) // T
    t = c // T
    loc = c % T
    key = ((t[:, 2] * nt[1] + t[:, 1]) * nt[0] + t[:, 0]) * int(np.prod(T)) + \
        (loc[:, 2] * T[1] + loc[:, 1]) * T[0] + loc[:, 0]
    key = np.where(act, key, np.iinfo(np.int64).max)
    order = np.lexsort((np.arange(len(key)), key))
    cs = c[order][act[order]]
    vols = []
    for b in range(0, len(cs), per):
        g = cs[b:b + per]
        vols.append(int(np.prod(g.max(0) - g.min(0) + 2)))
    return np.array(vols)


def test_deposit_box_overflow_paths_fp64():
    """8x8x8 sort tiles on a dense bunch: workgroups whose particles straddle
    rows of tiles overflow the LDS box and deposit through per-wavefront
    boxes, or global atomics for a wavefront that does not fit either."""
    w = W.Workload(name="box-overflow", nx=96, ny=96, nz=48, gamma=100.0, K=1.0, lambda_u=0.03, n_periods=20,
                   n_particles=60000, sigma_cells=(12.0, 12.0, 6.0), seed=31, tile=(8, 8, 8))
    d = w.descriptor()
    xyz, _, _ = W.make_bunch(w)
    blocks = _block_boxes(d, xyz, (8, 8, 8), 256)
    waves = _block_boxes(d, xyz, (8, 8, 8), 64)
    print(f"[parity] box-overflow: {int(np.sum(blocks > 1536))} of {len(blocks)} workgroups overflow; "
          f"{int(np.sum(waves <= 384))} of {len(waves)} wavefront boxes fit a quarter", flush=True)
    assert np.sum(blocks > 1536) > 0 and np.sum(waves > 384) > 0
    d, o, g = run_both(w, 30)
    cg, co, pg, po = compare(d, o, g, 1e-10)
    assert int(np.sum(cg != co)) == 0 and int(np.sum(pg != po)) == 0
