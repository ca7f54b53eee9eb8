"""Served stream on the GPU: a request's result is the same alone and in
the mix (continuous batching: runs join and leave the batch between
ticks), within the precision bars: FP64 results to 1e-11 relative and FP32
to 1e-5 (only the order of the deposit's atomic additions differs)."""
import numpy as np
import pytest
import torch  # noqa: F401

from paper_2009_13645_amd import workloads as W
from paper_2009_13645_amd.serve import Server, request_from_workload, summarize

pytestmark = pytest.mark.gpu


def stream():
    reqs = W.config5_requests(n_req=8, rate_hz=200.0, scale=0.02)
    out = []
    for i, (t, w) in enumerate(reqs):
        out.append(request_from_workload(i, t, w, steps=20 + 9 * i, keep_fields=("Ex", "Ay", "Q")))
    return out, [w for _, w in reqs]


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / nb) if nb > 0 else float(np.linalg.norm(a))


def test_alone_equals_in_the_mix():
    reqs, ws = stream()
    for r, w in zip(reqs, ws):
        print(f"[serve] request {r.rid} {w.name} np={r.n_particles} steps={r.steps} prec={w.field_precision}",
              flush=True)
    srv = Server(max_active=4, tick_steps=16)
    mix = {r.rid: r for r in srv.run(reqs, realtime=False)}
    print("[serve] stats", srv.stats, summarize(list(mix.values()), wall=1.0), flush=True)
    assert sorted(mix) == list(range(len(reqs)))
    assert srv.stats["rebuilds"] > 1  # runs joined and left mid-flight
    for rid in (0, 3, 6, 7):
        alone = Server(max_active=4, tick_steps=16).run([reqs[rid]], realtime=False)[0]
        m = mix[rid]
        tol = 1e-11 if ws[rid].field_precision == 64 else 1e-5
        errs = {"power": rel(m.power, alone.power), "b": abs(m.bunching - alone.bunching) / max(abs(alone.bunching), 1e-300)}
        for f in alone.fields:
            errs[f] = rel(m.fields[f], alone.fields[f])
        print(f"[serve] request {rid} alone vs mix:", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
        assert len(m.power) == reqs[rid].steps
        for k, v in errs.items():
            assert v < tol, (rid, k, v)
