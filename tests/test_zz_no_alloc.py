"""The allocation-free bunching entry point against the ordinary one, through
the C ABI, on two calls in a row (the second run has fewer particles)."""
import ctypes as C

import numpy as np
import pytest
import torch  # noqa: F401

from paper_2009_13645_amd import workloads as W

pytestmark = pytest.mark.gpu


def _both(n, steps, seed):
    from paper_2009_13645_amd.engine import Engine, lib
    w = W.config1()
    w.n_particles = n
    d = w.descriptor()
    xyz, u, q = W.make_bunch(w, seed=seed)
    g = Engine(d, max_particles=n)
    g.load_bunch(xyz, u, q)
    g.step(steps)
    ref = C.c_double()
    got = C.c_double()
    assert lib().mithra_bunching(g._h, C.byref(ref)) == 0
    assert lib().mithra_bunching_noalloc(g._h, C.byref(got)) == 0
    g.close()
    return ref.value, got.value


def test_noalloc_bunching_equals_the_ordinary_call_twice():
    r1, g1 = _both(4096, 30, 11)
    r2, g2 = _both(700, 12, 12)  # smaller input, same scratch
    print(f"[noalloc] {r1:.17e} {g1:.17e} | {r2:.17e} {g2:.17e}", flush=True)
    assert r1 > 0 and r2 > 0 and r1 != r2
    assert g1 == pytest.approx(r1, rel=1e-14, abs=0)
    assert g2 == pytest.approx(r2, rel=1e-14, abs=0)
