"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, sizes its arena exactly, and rejects bad
descriptors before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2009_13645_amd import engine as E
from paper_2009_13645_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "mithra.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(mithra_[a-z_0-9]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    L = E.lib()
    syms = declared_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(L, s), s


def _desc(**kw):
    d = W.config1().descriptor()
    d.update(kw)
    return d


def test_footprint_is_exact_monotone_and_zero_for_invalid():
    f1 = E.footprint_bytes(_desc(), 4096)
    f2 = E.footprint_bytes(_desc(), 8192)
    f3 = E.footprint_bytes(_desc(nx=40), 4096)
    f32 = E.footprint_bytes(_desc(field_precision=32), 4096)
    f32c = E.footprint_bytes(_desc(field_precision=32, compensated=1), 4096)
    assert 0 < f1 < f2 and f1 < f3
    assert f32 < f1 and f32 < f32c
    nn = 32 * 32 * 64
    # potentials (12 arrays), sources (8), vertex fields (6) at 8 bytes at least
    assert f1 >= 26 * nn * 8
    assert E.footprint_bytes(_desc(nx=3), 4096) == 0


@pytest.mark.parametrize("bad", [
    dict(nx=5), dict(truncation_order=3), dict(space_charge=2), dict(solver=2), dict(n_sub=0),
    dict(field_precision=16), dict(compensated=1, field_precision=64), dict(und_type=4), dict(n_freq=65),
    dict(n_freq=2, nu_min=float("nan")),
    dict(n_periods=0), dict(k_plane=0), dict(k_plane=63), dict(tile=(0, 8, 8)),
    dict(tile=(8, 65, 8)), dict(dx=0.0), dict(gamma=1.0), dict(K=0.0), dict(lambda_u=-1.0),
    dict(dz=1.0), dict(z_entrance=float("nan")), dict(nx=(1 << 20) + 1), dict(sort_every=-1),
    dict(sort_every=1025),
])
def test_invalid_descriptors_are_rejected_without_device(bad):
    g = E.make_desc(_desc(**bad), 4096)
    h = C.c_void_p()
    rc = E.lib().mithra_init_grid(C.byref(g), None, 0, None, C.byref(h))
    assert rc == -1
    msg = E.lib().mithra_last_error(h).decode()
    assert len(msg) > 5
    E.lib().mithra_destroy(h)


def test_small_arena_is_enomem_and_null_handle_calls_fail():
    g = E.make_desc(_desc(), 4096)
    h = C.c_void_p()
    rc = E.lib().mithra_init_grid(C.byref(g), None, 0, None, C.byref(h))
    assert rc == -2
    E.lib().mithra_destroy(h)
    assert E.lib().mithra_step(None, 1) == -1
    assert E.lib().mithra_destroy(None) == -1
    assert E.lib().mithra_last_error(None) == b"null handle"


def test_library_loads_after_torch_whatever_the_first_call():
    """A program whose first call is host-only (footprint_bytes) still gets
    torch, and with it torch's HIP runtime, into the process before the
    library is loaded (loaded first, the library's HIP calls found no
    device)."""
    import subprocess
    import sys
    code = ("import sys\n"
            "from paper_2009_13645_amd import engine as E, workloads as W\n"
            "assert 'torch' not in sys.modules\n"
            "w = W.config1()\n"
            "assert E.footprint_bytes(w.descriptor(), w.n_particles) > 0\n"
            "assert 'torch' in sys.modules\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]


def test_batch_workspace_and_argument_checks_without_device():
    L = E.lib()
    assert L.mithra_batch_workspace_bytes(0) == 0
    w1 = L.mithra_batch_workspace_bytes(1)
    w64 = L.mithra_batch_workspace_bytes(64)
    assert 0 < w1 < w64
    out = C.c_void_p()
    # no members, null workspace: rejected before any device call
    assert L.mithra_batch_create(None, 0, None, 0, None, C.byref(out)) == -1
    assert out.value is None
    assert L.mithra_batch_run(None, None) == -1
    assert L.mithra_batch_autotune_sweep(None, 3, None) == -1
    assert L.mithra_batch_destroy(None) == -1


def test_adapt_mesh_meets_the_nsfd_condition_and_divides_the_field_step():
    """MESH auto-adjustment (ch. 4 MESH): dx and dy scaled by one factor so
    that (dz/dx)^2 + (dz/dy)^2 = 0.98 when the NSFD condition fails, and
    n_sub = round(dt / bunch step) (at least 1); FD leaves the mesh."""
    d = _desc()
    d.update(dx=1.1 * d["dz"], dy=1.3 * d["dz"])
    assert E.footprint_bytes(d, 16) == 0  # rejected as given
    a, changed = E.adapt_mesh(d, bunch_time_step=0.0)
    q = (a["dz"] / a["dx"]) ** 2 + (a["dz"] / a["dy"]) ** 2
    assert changed == 1 and q == pytest.approx(0.98, rel=1e-14)
    assert a["dx"] / a["dy"] == pytest.approx(1.1 / 1.3, rel=1e-14)
    assert E.footprint_bytes(a, 16) > 0
    dt = a["dz"] / 299792458.0
    b, changed = E.adapt_mesh(a, bunch_time_step=dt / 3.3)
    assert changed == 2 and b["n_sub"] == 3 and b["dx"] == a["dx"]
    c, changed = E.adapt_mesh(b, bunch_time_step=10 * dt)
    assert c["n_sub"] == 1
    # FD: no NSFD condition; its field step is 0.99 of the stable step
    f = dict(d, solver=1)
    g, changed = E.adapt_mesh(f, bunch_time_step=0.0)
    assert changed == 0 and g["dx"] == f["dx"]
    assert E.footprint_bytes(f, 16) > 0
