"""Thin Python binding of the C ABI in include/mithra.h.

Argument marshalling only: every step of the PIC path runs in the HIP
library `libmithra.so`.  PyTorch provides the device arena (a uint8 tensor)
and the stream; nothing here computes physics.  If the library is missing
the import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmithra.so")

FIELD_IDS = {"Ex": 0, "Ey": 1, "Ez": 2, "Bx": 3, "By": 4, "Bz": 5, "Ax": 6, "Ay": 7,
             "Az": 8, "Jx": 9, "Jy": 10, "Jz": 11, "F": 12, "Q": 13}
ERRORS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "ENUMERIC"}


class MithraError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    """ctypes mirror of `mithra_grid_desc`."""
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("truncation_order", C.c_int32), ("space_charge", C.c_int32),
                ("solver", C.c_int32), ("n_sub", C.c_int32), ("field_precision", C.c_int32),
                ("compensated", C.c_int32), ("und_type", C.c_int32), ("n_periods", C.c_int32),
                ("k_plane", C.c_int32), ("tile", C.c_int32 * 3), ("record_power", C.c_int32),
                ("max_particles", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("gamma", C.c_double), ("K", C.c_double), ("lambda_u", C.c_double),
                ("pol_angle_deg", C.c_double), ("z_entrance", C.c_double),
                ("n_freq", C.c_int32), ("sort_every", C.c_int32), ("nu_min", C.c_double), ("nu_max", C.c_double)]


class UndulatorDesc(C.Structure):
    """ctypes mirror of `mithra_undulator_desc`."""
    _fields_ = [("n_modules", C.c_int32), ("signal", C.c_int32), ("gap", C.c_double), ("dK", C.c_double),
                ("ctau", C.c_double), ("ct0", C.c_double), ("cep_deg", C.c_double),
                ("w0_par", C.c_double), ("w0_perp", C.c_double), ("z_focus", C.c_double)]


class SeedDesc(C.Structure):
    """ctypes mirror of `mithra_seed_desc`."""
    _fields_ = [("type", C.c_int32), ("signal", C.c_int32), ("a0", C.c_double), ("wavelength", C.c_double),
                ("ctau", C.c_double), ("ct0", C.c_double), ("cep_deg", C.c_double), ("pol_deg", C.c_double),
                ("w0", C.c_double), ("z_focus", C.c_double)]


class BunchDesc(C.Structure):
    """ctypes mirror of `mithra_bunch_desc`."""
    _fields_ = [("long_profile", C.c_int32), ("trans_profile", C.c_int32), ("shot_noise", C.c_int32),
                ("tapers", C.c_int32), ("center", C.c_double * 3), ("size", C.c_double * 3),
                ("gamma", C.c_double), ("sigma_gamma_rel", C.c_double), ("sigma_u_perp", C.c_double),
                ("bunching", C.c_double), ("bunching_phase", C.c_double), ("n_electrons", C.c_double)]


def _fill(struct, d: dict):
    s = struct()
    for name, typ in struct._fields_:
        if name not in d:
            continue
        v = d[name]
        if hasattr(typ, "_length_"):
            arr = getattr(s, name)
            for i, x in enumerate(v):
                arr[i] = float(x)
        else:
            setattr(s, name, v)
    return s


_lib = None


def lib():
    """Load libmithra.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2009_13645_amd.build` (no CPU fallback exists)")
        # torch first: its HIP runtime must be in the process before the
        # library binds its own HIP dependency.  Loaded before torch, the
        # library's HIP calls failed with "no ROCm-capable device is
        # detected" on a machine with a GPU (footprint_bytes, host code
        # only, can be the first call of a program).
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.mithra_footprint_bytes.argtypes = [C.POINTER(GridDesc), C.c_int64]
        L.mithra_footprint_bytes.restype = C.c_size_t
        L.mithra_init_grid.argtypes = [C.POINTER(GridDesc), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(H)]
        L.mithra_init_grid.restype = C.c_int
        L.mithra_load_bunch.argtypes = [H, C.c_int64, dp, dp, C.c_double]
        L.mithra_load_bunch.restype = C.c_int
        L.mithra_step.argtypes = [H, C.c_int64]
        L.mithra_step.restype = C.c_int
        L.mithra_read_fields.argtypes = [H, C.c_int, C.c_int, C.c_void_p, C.c_size_t]
        L.mithra_read_fields.restype = C.c_int
        L.mithra_read_particles.argtypes = [H, dp, dp, ip, ip]
        L.mithra_read_particles.restype = C.c_int
        L.mithra_radiated_power.argtypes = [H, C.c_int32, dp]
        L.mithra_radiated_power.restype = C.c_int
        L.mithra_power_history.argtypes = [H, dp, C.c_int64]
        L.mithra_power_history.restype = C.c_int64
        L.mithra_bunching.argtypes = [H, dp]
        L.mithra_bunching.restype = C.c_int
        L.mithra_constants.argtypes = [H, dp]
        L.mithra_constants.restype = C.c_int
        L.mithra_last_error.argtypes = [H]
        L.mithra_last_error.restype = C.c_char_p
        L.mithra_destroy.argtypes = [H]
        L.mithra_destroy.restype = C.c_int
        L.mithra_set_sweep_shape.argtypes = [H, C.c_int]
        L.mithra_set_sweep_shape.restype = C.c_int
        L.mithra_sweep_shape_count.restype = C.c_int
        L.mithra_time_sweep.argtypes = [H, C.c_int, C.c_int, dp]
        L.mithra_time_sweep.restype = C.c_int
        L.mithra_step_timed.argtypes = [H, C.c_int64, dp, dp]
        L.mithra_step_timed.restype = C.c_int
        L.mithra_bunching_noalloc.argtypes = [H, dp]
        L.mithra_bunching_noalloc.restype = C.c_int
        L.mithra_spectral_power.argtypes = [H, dp, C.c_int64]
        L.mithra_spectral_power.restype = C.c_int64
        L.mithra_set_undulator.argtypes = [H, C.POINTER(UndulatorDesc)]
        L.mithra_set_undulator.restype = C.c_int
        L.mithra_set_seed.argtypes = [H, C.POINTER(SeedDesc)]
        L.mithra_set_seed.restype = C.c_int
        L.mithra_adapt_mesh.argtypes = [C.POINTER(GridDesc), C.c_double, C.POINTER(C.c_int32)]
        L.mithra_adapt_mesh.restype = C.c_int
        L.mithra_generate_bunch.argtypes = [H, C.POINTER(BunchDesc), C.c_int64, C.c_double]
        L.mithra_generate_bunch.restype = C.c_int
        L.mithra_step_profile.argtypes = [H, C.c_int64, dp]
        L.mithra_step_profile.restype = C.c_int
        L.mithra_autotune_sweep.argtypes = [H, C.c_int, C.POINTER(C.c_int)]
        L.mithra_autotune_sweep.restype = C.c_int
        L.mithra_batch_workspace_bytes.argtypes = [C.c_int32]
        L.mithra_batch_workspace_bytes.restype = C.c_size_t
        L.mithra_batch_create.argtypes = [C.POINTER(H), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                          C.POINTER(H)]
        L.mithra_batch_create.restype = C.c_int
        L.mithra_batch_run.argtypes = [H, C.POINTER(C.c_int64)]
        L.mithra_batch_run.restype = C.c_int
        L.mithra_batch_sync.argtypes = [H]
        L.mithra_batch_sync.restype = C.c_int
        L.mithra_batch_autotune_sweep.argtypes = [H, C.c_int, C.POINTER(C.c_int32)]
        L.mithra_batch_autotune_sweep.restype = C.c_int
        L.mithra_batch_last_error.argtypes = [H]
        L.mithra_batch_last_error.restype = C.c_char_p
        L.mithra_batch_destroy.argtypes = [H]
        L.mithra_batch_destroy.restype = C.c_int
        _lib = L
    return _lib


def make_desc(d: dict, max_particles: int, record_power: int = 1) -> GridDesc:
    g = GridDesc()
    for k in ("nx", "ny", "nz", "truncation_order", "space_charge", "solver", "n_sub",
              "field_precision", "compensated", "und_type", "n_periods", "k_plane"):
        setattr(g, k, int(d[k]))
    for a in range(3):
        g.tile[a] = int(d["tile"][a])
    g.record_power = int(d.get("record_power", record_power))
    g.max_particles = int(max_particles)
    for k in ("dx", "dy", "dz", "x0", "y0", "z0", "gamma", "K", "lambda_u", "pol_angle_deg",
              "z_entrance"):
        setattr(g, k, float(d[k]))
    g.n_freq = int(d.get("n_freq", 0))
    g.sort_every = int(d.get("sort_every", 1))
    g.nu_min = float(d.get("nu_min", 1.0))
    g.nu_max = float(d.get("nu_max", 1.0))
    return g


def adapt_mesh(d: dict, bunch_time_step: float = 0.0) -> Tuple[dict, int]:
    """The MESH auto-adjustment: returns the adapted descriptor and the
    mask of what changed (1: dx and dy, 2: n_sub)."""
    g = make_desc(d, 1)
    changed = C.c_int32(0)
    rc = lib().mithra_adapt_mesh(C.byref(g), float(bunch_time_step), C.byref(changed))
    if rc != 0:
        raise MithraError(rc, "mesh adjustment refused")
    out = dict(d)
    out.update(dx=g.dx, dy=g.dy, n_sub=g.n_sub)
    return out, int(changed.value)


def footprint_bytes(d: dict, n_particles: int) -> int:
    g = make_desc(d, n_particles)
    return int(lib().mithra_footprint_bytes(C.byref(g), int(n_particles)))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Engine:
    """One run on the current CUDA/HIP device (torch provides arena and stream)."""

    def __init__(self, desc: dict, max_particles: int, device: str = "cuda:0",
                 stream=None, arena=None):
        import torch
        self._L = lib()
        self.desc = dict(desc)
        self.shape = (int(desc["nz"]), int(desc["ny"]), int(desc["nx"]))
        self._g = make_desc(desc, max_particles)
        nbytes = int(self._L.mithra_footprint_bytes(C.byref(self._g), int(max_particles)))
        if nbytes == 0:
            raise MithraError(-1, "invalid descriptor (footprint 0)")
        self.footprint = nbytes
        self.device = torch.device(device)
        if arena is None:
            arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.arena = arena
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self._L.mithra_init_grid(C.byref(self._g), C.c_void_p(arena.data_ptr()),
                                      C.c_size_t(arena.numel()), C.c_void_p(self.stream.cuda_stream),
                                      C.byref(h))
        self._h = h
        if rc != 0:
            msg = self.last_error()
            self.close()
            raise MithraError(rc, msg)

    # -- lifecycle --
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._L.mithra_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self._L.mithra_last_error(self._h).decode()

    def _check(self, rc: int):
        if rc != 0:
            raise MithraError(rc, self.last_error())

    # -- the six calls --
    def load_bunch(self, xyz: np.ndarray, u: np.ndarray, q_macro: float):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        self._check(self._L.mithra_load_bunch(self._h, xyz.shape[0], _dp(xyz), _dp(u), float(q_macro)))
        self.np = xyz.shape[0]

    def step(self, n: int = 1):
        self._check(self._L.mithra_step(self._h, int(n)))

    def read_field(self, name: str, dtype=np.float64) -> np.ndarray:
        dt = 1 if np.dtype(dtype) == np.float64 else 0
        out = np.empty(self.shape, dtype=np.float64 if dt else np.float32)
        self._check(self._L.mithra_read_fields(self._h, FIELD_IDS[name], dt,
                                               out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def read_particles(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        n = self.np
        xyz = np.empty((n, 3))
        u = np.empty((n, 3))
        cell = np.empty(n, dtype=np.int32)
        perm = np.empty(n, dtype=np.int32)
        self._check(self._L.mithra_read_particles(self._h, _dp(xyz), _dp(u),
                                                  cell.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  perm.ctypes.data_as(C.POINTER(C.c_int32))))
        return xyz, u, cell, perm

    def radiated_power(self, k: Optional[int] = None) -> float:
        k = int(self.desc["k_plane"]) if k is None else int(k)
        out = C.c_double()
        self._check(self._L.mithra_radiated_power(self._h, k, C.byref(out)))
        return out.value

    # -- extras --
    def power_history(self, n: int) -> np.ndarray:
        out = np.zeros(n)
        m = self._L.mithra_power_history(self._h, _dp(out), n)
        if m < 0:
            self._check(int(m))
        return out[:m]

    def bunching(self) -> float:
        out = C.c_double()
        self._check(self._L.mithra_bunching(self._h, C.byref(out)))
        return out.value

    def spectral_power(self) -> np.ndarray:
        """dW/domega at the descriptor's normalised frequencies (J s)."""
        n = int(self.desc.get("n_freq", 0))
        out = np.zeros(max(n, 1))
        m = self._L.mithra_spectral_power(self._h, _dp(out), n)
        if m < 0:
            self._check(int(m))
        return out[:m]

    def set_undulator(self, params: dict):
        """Undulator arrays / tapering / optical pulse (mithra_undulator_desc keys)."""
        p = dict(params)
        p.setdefault("n_modules", 1)
        s = _fill(UndulatorDesc, p)
        self._check(self._L.mithra_set_undulator(self._h, C.byref(s)))

    def set_seed(self, params: dict):
        """TF/SF seed (mithra_seed_desc keys)."""
        s = _fill(SeedDesc, params)
        self._check(self._L.mithra_set_seed(self._h, C.byref(s)))

    def generate_bunch(self, params: dict, n: int, q_macro: float):
        """Halton bunch generated and loaded on the device (mithra_bunch_desc keys)."""
        s = _fill(BunchDesc, params)
        self._check(self._L.mithra_generate_bunch(self._h, C.byref(s), int(n), float(q_macro)))
        self.np = int(n)

    def constants(self) -> dict:
        out = np.zeros(8)
        self._check(self._L.mithra_constants(self._h, _dp(out)))
        return dict(zip(["gamma0", "beta0", "dt", "dtb", "A", "q", "steps", "np"], out.tolist()))

    def set_sweep_shape(self, shape: int):
        self._check(self._L.mithra_set_sweep_shape(self._h, int(shape)))

    def time_sweep(self, shape: int = -1, iters: int = 20) -> float:
        """Average ms of one field-sweep launch (tile shape `shape`, -1: current)."""
        out = C.c_double()
        self._check(self._L.mithra_time_sweep(self._h, int(shape), int(iters), C.byref(out)))
        return out.value

    def step_timed(self, n: int) -> Tuple[float, float]:
        """n steps with HIP events around each sweep and each step:
        returns (summed sweep ms, summed step ms)."""
        a, b = C.c_double(0.0), C.c_double(0.0)
        self._check(self._L.mithra_step_timed(self._h, int(n), C.byref(a), C.byref(b)))
        return a.value, b.value

    STAGES = ("sweep", "mur", "vertex", "push", "sort", "tail", "step")

    def step_profile(self, n: int) -> dict:
        """n steps with HIP events between the stages of every step: summed
        ms per stage (sweep, mur, vertex, push, sort, tail) and per step."""
        out = np.zeros(7)
        self._check(self._L.mithra_step_profile(self._h, int(n), _dp(out)))
        return dict(zip(self.STAGES, out.tolist()))

    def autotune_sweep(self, iters: int = 10) -> int:
        """Time every sweep tile shape on this run's grid, keep the fastest."""
        out = C.c_int(-1)
        self._check(self._L.mithra_autotune_sweep(self._h, int(iters), C.byref(out)))
        return out.value

    @staticmethod
    def sweep_shape_count() -> int:
        return int(lib().mithra_sweep_shape_count())


class Batch:
    """Several loaded runs stepped together by grouped launches (one graph
    per batched step).  Members keep their own read calls; they cannot be
    stepped alone while the batch exists."""

    def __init__(self, engines, stream=None):
        import torch
        self._L = lib()
        self.engines = list(engines)
        n = len(self.engines)
        if n == 0:
            raise ValueError("empty batch")
        dev = self.engines[0].device
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        nbytes = int(self._L.mithra_batch_workspace_bytes(n))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        hs = (C.c_void_p * n)(*[e._h.value for e in self.engines])
        b = C.c_void_p()
        rc = self._L.mithra_batch_create(hs, n, C.c_void_p(self.workspace.data_ptr()), C.c_size_t(nbytes),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(b))
        if rc != 0:
            raise MithraError(rc, "batch creation failed")
        self._b = b

    def last_error(self) -> str:
        return self._L.mithra_batch_last_error(self._b).decode()

    def _check(self, rc: int):
        if rc != 0:
            raise MithraError(rc, self.last_error())

    def run(self, steps):
        """Advance member i by steps[i] (an int applies to every member)."""
        n = len(self.engines)
        if isinstance(steps, (int, np.integer)):
            steps = [int(steps)] * n
        arr = (C.c_int64 * n)(*[int(x) for x in steps])
        self._check(self._L.mithra_batch_run(self._b, arr))

    def autotune_sweep(self, iters: int = 3):
        """Choose the members' sweep tile shapes by timing grouped launches
        with the whole batch on the device; returns each member's shape."""
        n = len(self.engines)
        out = (C.c_int32 * n)()
        self._check(self._L.mithra_batch_autotune_sweep(self._b, int(iters), out))
        return [int(x) for x in out]

    def sync(self):
        self._check(self._L.mithra_batch_sync(self._b))

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            self._L.mithra_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
