"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this module.  It loads `libmithra_oracle.so`, built from `mithra_oracle.c`
by `build_oracle()`, and shares nothing with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mithra_oracle.c")
LIB = os.environ.get("MITHRA_ORACLE_LIB") or os.path.join(HERE, "libmithra_oracle.so")

FIELD_IDS = {"Ex": 0, "Ey": 1, "Ez": 2, "Bx": 3, "By": 4, "Bz": 5, "Ax": 6, "Ay": 7,
             "Az": 8, "Jx": 9, "Jy": 10, "Jz": 11, "F": 12, "Q": 13}


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-std=c99", "-D_DEFAULT_SOURCE", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("truncation_order", C.c_int32), ("space_charge", C.c_int32),
                ("solver", C.c_int32), ("n_sub", C.c_int32), ("und_type", C.c_int32),
                ("n_periods", C.c_int32), ("k_plane", C.c_int32),
                ("tile", C.c_int32 * 3), ("sort_every", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("gamma", C.c_double), ("K", C.c_double), ("lambda_u", C.c_double),
                ("pol_angle_deg", C.c_double), ("z_entrance", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.ora_create.restype = P
        L.ora_create.argtypes = [C.POINTER(_Desc)]
        L.ora_destroy.argtypes = [P]
        L.ora_consts.argtypes = [P, dp]
        L.ora_load_bunch.argtypes = [P, C.c_int64, dp, dp, C.c_double]
        L.ora_load_bunch.restype = C.c_int
        L.ora_step.argtypes = [P, C.c_int64]
        L.ora_field_step.argtypes = [P, C.c_int64]
        L.ora_set_potential.argtypes = [P, C.c_int, C.c_int, dp]
        L.ora_get_potential.argtypes = [P, C.c_int, C.c_int, dp]
        L.ora_get_field.argtypes = [P, C.c_int, dp]
        L.ora_get_field.restype = C.c_int
        L.ora_get_particles.argtypes = [P, dp, dp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.ora_get_keys.argtypes = [P, C.POINTER(C.c_uint32)]
        L.ora_gather.argtypes = [P, dp, dp, dp]
        L.ora_external_field.argtypes = [P, dp, C.c_double, dp, dp]
        L.ora_boris.argtypes = [dp, dp, dp, C.c_double, dp]
        L.ora_radiated_power.argtypes = [P, C.c_int]
        L.ora_radiated_power.restype = C.c_double
        L.ora_bunching.argtypes = [P]
        L.ora_bunching.restype = C.c_double
        L.ora_threads.restype = C.c_int
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_set_generic_faces.argtypes = [P, C.c_int]
        L.ora_set_undulator.argtypes = [P, dp]
        L.ora_set_seed.argtypes = [P, dp]
        L.ora_seed_incident.argtypes = [P, C.c_int, dp, C.c_double]
        L.ora_seed_incident.restype = C.c_double
        L.ora_set_spectrum.argtypes = [P, C.c_int, C.c_double, C.c_double]
        L.ora_spectral_power.argtypes = [P, dp]
        L.ora_halton.argtypes = [C.c_int, C.c_uint64]
        L.ora_halton.restype = C.c_double
        L.ora_generate_bunch.argtypes = [P, dp, C.c_int64, dp, dp]
        L.ora_compute_fields.argtypes = [P]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def boris(u, E, B, dtb) -> np.ndarray:
    """One Boris momentum update (q = -e)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    out = np.zeros(3)
    lib().ora_boris(_dp(u), _dp(E), _dp(B), float(dtb), _dp(out))
    return out


def halton(i: int, j: int) -> float:
    """Element j of the i-th Halton sequence (1 - radical inverse, base prime i)."""
    return float(lib().ora_halton(int(i), int(j)))


UNDULATOR_KEYS = ("n_modules", "gap", "dK", "signal", "ctau", "ct0", "cep_deg", "w0_par", "w0_perp", "z_focus")
SEED_KEYS = ("type", "signal", "a0", "wavelength", "ctau", "ct0", "cep_deg", "pol_deg", "w0", "z_focus")
BUNCH_KEYS = ("long_profile", "trans_profile", "xc", "yc", "zc", "size_x", "size_y", "size_z", "gamma",
              "sigma_gamma_rel", "sigma_u_perp", "bunching", "bunching_phase", "shot_noise", "n_electrons",
              "tapers")


def _params(keys, d: dict) -> np.ndarray:
    return np.array([float(d.get(k, 0.0)) for k in keys], dtype=np.float64)


def threads() -> int:
    return int(lib().ora_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops for later calls."""
    lib().ora_set_threads(int(n))


class Oracle:
    """One oracle run.  `desc` is the plain dict from Workload.descriptor()."""

    CONST_NAMES = ["gamma0", "beta0", "dt", "dtb", "A", "a1", "a2", "a3", "a4", "a5",
                   "a6", "a7", "a8", "q", "np", "step"]

    def __init__(self, desc: dict):
        d = _Desc()
        for k in ("nx", "ny", "nz", "truncation_order", "space_charge", "solver", "n_sub",
                  "und_type", "n_periods", "k_plane"):
            setattr(d, k, int(desc[k]))
        for a in range(3):
            d.tile[a] = int(desc["tile"][a])
        d.sort_every = int(desc.get("sort_every", 1))
        for k in ("dx", "dy", "dz", "x0", "y0", "z0", "gamma", "K", "lambda_u",
                  "pol_angle_deg", "z_entrance"):
            setattr(d, k, float(desc[k]))
        self.desc = dict(desc)
        self.shape = (int(desc["nz"]), int(desc["ny"]), int(desc["nx"]))
        self._h = lib().ora_create(C.byref(d))
        self.np = 0

    def close(self):
        if self._h:
            lib().ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def consts(self) -> dict:
        out = np.zeros(16)
        lib().ora_consts(self._h, _dp(out))
        return dict(zip(self.CONST_NAMES, out.tolist()))

    def load_bunch(self, xyz: np.ndarray, u: np.ndarray, q: float):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        rc = lib().ora_load_bunch(self._h, xyz.shape[0], _dp(xyz), _dp(u), float(q))
        if rc != 0:
            raise ValueError("oracle rejected the bunch")
        self.np = xyz.shape[0]

    def step(self, n: int = 1):
        lib().ora_step(self._h, int(n))

    def field_step(self, n: int = 1):
        lib().ora_field_step(self._h, int(n))

    def set_potential(self, comp: int, level: int, arr: np.ndarray):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.shape)
        lib().ora_set_potential(self._h, comp, level, _dp(a))

    def potential(self, comp: int, level: int = 1) -> np.ndarray:
        out = np.zeros(self.shape)
        lib().ora_get_potential(self._h, comp, level, _dp(out))
        return out

    def field(self, name: str) -> np.ndarray:
        out = np.zeros(self.shape)
        rc = lib().ora_get_field(self._h, FIELD_IDS[name], _dp(out))
        if rc != 0:
            raise KeyError(name)
        return out

    def particles(self):
        n = self.np
        xyz = np.zeros((n, 3))
        u = np.zeros((n, 3))
        cell = np.zeros(n, dtype=np.int32)
        perm = np.zeros(n, dtype=np.int32)
        lib().ora_get_particles(self._h, _dp(xyz), _dp(u), cell.ctypes.data_as(C.POINTER(C.c_int32)),
                                perm.ctypes.data_as(C.POINTER(C.c_int32)))
        return xyz, u, cell, perm

    def keys(self) -> np.ndarray:
        k = np.zeros(self.np, dtype=np.uint32)
        lib().ora_get_keys(self._h, k.ctypes.data_as(C.POINTER(C.c_uint32)))
        return k

    def gather(self, r) -> tuple:
        r = np.ascontiguousarray(r, dtype=np.float64)
        E = np.zeros(3)
        B = np.zeros(3)
        lib().ora_gather(self._h, _dp(r), _dp(E), _dp(B))
        return E, B

    def external_field(self, r, t: float) -> tuple:
        r = np.ascontiguousarray(r, dtype=np.float64)
        E = np.zeros(3)
        B = np.zeros(3)
        lib().ora_external_field(self._h, _dp(r), float(t), _dp(E), _dp(B))
        return E, B

    def radiated_power(self, k: Optional[int] = None) -> float:
        k = int(self.desc["k_plane"]) if k is None else int(k)
        return float(lib().ora_radiated_power(self._h, k))

    def bunching(self) -> float:
        return float(lib().ora_bunching(self._h))

    def compute_fields(self):
        lib().ora_compute_fields(self._h)

    def set_undulator(self, params: dict):
        """Undulator arrays (modules, gap, tapering) and optical-undulator
        pulse parameters; keys UNDULATOR_KEYS."""
        d = dict(params)
        d.setdefault("n_modules", 1)
        a = _params(UNDULATOR_KEYS, d)
        lib().ora_set_undulator(self._h, _dp(a))

    def set_seed(self, params: dict):
        """TF/SF seed wave; keys SEED_KEYS."""
        a = _params(SEED_KEYS, params)
        lib().ora_set_seed(self._h, _dp(a))

    def seed_incident(self, comp: int, r, t: float) -> float:
        r = np.ascontiguousarray(r, dtype=np.float64)
        return float(lib().ora_seed_incident(self._h, int(comp), _dp(r), float(t)))

    def set_spectrum(self, nf: int, nu_min: float, nu_max: float):
        lib().ora_set_spectrum(self._h, int(nf), float(nu_min), float(nu_max))
        self.nf = int(nf)

    def spectral_power(self) -> np.ndarray:
        out = np.zeros(max(getattr(self, "nf", 0), 1))
        lib().ora_spectral_power(self._h, _dp(out))
        return out[:getattr(self, "nf", 0)]

    def generate_bunch(self, params: dict, n: int):
        """Halton quiet-start bunch (keys BUNCH_KEYS): returns (xyz, u)."""
        a = _params(BUNCH_KEYS, params)
        xyz = np.zeros((n, 3))
        u = np.zeros((n, 3))
        lib().ora_generate_bunch(self._h, _dp(a), int(n), _dp(xyz), _dp(u))
        return xyz, u

    def set_generic_faces(self, on: bool):
        lib().ora_set_generic_faces(self._h, 1 if on else 0)
