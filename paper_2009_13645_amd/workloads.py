"""Seeded synthetic workloads for the boosted-frame FEL PIC step.

This module is shared by the tests, the benchmark and the CPU oracle's
callers.  It only *draws inputs*: grid geometry, a bunch of macro-electrons
and the run descriptor fields.  It contains none of the field solver, pusher
or deposit arithmetic, and it imports nothing else from this package.

Recipe (MITHRA 2.0 manual, ch. 3 "Quantity Initialization" and ch. 5
"Examples"; all sizes are the synthetic stand-ins described in the design
notes):

* The simulation runs in the bunch rest frame moving at beta0 along z.  The
  reference Lorentz factor of that frame is gamma0 = gamma / sqrt(1 + K^2/2)
  for a planar undulator (sec. "Lorentz Transformation") and
  gamma / sqrt(1 + K^2) for a helical one (reading, textbook resonance).
* The boosted undulator wavelength is lambda* = lambda_u / (gamma0 beta0);
  the grid uses dz = lambda*/16 and dx = dy = 4 dz, so that the NSFD
  condition (dz/dx)^2 + (dz/dy)^2 < 1 holds with margin.
* Bunches are drawn directly in the boosted frame at the common boosted time
  of the first half step.  Positions are drawn in cells (Gaussian or
  flat-top with half-Gaussian tapers one lambda* wide); the longitudinal
  momentum is the exact 4-velocity boost u_z = gamma0 (u'_z - beta0 gamma')
  of a lab-frame energy drawn from N(gamma, sigma_gamma); transverse momenta
  are zero (zero emittance).
* The undulator entrance sits 2 lab periods (2 lambda_u / gamma0 in the
  boosted frame) ahead of the bunch head at t = 0 (sec. "UNDULATOR",
  distance-to-bunch-head default).
* Random numbers: numpy PCG64 with an explicit seed per workload.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# SI constants (CODATA 2018), kept local to this module.
C_LIGHT = 299792458.0
Q_E = 1.602176634e-19
M_E = 9.1093837015e-31
EPS_0 = 8.8541878128e-12
I_ALFVEN = 4.0 * math.pi * EPS_0 * M_E * C_LIGHT ** 3 / Q_E  # ~17045 A

PLANAR = 0
HELICAL = 1


@dataclasses.dataclass
class Workload:
    """One synthetic run: grid, undulator, bunch recipe and run length."""

    name: str
    nx: int
    ny: int
    nz: int
    gamma: float
    K: float
    lambda_u: float
    n_periods: int
    und_type: int = PLANAR
    pol_angle_deg: float = 0.0
    cells_per_wavelength: float = 16.0
    transverse_ratio: float = 4.0  # dx/dz = dy/dz
    truncation_order: int = 2
    space_charge: int = 1
    n_sub: int = 1
    field_precision: int = 64  # 32 or 64
    compensated: int = 0
    steps: int = 200
    n_particles: int = 4096
    charge_C: float = 1e-12
    bunch: str = "gaussian"  # "gaussian" | "flattop"
    sigma_cells: Tuple[float, float, float] = (2.0, 2.0, 2.0)
    flat_len_cells: float = 0.0
    center_frac_z: float = 0.4
    sigma_gamma_rel: float = 1e-4
    shot_noise: bool = False
    seed: int = 1
    tile: Tuple[int, int, int] = (8, 8, 8)
    sort_every: int = 1  # sort after every sort_every-th push
    k_plane: int = -1  # radiated-power plane (node index), -1: 3/4 of nz

    # ---- derived geometry (recipe only) ----
    @property
    def gamma0(self) -> float:
        if self.und_type == HELICAL:
            return self.gamma / math.sqrt(1.0 + self.K ** 2)
        return self.gamma / math.sqrt(1.0 + 0.5 * self.K ** 2)

    @property
    def beta0(self) -> float:
        g0 = self.gamma0
        return math.sqrt(1.0 - 1.0 / (g0 * g0))

    @property
    def lambda_star(self) -> float:
        return self.lambda_u / (self.gamma0 * self.beta0)

    @property
    def dz(self) -> float:
        return self.lambda_star / self.cells_per_wavelength

    @property
    def dx(self) -> float:
        return self.transverse_ratio * self.dz

    @property
    def dy(self) -> float:
        return self.transverse_ratio * self.dz

    @property
    def origin(self) -> Tuple[float, float, float]:
        """Coordinates of node (0,0,0): x and y centred on the axis, z from 0."""
        return (-0.5 * (self.nx - 1) * self.dx, -0.5 * (self.ny - 1) * self.dy, 0.0)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def center_z_cells(self) -> float:
        return self.center_frac_z * (self.nz - 1)

    @property
    def head_z_cells(self) -> float:
        sz = self.sigma_cells[2]
        if self.bunch == "flattop":
            return self.center_z_cells + 0.5 * self.flat_len_cells + 3.0 * self.cells_per_wavelength
        return self.center_z_cells + 4.0 * sz

    @property
    def tail_z_cells(self) -> float:
        sz = self.sigma_cells[2]
        if self.bunch == "flattop":
            return self.center_z_cells - 0.5 * self.flat_len_cells - 3.0 * self.cells_per_wavelength
        return self.center_z_cells - 4.0 * sz

    def steps_bunch_inside(self) -> int:
        """NSFD steps (dt = dz/c) after which the undulator entrance, moving
        at -beta0 c, lies two boosted periods behind the bunch tail.  Taking
        the particles at rest makes it an upper bound on the steps until the
        whole bunch is inside the undulator (they drift forward until they
        enter)."""
        z_tail = self.origin[2] + self.tail_z_cells * self.dz
        dist = self.z_entrance - z_tail + 2.0 * self.lambda_u / self.gamma0
        return int(math.ceil(dist / (self.beta0 * self.dz)))

    @property
    def z_entrance(self) -> float:
        """Boosted-frame z of the undulator entrance at t = 0 (metres)."""
        z_head = self.origin[2] + self.head_z_cells * self.dz
        return z_head + 2.0 * self.lambda_u / self.gamma0

    @property
    def plane_k(self) -> int:
        return self.k_plane if self.k_plane >= 0 else int(0.75 * (self.nz - 1))

    def descriptor(self) -> dict:
        """Plain run descriptor (SI, boosted-frame mesh) handed to both sides."""
        x0, y0, z0 = self.origin
        return dict(
            nx=self.nx, ny=self.ny, nz=self.nz,
            dx=self.dx, dy=self.dy, dz=self.dz,
            x0=x0, y0=y0, z0=z0,
            truncation_order=self.truncation_order,
            space_charge=self.space_charge,
            solver=0,
            n_sub=self.n_sub,
            field_precision=self.field_precision,
            compensated=self.compensated,
            gamma=self.gamma,
            und_type=self.und_type,
            K=self.K,
            lambda_u=self.lambda_u,
            n_periods=self.n_periods,
            pol_angle_deg=self.pol_angle_deg,
            z_entrance=self.z_entrance,
            tile=tuple(self.tile),
            k_plane=self.plane_k,
            sort_every=self.sort_every,
        )

    def footprint_guess_bytes(self) -> int:
        """Rough device bytes (fields + particles), used only for sizing tests."""
        pf = 4 if self.field_precision == 32 else 8
        return self.n_nodes * pf * (3 * 4 + 2 * 4 + 6) + self.n_particles * 120


# ---------------------------------------------------------------------------
# Bunch generation
# ---------------------------------------------------------------------------

def _boost_uz(gamma_lab: np.ndarray, gamma0: float, beta0: float) -> np.ndarray:
    """Exact 4-velocity boost along z of a purely longitudinal lab momentum."""
    uz_lab = np.sqrt(gamma_lab * gamma_lab - 1.0)
    return gamma0 * (uz_lab - beta0 * gamma_lab)


def _flattop_z(rng: np.random.Generator, n: int, length: float, taper_sigma: float) -> np.ndarray:
    """Uniform profile of `length` with half-Gaussian tapers of rms `taper_sigma`.

    The tapers hold the particle count a Gaussian of the same peak density
    would put in each half, so the density is continuous at the joins.
    """
    w_taper = taper_sigma * math.sqrt(2.0 * math.pi)  # equivalent length of both halves
    frac_flat = length / (length + w_taper)
    n_flat = int(round(n * frac_flat))
    n_tap = n - n_flat
    z_flat = (rng.random(n_flat) - 0.5) * length
    g = np.abs(rng.standard_normal(n_tap))
    side = np.where(rng.random(n_tap) < 0.5, -1.0, 1.0)
    z_tap = side * (0.5 * length + taper_sigma * g)
    z = np.concatenate([z_flat, z_tap])
    return z[rng.permutation(n)]


def fel_rho_1d(gamma: float, K: float, lambda_u: float, n_e: float, helical: bool) -> float:
    """1-D FEL parameter from the lab-frame electron density (used for sizing).

    rho = (1 / 2 gamma) * (K_JJ * omega_p / (4 c k_u))^(2/3), with
    K_JJ = K [JJ] for a planar and K for a helical undulator.  With the
    numbers of the manual's infrared example (51.4 MeV, K = 1.4,
    lambda_u = 3 cm, 2.72e13 cm^-3) this gives 0.0063, against the printed
    0.006.
    """
    ku = 2.0 * math.pi / lambda_u
    wp = math.sqrt(n_e * Q_E * Q_E / (EPS_0 * M_E))
    if helical:
        kjj = K
    else:
        xi = K * K / (4.0 + 2.0 * K * K)
        from scipy.special import j0, j1  # scipy is available in this image
        kjj = K * (j0(xi) - j1(xi))
    return (1.0 / (2.0 * gamma)) * (kjj * wp / (4.0 * C_LIGHT * ku)) ** (2.0 / 3.0)


def xie_estimate(gamma: float, K: float, lambda_u: float, charge: float, box_lab, sigma_gamma_rel: float,
                 transverse: str = "box") -> dict:
    """3-D gain length and saturation power of a planar-undulator FEL with a
    zero-emittance beam, uniform over its lab length box_lab[2] and either
    uniform over a transverse box (transverse="box") or Gaussian with rms
    box_lab[0], box_lab[1] across (transverse="gaussian", on-axis density),
    from M. Xie's fitting formula
    (Proc. PAC 1995): L_G = L_G1D (1 + Lambda(eta_d, eta_eps, eta_gamma)),
    with the 1-D parameter rho = (1/gamma) (a_w [JJ] omega_p / (4 c k_u))^(2/3),
    a_w = K / sqrt(2), L_G1D = lambda_u / (4 pi sqrt(3) rho), the rms beam
    size (a box's width / sqrt(12)) in eta_d = L_G1D / (2 k_r sigma^2),
    eta_eps = 0, eta_gamma = 4 pi (L_G1D / lambda_u) sigma_gamma, and
    P_sat = 1.6 rho P_beam (L_G1D / L_G)^2.  An estimate for sizing and for
    comparison, not part of the method."""
    from scipy.special import j0, j1
    ku = 2.0 * math.pi / lambda_u
    if transverse == "gaussian":
        n_e = charge / Q_E / (2.0 * math.pi * box_lab[0] * box_lab[1] * box_lab[2])
    else:
        n_e = charge / Q_E / (box_lab[0] * box_lab[1] * box_lab[2])
    wp = math.sqrt(n_e * Q_E * Q_E / (EPS_0 * M_E))
    xi = K * K / (4.0 + 2.0 * K * K)
    jj = j0(xi) - j1(xi)
    rho = (1.0 / gamma) * ((K / math.sqrt(2.0)) * jj * wp / (4.0 * C_LIGHT * ku)) ** (2.0 / 3.0)
    lg1 = lambda_u / (4.0 * math.pi * math.sqrt(3.0) * rho)
    lam_r = lambda_u * (1.0 + 0.5 * K * K) / (2.0 * gamma * gamma)
    kr = 2.0 * math.pi / lam_r
    sig = math.sqrt(box_lab[0] * box_lab[1] / (1.0 if transverse == "gaussian" else 12.0))
    eta_d = lg1 / (2.0 * kr * sig * sig)
    eta_g = 4.0 * math.pi * (lg1 / lambda_u) * sigma_gamma_rel
    lam = 0.45 * eta_d ** 0.57 + 3.0 * eta_g ** 2 + 51.0 * eta_d ** 0.95 * eta_g ** 3
    lg3 = lg1 * (1.0 + lam)
    p_beam = gamma * M_E * C_LIGHT ** 3 * charge / Q_E / box_lab[2]
    return {"rho_1d": rho, "gain_length_1d_m": lg1, "eta_d": eta_d, "eta_gamma": eta_g,
            "gain_length_3d_m": lg3, "p_beam_W": p_beam, "p_sat_3d_W": 1.6 * rho * p_beam * (lg1 / lg3) ** 2}


def make_bunch(w: Workload, n: Optional[int] = None, seed: Optional[int] = None
               ) -> Tuple[np.ndarray, np.ndarray, float]:
    """Draw the bunch of workload `w`.

    Returns (xyz[n,3] metres, u[n,3] = gamma*beta, q_macro coulomb).  The
    positions are boosted-frame positions at the first half step; the
    momenta are boosted-frame u at field time 0.
    """
    n = w.n_particles if n is None else n
    rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
    x0, y0, z0 = w.origin
    sx, sy, sz = w.sigma_cells
    cx = 0.5 * (w.nx - 1)
    cy = 0.5 * (w.ny - 1)
    cz = w.center_z_cells

    def trunc_normal(size, lim=4.0):
        out = rng.standard_normal(size)
        bad = np.abs(out) > lim
        while bad.any():
            out[bad] = rng.standard_normal(int(bad.sum()))
            bad = np.abs(out) > lim
        return out

    xc = cx + sx * trunc_normal(n)
    yc = cy + sy * trunc_normal(n)
    if w.bunch == "flattop":
        zc = cz + _flattop_z(rng, n, w.flat_len_cells, w.cells_per_wavelength)
    else:
        zc = cz + sz * trunc_normal(n)

    g0, b0 = w.gamma0, w.beta0
    if w.shot_noise:
        # Shot-noise reading: slices one pre-entry wavelength long, slice
        # bunching b_j = sqrt(-2 ln x_j) / sqrt(N_e,slice), phase U[0, 2pi),
        # dz = (2 b_j / k) sin(k z + phi_j).  The pre-entry wavenumber is the
        # boosted resonant one scaled by the entry compression
        # beta0 / (beta_rel + beta0).
        g = w.gamma
        beta_rel = (g * g - g0 * g0) / (g * g + g0 * g0)
        k_cells = (2.0 * math.pi / w.cells_per_wavelength) * b0 / (beta_rel + b0)
        slice_len = 2.0 * math.pi / k_cells
        n_e_total = abs(w.charge_C) / Q_E
        zmin = zc.min()
        sl = np.floor((zc - zmin) / slice_len).astype(np.int64)
        nslices = int(sl.max()) + 1
        counts = np.bincount(sl, minlength=nslices).astype(np.float64)
        n_e_slice = np.maximum(counts * (n_e_total / n), 1.0)
        xs = rng.random(nslices)
        xs = np.where(xs <= 0.0, 1e-300, xs)
        bj = np.sqrt(-2.0 * np.log(xs)) / np.sqrt(n_e_slice)
        phij = 2.0 * math.pi * rng.random(nslices)
        zc = zc + (2.0 * bj[sl] / k_cells) * np.sin(k_cells * zc + phij[sl])

    gam = w.gamma * (1.0 + w.sigma_gamma_rel * trunc_normal(n))
    uz = _boost_uz(gam, g0, b0)

    xyz = np.empty((n, 3), dtype=np.float64)
    xyz[:, 0] = x0 + xc * w.dx
    xyz[:, 1] = y0 + yc * w.dy
    xyz[:, 2] = z0 + zc * w.dz
    u = np.zeros((n, 3), dtype=np.float64)
    u[:, 2] = uz
    q_macro = -abs(w.charge_C) / n
    return xyz, u, q_macro


# ---------------------------------------------------------------------------
# The five configurations
# ---------------------------------------------------------------------------

def config1() -> Workload:
    """Tiny undulator-radiation run: 32x32x64 nodes, 4096 e-, 200 steps, FP64."""
    return Workload(name="cfg1-tiny-undulator-32x32x64", nx=32, ny=32, nz=64,
                    gamma=100.0, K=1.0, lambda_u=0.03, n_periods=40,
                    und_type=PLANAR, steps=200, n_particles=4096,
                    charge_C=1e-12, bunch="gaussian", sigma_cells=(2.0, 2.0, 2.0),
                    sigma_gamma_rel=1e-4, seed=1, field_precision=64,
                    tile=(8, 8, 8))


def _cfg2_charge(w: Workload, rho_target: float = 3e-3) -> float:
    """Bunch charge giving rho_FEL ~ rho_target for the cfg2 geometry."""
    # lab-frame density of the flat-top core: transverse Gaussian sigma,
    # lab length = boosted length * gamma_rel / gamma.
    g, g0 = w.gamma, w.gamma0
    beta_rel = (g * g - g0 * g0) / (g * g + g0 * g0)
    gam_rel = 1.0 / math.sqrt(1.0 - beta_rel ** 2)
    l_lab = w.flat_len_cells * w.dz * gam_rel / g
    sig = w.sigma_cells[0] * w.dx
    # invert rho(n) ~ n^(1/3): rho(n) = rho(1) * n^(1/3)
    r1 = fel_rho_1d(g, w.K, w.lambda_u, 1.0, helical=(w.und_type == HELICAL))
    n_e = (rho_target / r1) ** 3
    n_tot = n_e * 2.0 * math.pi * sig * sig * l_lab
    return n_tot * Q_E


def config2(field_precision: int = 32, compensated: int = 0, steps: int = 4000) -> Workload:
    """FEL amplifier: 128x128x1024 nodes, 2^21 e-, helical K=1.4, gamma=200."""
    w = Workload(name="cfg2-fel-amplifier-128x128x1024", nx=128, ny=128, nz=1024,
                 gamma=200.0, K=1.4, lambda_u=0.03, n_periods=400,
                 und_type=HELICAL, steps=steps, n_particles=2 ** 21,
                 bunch="flattop", sigma_cells=(8.0, 8.0, 0.0), flat_len_cells=512.0,
                 center_frac_z=0.4, sigma_gamma_rel=1e-4, shot_noise=True, seed=2,
                 field_precision=field_precision, compensated=compensated,
                 tile=(4, 2, 2))
    w.charge_C = _cfg2_charge(w)
    return w


def config2_small(field_precision: int = 32, compensated: int = 0) -> Workload:
    """Reduced FEL-amplifier geometry (same physics recipe) for oracle parity."""
    w = Workload(name="cfg2-small-48x48x160", nx=48, ny=48, nz=160,
                 gamma=200.0, K=1.4, lambda_u=0.03, n_periods=400,
                 und_type=HELICAL, steps=200, n_particles=20000,
                 bunch="flattop", sigma_cells=(3.0, 3.0, 0.0), flat_len_cells=48.0,
                 center_frac_z=0.4, sigma_gamma_rel=1e-4, shot_noise=True, seed=2,
                 field_precision=field_precision, compensated=compensated,
                 tile=(8, 8, 8))
    w.charge_C = 5e-12
    return w


def config4_runs(n_runs: int = 64, base_seed: int = 4000, steps_cap: Optional[int] = None,
                 scale: float = 1.0) -> List[Workload]:
    """Batched scan: independent undulator-radiation runs of uneven size.

    n_x, n_y ~ U{32, 40, ..., 96}, n_z ~ U{32, 40, ..., 256},
    N_p ~ U[1e4, 5e5], gamma ~ U[50, 300], K ~ U[0.5, 2.0], planar,
    40 periods, Gaussian sigma = (n_x/16, n_y/16, n_z/32) cells, precision
    FP64-all or FP32 fields with probability 1/2, steps ~ U{500, ..., 3000};
    particles sorted after every 16th push.
    `scale` < 1 shrinks particle counts (used by CPU-side tests).
    """
    runs = []
    for r in range(n_runs):
        rng = np.random.Generator(np.random.PCG64(base_seed + r))
        nx = int(rng.choice(np.arange(32, 97, 8)))
        ny = int(rng.choice(np.arange(32, 97, 8)))
        nz = int(rng.choice(np.arange(32, 257, 8)))
        npart = int(rng.integers(10_000, 500_001))
        gamma = float(rng.uniform(50.0, 300.0))
        K = float(rng.uniform(0.5, 2.0))
        prec = 32 if rng.random() < 0.5 else 64
        steps = int(rng.integers(500, 3001))
        if steps_cap is not None:
            steps = min(steps, steps_cap)
        npart = max(64, int(npart * scale))
        w = Workload(name=f"cfg4-run{r:02d}-{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                     gamma=gamma, K=K, lambda_u=0.03, n_periods=40, und_type=PLANAR,
                     steps=steps, n_particles=npart, charge_C=1e-12,
                     bunch="gaussian", sigma_cells=(nx / 16.0, ny / 16.0, nz / 32.0),
                     sigma_gamma_rel=1e-4, seed=base_seed + r, field_precision=prec,
                     tile=(8, 8, 8), sort_every=16)
        runs.append(w)
    return runs


def config5_requests(n_req: int = 1000, rate_hz: float = 20.0, seed: int = 5,
                     steps_cap: Optional[int] = None, scale: float = 1.0
                     ) -> List[Tuple[float, Workload]]:
    """Served stream: Poisson arrivals (rate 20/s) of config-4-like runs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)
    t = np.cumsum(gaps)
    out = []
    for r in range(n_req):
        w = config4_runs(1, base_seed=5000 + r, steps_cap=steps_cap, scale=scale)[0]
        w.name = f"cfg5-req{r:04d}-{w.nx}x{w.ny}x{w.nz}"
        out.append((float(t[r]), w))
    return out


# ---------------------------------------------------------------------------
# The manual's Example 1 (ch. 5 "Example 1: Infrared FEL", table example1,
# and its job file): the run description and the bunch description.
# ---------------------------------------------------------------------------

EX1_GAMMA = 100.41            # 51.4 MeV
EX1_K = 1.417                 # undulator-parameter of the job file
EX1_LAMBDA_U = 0.03           # 3 cm
EX1_CHARGE_C = 29.5e-12       # 29.5 pC (1.846e8 electrons)
EX1_PARTICLES = 131072
EX1_BUNCH_LAB = (260e-6, 260e-6, 100.5e-6)   # sigma-position: rms 260 um across (Gaussian), 100.5 um long (lab)
EX1_MESH_LAB = (50e-6, 50e-6, 0.1e-6)        # mesh-resolution (lab)
EX1_MESH_LENGTHS_LAB = (3200e-6, 3200e-6, 280e-6)  # mesh-lengths (lab)
EX1_NODES = (64, 64, 2800)                   # mesh-lengths / mesh-resolution
EX1_PLANE_LAB = 110e-6                       # power plane ahead of the bunch centre (lab)
EX1_BUNCH_STEP_LAB = 1.6e-12                 # bunch-time-step (lab)


def example1(solver: int = 0, field_precision: int = 64, plane_lab: float = EX1_PLANE_LAB,
             mesh_lab=EX1_MESH_LAB, lengths_lab=EX1_MESH_LENGTHS_LAB,
             n_particles: int = EX1_PARTICLES, transverse: str = "gaussian") -> Tuple[dict, dict, int, float]:
    """Example 1 in the boosted frame: the run descriptor, the device bunch
    description (Halton quiet start, flat-top with tapers, Gaussian rms
    260 um across, bunching factor 0.01, no shot noise), the particle count
    and the macro-particle charge.

    Lab lengths along z become boosted lengths times gamma0 (a mesh at rest
    in the bunch frame); the transverse ones are unchanged.  The bunch centre
    sits at the middle of the mesh, the undulator entrance two lab periods
    ahead of the bunch head (distance-to-bunch-head default), the power
    plane plane_lab (lab) ahead of the bunch centre.  Space charge off, Mur
    second order, NSFD (or FD), as in the job file.  The bunch step of the
    job file (1.6 ps lab) is turned into the sub-step count by the mesh
    auto-adjustment (mithra_adapt_mesh).  mesh_lab, lengths_lab and
    n_particles vary the job's mesh-resolution, mesh-lengths and
    number-of-particles (the manual's convergence study); node counts are
    lengths over resolution.  transverse: "gaussian" (the job file: MITHRA's
    transverse profiles are always Gaussian, sigma-position their rms) or
    "box" (the uniform 260 x 260 um box that the table's electron density
    corresponds to).
    """
    g0 = EX1_GAMMA / math.sqrt(1.0 + 0.5 * EX1_K ** 2)
    b0 = math.sqrt(1.0 - 1.0 / (g0 * g0))
    nx, ny, nz = (int(round(lengths_lab[a] / mesh_lab[a])) for a in range(3))
    dx, dy = mesh_lab[0], mesh_lab[1]
    dz = g0 * mesh_lab[2]
    beta = math.sqrt(1.0 - 1.0 / (EX1_GAMMA ** 2))
    lz = 1.0 / (g0 * (1.0 - beta * b0))
    zc = 0.5 * (nz - 1) * dz
    kr = 2.0 * math.pi * g0 * b0 / EX1_LAMBDA_U
    lam_lab = (2.0 * math.pi / kr) / (g0 * (1.0 + b0))
    half = 0.5 * EX1_BUNCH_LAB[2] * lz + 3.0 * lam_lab * lz  # flat top plus the taper tails
    z_head = zc + half
    desc = dict(nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz,
                x0=-0.5 * (nx - 1) * dx, y0=-0.5 * (ny - 1) * dy, z0=0.0,
                truncation_order=2, space_charge=0, solver=solver, n_sub=1,
                field_precision=field_precision, compensated=0, gamma=EX1_GAMMA, und_type=PLANAR,
                K=EX1_K, lambda_u=EX1_LAMBDA_U, n_periods=300, pol_angle_deg=0.0,
                z_entrance=z_head + 2.0 * EX1_LAMBDA_U / g0, tile=(4, 4, 4),
                k_plane=int(round((zc + g0 * plane_lab) / dz)), n_freq=1, nu_min=1.0, nu_max=1.0)
    if transverse not in ("gaussian", "box"):
        raise ValueError("transverse must be 'gaussian' or 'box'")
    bunch = dict(long_profile=0, trans_profile=1 if transverse == "gaussian" else 0, shot_noise=0, tapers=1,
                 center=(0.0, 0.0, zc),
                 size=EX1_BUNCH_LAB, gamma=EX1_GAMMA, sigma_gamma_rel=1e-4, sigma_u_perp=0.0,
                 bunching=0.01, bunching_phase=0.0, n_electrons=EX1_CHARGE_C / Q_E)
    return desc, bunch, n_particles, -EX1_CHARGE_C / n_particles
