"""Pins of the oracle's source coupling and of its undulator conventions.

The potentials' sources (mu0 J for A, rho / eps0 for phi) enter the NSFD
update only inside the oracle, so parity with the GPU cannot show whether
they are right.  These tests check them against physics the paper fixes:

* the discrete Lorenz gauge: with a charge-conserving deposit the gauge
  condition holds (sec. "Current Deposition": once the deposit conserves
  charge, the Lorenz condition is kept).  For the scheme as built, a
  smoothed form of (phi^{n+1/2} - phi^{n-1/2}) / dt + c^2 div A obeys the
  homogeneous NSFD wave equation exactly, so its discrete d'Alembertian is
  zero to round-off.  That fixes the factor, the sign and the edge average
  of the A source relative to the phi source, and the time level of rho;
* the retarded (Lienard-Wiechert) E and B of a few electrons computed from
  the oracle's own trajectories, which the grid fields must approach at
  second order in the mesh spacing;
* the stated conventions of the polarisation angle and of the helical
  handedness (both silent or ambiguous in the paper; see the design notes).
"""
import math

import numpy as np
import pytest
from scipy.ndimage import gaussian_filter1d

from oracle.oracle import Oracle

C = 299792458.0
QE = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12


def _desc(nx, ny, nz, dz, rx, ry, K=0.5, und_type=0, pol=0.0, z_entrance=-1e-3, origin=None):
    x0, y0, z0 = origin if origin is not None else (-0.5 * (nx - 1) * rx * dz, -0.5 * (ny - 1) * ry * dz, 0.0)
    return dict(nx=nx, ny=ny, nz=nz, dx=rx * dz, dy=ry * dz, dz=dz, x0=x0, y0=y0, z0=z0,
                truncation_order=2, space_charge=1, solver=0, n_sub=1, field_precision=64,
                compensated=0, gamma=100.0, und_type=und_type, K=K, lambda_u=0.03,
                n_periods=400, pol_angle_deg=pol, z_entrance=z_entrance, tile=(4, 4, 4),
                k_plane=nz // 2)


# ---------------------------------------------------------------------------
# Discrete Lorenz gauge
# ---------------------------------------------------------------------------

def _avg121(f, ax):
    """[1, 2, 1] / 4 node average along one array axis (periodic; only the
    interior is used)."""
    return 0.5 * f + 0.25 * (np.roll(f, 1, axis=ax) + np.roll(f, -1, axis=ax))


def _central(f, ax, h):
    return (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) / (2.0 * h)


def test_discrete_lorenz_gauge_is_kept_exactly():
    """With J on edges, J_bar = edge mean along l, and the deposit exactly
    charge conserving, define at each step n

        G^n = M (phi^{n+1/2} - phi^{n-1/2}) / dt + c^2 sum_l P_l D_l A_l^n,

    M = product of [1,2,1]/4 averages over the three axes, P_l = the product
    over the two axes other than l, D_l = central difference.  Because
    D_l(edge mean) = [1,2,1]/4 average of the edge difference, applying the
    update equation to every term gives
        G^{n+1} + G^{n-1} - (NSFD spatial operator) G^n
            = (c dt)^2 / eps0 * M [ (rho^{n+1/2} - rho^{n-1/2}) / dt + div_edge J^n ],
    which the continuity equation makes zero.  Every factor of the A source
    (mu0, its sign, the edge average) and the time level of rho enter this
    identity, which holds at interior nodes three or more from the faces."""
    nx, ny, nz = 20, 22, 26
    d = _desc(nx, ny, nz, 2.0e-5, 2.0, 1.5, K=0.5)
    o = Oracle(d)
    c = o.consts()
    dt = c["dt"]
    rng = np.random.default_rng(3)
    n = 6
    g = np.stack([rng.uniform(8, 12, n), rng.uniform(9, 13, n), rng.uniform(11, 15, n)], 1)
    xyz = np.stack([d["x0"] + g[:, 0] * d["dx"], d["y0"] + g[:, 1] * d["dy"], d["z0"] + g[:, 2] * d["dz"]], 1)
    u = rng.uniform(-0.4, 0.4, (n, 3))
    o.load_bunch(xyz, u, -QE)
    h = (d["dx"], d["dy"], d["dz"])
    ax_of = (2, 1, 0)  # array axis of x, y, z in [z][y][x]

    def M3(f):
        return _avg121(_avg121(_avg121(f, 0), 1), 2)

    def gauge():
        A = [o.potential(l, 1) for l in range(3)]
        dphi = (o.potential(3, 1) - o.potential(3, 0)) / dt  # (phi^{n+1/2} - phi^{n-1/2}) / dt
        G = M3(dphi)
        for l in range(3):
            t = _central(A[l], ax_of[l], h[l])
            for m in range(3):
                if m != l:
                    t = _avg121(t, ax_of[m])
            G = G + C * C * t
        return G, np.max(np.abs(M3(dphi)))

    a1, a2, a4, a6, Ac = c["a1"], c["a2"], c["a4"], c["a6"], c["A"]

    def nsfd_spatial(f):
        """a1 f + a2 (bar(x+) + bar(x-)) + a4 (bar(y+) + bar(y-)) + a6 (f(z+) + f(z-)),
        bar = z average A f(k-1) + (1 - 2A) f(k) + A f(k+1) (eq. updateEquation)."""
        def bar(sh, ax):
            s = np.roll(f, sh, ax)
            return Ac * np.roll(s, 1, 0) + (1 - 2 * Ac) * s + Ac * np.roll(s, -1, 0)
        return (a1 * f + a2 * (bar(1, 2) + bar(-1, 2)) + a4 * (bar(1, 1) + bar(-1, 1))
                + a6 * (np.roll(f, 1, 0) + np.roll(f, -1, 0)))

    Gs, scales = [], []
    for _ in range(12):
        G, s = gauge()
        Gs.append(G)
        scales.append(s)
        o.step(1)
    assert min(scales[1:]) > 0
    for k in range(1, 11):
        resid = Gs[k + 1] + Gs[k - 1] - nsfd_spatial(Gs[k])
        inner = resid[3:-3, 3:-3, 3:-3]
        # G itself is of the order of the scale (the charge appeared at t = 0)
        assert np.max(np.abs(Gs[k][3:-3, 3:-3, 3:-3])) > 0.1 * scales[k]
        assert np.max(np.abs(inner)) < 1e-12 * scales[k], (k, np.max(np.abs(inner)) / scales[k])
    # every particle stayed active (continuity then holds at every node used)
    assert np.all(o.particles()[2] >= 0)


# ---------------------------------------------------------------------------
# Lienard-Wiechert fields of the oracle's own trajectories
# ---------------------------------------------------------------------------

class _Trajectory:
    """Positions sampled every dt, interpolated by quintic Lagrange pieces
    through six samples; velocity and acceleration are the piece's
    derivatives."""

    def __init__(self, t0, dt, rs):
        self.t0, self.dt = t0, dt
        T = rs.shape[0]
        Vinv = np.linalg.inv(np.vander(np.arange(6.0), 6, increasing=True))
        win = np.stack([rs[i:i + 6] for i in range(T - 5)], 0)  # [seg, 6, particle, axis]
        self.coef = np.ascontiguousarray(np.einsum("pm,imab->aipb", Vinv, win))  # [particle, seg, power, axis]
        self.nseg = T - 5

    def __call__(self, p, t):
        x = (t - self.t0) / self.dt
        i = np.clip(np.floor(x).astype(int) - 2, 0, self.nseg - 1)
        tau = (x - i)[:, None]
        c = self.coef[p][i]
        r = np.zeros((len(t), 3))
        v = np.zeros_like(r)
        a = np.zeros_like(r)
        for k in range(5, -1, -1):
            r = r * tau + c[:, k]
        for k in range(5, 0, -1):
            v = v * tau + k * c[:, k]
        for k in range(5, 1, -1):
            a = a * tau + k * (k - 1) * c[:, k]
        return r, v / self.dt, a / self.dt ** 2


def _lienard_wiechert(traj, nparticles, q, X, t):
    """Retarded E and B at points X and time t: for each charge, solve
    t - t_r = |X - r(t_r)| / c (bisection, then Newton), then
        E = q / (4 pi eps0) [ (n - b)(1 - b^2) / (k^3 R^2) + n x ((n - b) x b') / (c k^3 R) ],
        B = n x E / c,  k = 1 - n.b, all at t_r."""
    E = np.zeros_like(X)
    B = np.zeros_like(X)
    for p in range(nparticles):
        lo = np.full(len(X), traj.t0 + 2 * traj.dt)
        hi = np.full(len(X), t)
        for _ in range(9):
            mid = 0.5 * (lo + hi)
            r, _, _ = traj(p, mid)
            f = t - mid - np.linalg.norm(X - r, axis=1) / C
            lo = np.where(f > 0, mid, lo)
            hi = np.where(f > 0, hi, mid)
        tr = 0.5 * (lo + hi)
        for _ in range(8):
            r, v, _ = traj(p, tr)
            Rv = X - r
            R = np.linalg.norm(Rv, axis=1)
            step = (t - tr - R / C) / (-1.0 + np.sum(Rv * v, 1) / (R * C * C))
            tr = tr - step
            if np.max(np.abs(step)) < 1e-6 * traj.dt:
                break
        r, v, a = traj(p, tr)
        Rv = X - r
        R = np.linalg.norm(Rv, axis=1)
        n = Rv / R[:, None]
        b = v / C
        bd = a / C
        k = 1.0 - np.sum(n * b, 1)
        nb = n - b
        Ev = nb * ((1.0 - np.sum(b * b, 1)) / (k ** 3 * R ** 2))[:, None]
        Ea = np.cross(n, np.cross(nb, bd)) / (C * k ** 3 * R)[:, None]
        Ep = q / (4.0 * math.pi * EPS0) * (Ev + Ea)
        E += Ep
        B += np.cross(n, Ep) / C
    return E, B


_H = 2.3e-5  # coarse dz (m)
_P0 = np.array([[0.3, -0.4, -2.2], [-1.1, 0.8, 1.7], [0.6, 1.3, 0.4]]) * _H
_U0 = np.array([[0.25, 0.0, 0.35], [0.0, -0.3, -0.25], [-0.2, 0.15, 0.1]])


def _lw_error(level, T0=24, ratio=1.5, sigma=1.0, rmin=5.0, rmax=0.4):
    """Relative L2 error of the grid E and B against the Lienard-Wiechert
    fields of three electrons in a planar undulator (K = 0.5), after T0
    coarse steps, at the nodes of the coarse mesh between rmin coarse cells
    from every electron and rmax c t from their start.

    Mesh level L halves dx, dy, dz L times over the same physical box and
    runs 2^L times as many steps, so the compared nodes and the time are the
    same physical ones.  A charge that appears at t = 0 and moves across the
    lattice also excites lattice-scale waves with little group velocity
    (and numerical Cherenkov waves), which have no continuum counterpart;
    both the grid fields and the Lienard-Wiechert fields are therefore
    smoothed by the same Gaussian of a fixed physical width (sigma coarse
    cells on each axis) before they are compared."""
    s = 2 ** level
    h = _H / s
    T = T0 * s
    hz = T0 + 8
    hx = int(math.ceil(T0 / ratio)) + 8
    nz, nx = 2 * hz * s + 1, 2 * hx * s + 1
    d = _desc(nx, nx, nz, h, ratio, ratio, K=0.5, z_entrance=-0.01,
              origin=(-hx * ratio * _H, -hx * ratio * _H, -hz * _H))
    o = Oracle(d)
    dt = o.consts()["dt"]
    ig = 1.0 / np.sqrt(1.0 + np.sum(_U0 ** 2, 1))
    xyz = _P0 + 0.5 * dt * C * _U0 * ig[:, None]  # positions at t = dt/2
    o.load_bunch(xyz, _U0, -QE)
    rs = [xyz - dt * C * _U0 * ig[:, None], o.particles()[0].copy()]  # t = -dt/2, +dt/2
    for _ in range(T + 3):
        o.step(1)
        rs.append(o.particles()[0].copy())
        if len(rs) == T + 2:  # T steps done: E, B at t_{T-1/2}
            F = np.stack([o.field(f) for f in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")], -1)
    rs = np.array(rs)
    traj = _Trajectory(-0.5 * dt, dt, rs)
    t = (T - 0.5) * dt
    # node box around the start holding every compared node plus the filter support
    Rb = rmax * C * t + 4 * sigma * ratio * _H
    c0 = rs[1].mean(0)

    def span(lo0, step, n, a, b):
        return max(0, int(math.floor((a - lo0) / step))), min(n - 1, int(math.ceil((b - lo0) / step)))

    ia = span(d["x0"], d["dx"], nx, c0[0] - Rb, c0[0] + Rb)
    ja = span(d["y0"], d["dy"], nx, c0[1] - Rb, c0[1] + Rb)
    ka = span(d["z0"], d["dz"], nz, c0[2] - Rb, c0[2] + Rb)
    kk, jj, ii = np.meshgrid(np.arange(ka[0], ka[1] + 1), np.arange(ja[0], ja[1] + 1),
                             np.arange(ia[0], ia[1] + 1), indexing="ij")
    X = np.stack([d["x0"] + ii * d["dx"], d["y0"] + jj * d["dy"], d["z0"] + kk * d["dz"]], -1)
    # nodes within a fraction of a cell of a charge have no finite retarded
    # field (and Newton may leave them non-finite); they lie outside the
    # smoothing support of every compared node, which the finiteness check
    # below confirms
    with np.errstate(all="ignore"):
        E, B = _lienard_wiechert(traj, len(_P0), -QE, X.reshape(-1, 3), t)
    Fl = np.concatenate([E, B], 1).reshape(X.shape[:3] + (6,))
    Fg = F[ka[0]:ka[1] + 1, ja[0]:ja[1] + 1, ia[0]:ia[1] + 1]

    def smooth(G):
        for ax in range(3):
            G = gaussian_filter1d(G, sigma * s, axis=ax, mode="constant", truncate=3.0)
        return G

    with np.errstate(all="ignore"):
        Fl, Fg = smooth(Fl), smooth(Fg)
    r_now = rs[T + 1]
    near = np.min(np.linalg.norm(X[..., None, :] - r_now, axis=-1), -1)
    far = np.max(np.linalg.norm(X[..., None, :] - rs[1], axis=-1), -1)
    coarse = ((kk % s) == 0) & ((jj % s) == 0) & ((ii % s) == 0)
    sel = coarse & (near > rmin * _H) & (far < rmax * C * t)
    assert np.all(np.isfinite(Fl[sel])) and np.all(np.isfinite(Fg[sel]))
    eE = np.linalg.norm(Fg[sel][:, :3] - Fl[sel][:, :3]) / np.linalg.norm(Fl[sel][:, :3])
    eB = np.linalg.norm(Fg[sel][:, 3:] - Fl[sel][:, 3:]) / np.linalg.norm(Fl[sel][:, 3:])
    return eE, eB, int(sel.sum()), C * np.linalg.norm(Fl[sel][:, 3:]) / np.linalg.norm(Fl[sel][:, :3])


def test_lienard_wiechert_fields_converge_at_second_order():
    """Three electrons (q = -e, so their own fields do not bend their paths
    measurably) wiggle in a planar undulator with |beta| up to ~0.5.  The
    grid E and B approach the retarded fields of the trajectories the oracle
    itself produced, and the error falls about fourfold when the mesh is
    halved: measured 14.8 % -> 2.8 % (E) and 16.9 % -> 5.1 % (B) on about 900
    nodes 5 to 9.6 coarse cells from the charges.  A doubled or
    sign-flipped A source leaves errors of 40-120 % that do not converge."""
    e0, b0, n0, cb = _lw_error(0)
    e1, b1, n1, _ = _lw_error(1)
    assert n0 > 500 and n1 == pytest.approx(n0, rel=0.1)
    assert cb > 0.3  # the magnetic field is a large part of the comparison
    assert e1 < 0.04 and b1 < 0.07, (e1, b1)
    assert 3.0 < e0 / e1 < 8.0, (e0, e1)
    assert 2.8 < b0 / b1 < 8.0, (b0, b1)


# ---------------------------------------------------------------------------
# Undulator conventions
# ---------------------------------------------------------------------------

def _lab_field(o, zl, x=0.0, y=0.0):
    """Lab-frame undulator B' at lab position z' (entrance at 0), recovered
    from the boosted field at t = 0: B_x = gamma0 B'_x, B_y = gamma0 B'_y,
    B_z = B'_z (the boost of a pure magnetic field)."""
    c = o.consts()
    g0 = c["gamma0"]
    z = o.desc["z_entrance"] + zl / g0
    E, B = o.external_field(np.array([x, y, z]), 0.0)
    return np.array([B[0] / g0, B[1] / g0, B[2]]), E


def test_polarisation_angle_turns_the_field_from_y_toward_x():
    """Reading: the planar field at angle theta points along (sin theta,
    cos theta, 0) in (x, y): theta = 0 is the field along y of eq.
    undulatorField, and a positive theta turns it toward +x."""
    lam = 0.03
    B0 = 2 * math.pi * ME * C * 1.0 / (QE * lam)
    zl = 10.25 * lam  # sin(k_u z') = 1 inside the magnet
    for theta in (30.0, 90.0, 135.0):
        o = Oracle(_desc(16, 16, 20, 2e-5, 4.0, 4.0, K=1.0, pol=theta))
        Bl, E = _lab_field(o, zl)
        th = math.radians(theta)
        assert Bl[0] == pytest.approx(B0 * math.sin(th), rel=1e-12, abs=1e-12 * B0)
        assert Bl[1] == pytest.approx(B0 * math.cos(th), rel=1e-12, abs=1e-12 * B0)
        # the field sets the wiggle plane: the boosted E is along z x B'
        # (E_x = -gamma0 beta0 c B'_y, E_y = +gamma0 beta0 c B'_x)
        assert E[0] * Bl[1] <= 0 and E[1] * Bl[0] >= 0


def test_helical_field_turns_from_x_toward_y_along_z():
    """Reading (the paper has no helical formula): inside the magnet the
    helical field is B'_perp = B0 (cos k_u z', sin k_u z'), the planar
    pattern along y plus the pattern along x a quarter period upstream.  The
    field therefore turns from +x toward +y as z' grows (a right-handed
    helix about +z): z . (B' x dB'/dz') = B0^2 k_u > 0."""
    lam = 0.03
    K = 1.4
    ku = 2 * math.pi / lam
    B0 = 2 * math.pi * ME * C * K / (QE * lam)
    o = Oracle(_desc(16, 16, 20, 2e-5, 4.0, 4.0, K=K, und_type=1))
    for zl in (7.0 * lam, 7.1 * lam, 23.37 * lam):
        Bl, _ = _lab_field(o, zl)
        assert Bl[0] == pytest.approx(B0 * math.cos(ku * zl), abs=1e-9 * B0)
        assert Bl[1] == pytest.approx(B0 * math.sin(ku * zl), abs=1e-9 * B0)
        eps = 1e-4 * lam
        Bp, _ = _lab_field(o, zl + eps)
        Bm, _ = _lab_field(o, zl - eps)
        dB = (Bp - Bm) / (2 * eps)
        twist = Bl[0] * dB[1] - Bl[1] * dB[0]
        assert twist == pytest.approx(B0 * B0 * ku, rel=1e-6)
