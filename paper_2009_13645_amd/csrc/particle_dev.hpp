// particle_dev.hpp -- device functions of the particle phase:
//  * external static undulator field: lab-frame field at the position
//    z' = gamma0 (z - z_entrance + beta0 c t) with entrance and exit fringes,
//    boosted with E' = 0 (MITHRA 2.0 manual, eqs. undulatorField,
//    fringingField, LorentzTransformR2L, LorentzTransformElectric/Magnetic);
//    helical = the planar pattern plus its 90-degree rotation a quarter
//    period upstream;
//  * Boris momentum update (eq. BorisScheme);
//  * charge-conserving deposit: zigzag split at the printed relay point,
//    each segment carrying the exact current of a straight move inside one
//    cell under linear weights; cloud-in-cell charge.
#pragma once

#include "mithra_dev.hpp"

namespace mithra {

__device__ inline void cosh_sinh(double x, double &ch, double &sh)
{
    const double em = expm1(x);
    const double inv = 1.0 / (1.0 + em);
    sh = 0.5 * em * (2.0 + em) * inv;
    ch = 1.0 + 0.5 * em * em * inv;
}

// longitudinal profile of the planar pattern at lab z': (g, h) multiply
// cosh / sinh of the transverse argument for the transverse / longitudinal
// field: periodic body, fringe before the entrance and (mirrored) after
// the exit
__device__ inline void profile(const RunDev &R, double zl, double &g, double &h)
{
    if (zl < 0.0 || zl > R.Lu) {
        const double a = R.ku * (zl < 0.0 ? zl : zl - R.Lu);
        const double e = exp(-0.5 * a * a);
        g = a * e;
        h = e;
    } else {
        sincos(R.ku * zl, &g, &h);
    }
}

__device__ inline void undulator_field(const RunDev &R, double x, double y, double z, double t, double E[3],
                                       double B[3])
{
    const double zl = R.gamma0 * (z - R.z_ent + R.beta0 * kC * t);
    double Bl[3];
    if (R.und_type == 1) {
        // planar pattern along y at z' plus planar pattern along x at
        // z' + lambda_u/4; inside the magnet the second profile is the
        // first shifted by a quarter period: (g, h) -> (h, -g)
        const double zq = zl + 0.25 * (2.0 * kPi / R.ku);
        double g1, h1, g2, h2;
        profile(R, zl, g1, h1);
        if (zq >= 0.0 && zq <= R.Lu && zl >= 0.0) {
            g2 = h1;
            h2 = -g1;
        } else {
            profile(R, zq, g2, h2);
        }
        double chy, shy, chx, shx;
        cosh_sinh(R.ku * y, chy, shy);
        cosh_sinh(R.ku * x, chx, shx);
        Bl[0] = R.B0 * chx * g2;
        Bl[1] = R.B0 * chy * g1;
        Bl[2] = R.B0 * (shy * h1 + shx * h2);
    } else {
        double sth, cth, g, h, ch, sh;
        sincos(R.theta, &sth, &cth);
        profile(R, zl, g, h);
        cosh_sinh(R.ku * (x * sth + y * cth), ch, sh);
        const double bp = R.B0 * ch * g;
        Bl[0] = bp * sth;
        Bl[1] = bp * cth;
        Bl[2] = R.B0 * sh * h;
    }
    const double gbc = R.gamma0 * R.beta0 * kC;
    E[0] = -gbc * Bl[1];
    E[1] = gbc * Bl[0];
    E[2] = 0.0;
    B[0] = R.gamma0 * Bl[0];
    B[1] = R.gamma0 * Bl[1];
    B[2] = Bl[2];
}

// ---- general external field: undulator arrays and optical undulators ----

// window of the gap fringes of an undulator array: 1 at the module edge,
// ~6e-5 at the far end of the gap
__device__ inline double gap_window(double dz, double g)
{
    const double t = kPi * dz / g;
    return 0.35875 + 0.48829 * cos(t) + 0.14128 * cos(2.0 * t) + 0.01168 * cos(3.0 * t);
}

// longitudinal profile of the planar pattern of a module array at lab z'
// (first entrance at 0), scaled by the module's B0 (K_m = K + m dK): body,
// fringe before the first module and after the last, windowed fringes of
// the two modules around a gap
__device__ inline void array_profile(const RunDev &R, double zl, double &gB, double &hB)
{
    const int M = R.n_modules;
    const double pitch = R.Lu + R.gap;
    int m = (int)floor(zl / pitch);
    m = m < 0 ? 0 : (m > M - 1 ? M - 1 : m);
    const double ent = m * pitch, ext = ent + R.Lu;
    const double b0 = 2.0 * kPi * kMe * kC * (R.Kund + m * R.dK) / (kQe * R.lam_u);
    if (zl >= ent && zl <= ext) {
        gB = b0 * sin(R.ku * (zl - ent));
        hB = b0 * cos(R.ku * (zl - ent));
        return;
    }
    if (zl < ent) {
        const double a = R.ku * (zl - ent), e = exp(-0.5 * a * a);
        gB = b0 * (a * e);
        hB = b0 * e;
        return;
    }
    const double a1 = R.ku * (zl - ext), e1 = exp(-0.5 * a1 * a1);
    if (m == M - 1) {
        gB = b0 * (a1 * e1);
        hB = b0 * e1;
        return;
    }
    const double ent2 = (m + 1) * pitch;
    const double b1 = 2.0 * kPi * kMe * kC * (R.Kund + (m + 1) * R.dK) / (kQe * R.lam_u);
    const double a2 = R.ku * (zl - ent2), e2 = exp(-0.5 * a2 * a2);
    const double f1 = gap_window(zl - ext, R.gap), f2 = gap_window(ent2 - zl, R.gap);
    gB = b0 * (a1 * e1) * f1 + b1 * (a2 * e2) * f2;
    hB = b0 * e1 * f1 + b1 * e2 * f2;
}

__device__ inline void array_planar(const RunDev &R, double x, double y, double zl, double th, double Bl[3])
{
    double gB, hB, sth, cth;
    array_profile(R, zl, gB, hB);
    sincos(th, &sth, &cth);
    const double eta = x * sth + y * cth;
    const double Bperp = gB * cosh(R.ku * eta);
    Bl[0] = Bperp * sth;
    Bl[1] = Bperp * cth;
    Bl[2] = hB * sinh(R.ku * eta);
}

// optical pulse signature with unit amplitude (modulated Neumann scaled by
// the duration to be dimensionless, modulated Gaussian, modulated sech,
// sinusoidal pulse with a Gaussian rise)
__device__ inline double signal_value(int type, double tau, double f, double tp, double t0, double ph)
{
    const double d = tau - t0;
    const double car = cos(2.0 * kPi * f * d + ph);
    const double ln2 = 0.69314718055994530942;
    switch (type) {
    case 0:
        return -4.0 * ln2 * car * (d / tp) * exp(-2.0 * ln2 * d * d / (tp * tp));
    case 1:
        return car * exp(-2.0 * ln2 * d * d / (tp * tp));
    case 2:
        return car / cosh(d / tp);
    default:
        return d <= 0.0 ? car * exp(-2.0 * ln2 * d * d / (tp * tp)) : car;
    }
}

// lab fields of the optical undulator (strength a0 = K, wavelength
// 2 lambda_u, propagating along -z; B along (sin th, cos th), E along
// (-cos th, sin th)); plane wave or Gaussian beam
__device__ inline void optical_lab(const RunDev &R, double x, double y, double zl, double tl, double El[3],
                                   double Bl[3])
{
    const double lam = 2.0 * R.lam_u;
    const double om = 2.0 * kPi * kC / lam;
    const double E0 = R.Kund * kMe * kC * om / kQe;
    const double f = kC / lam, tp = R.opt_ctau / kC, t0 = R.opt_ct0 / kC;
    double sth, cth;
    sincos(R.theta, &sth, &cth);
    const double p[2] = {-cth, sth}, q[2] = {sth, cth};
    if (R.und_type == 2) {
        const double sv = signal_value(R.opt_signal, tl + zl / kC, f, tp, t0, R.opt_cep);
        for (int a = 0; a < 2; ++a) {
            El[a] = E0 * sv * p[a];
            Bl[a] = (E0 / kC) * sv * q[a];
        }
        El[2] = 0.0;
        Bl[2] = 0.0;
        return;
    }
    const double k0 = 2.0 * kPi / lam;
    const double l = R.opt_zf - zl;
    const double rp = x * p[0] + y * p[1], rq = x * q[0] + y * q[1];
    const double w0p = R.opt_w0[0], w0q = R.opt_w0[1];
    const double zRp = kPi * w0p * w0p / lam, zRq = kPi * w0q * w0q / lam;
    const double wp = w0p * sqrt(1.0 + (l / zRp) * (l / zRp)), wq = w0q * sqrt(1.0 + (l / zRq) * (l / zRq));
    const double iRp = l / (l * l + zRp * zRp), iRq = l / (l * l + zRq * zRq);
    const double amp = sqrt((w0p * w0q) / (wp * wq)) * exp(-rq * rq / (wq * wq) - rp * rp / (wp * wp));
    const double curv = -0.5 * k0 * rp * rp * iRp - 0.5 * k0 * rq * rq * iRq;
    const double Gp = atan(l / zRp), Gq = atan(l / zRq);
    const double tau = tl - l / kC;
    const double Epar = E0 * amp * signal_value(R.opt_signal, tau, f, tp, t0, R.opt_cep + curv - 0.5 * kPi + 0.5 * (Gp + Gq));
    const double Elon = E0 * (rp * w0p / (zRp * wp)) * amp *
                        signal_value(R.opt_signal, tau, f, tp, t0, R.opt_cep + curv + 0.5 * (3.0 * Gp + Gq));
    const double Blon = (E0 / kC) * (rq * w0q / (zRq * wq)) * amp *
                        signal_value(R.opt_signal, tau, f, tp, t0, R.opt_cep + curv + 0.5 * (Gp + 3.0 * Gq));
    for (int a = 0; a < 2; ++a) {
        El[a] = Epar * p[a];
        Bl[a] = (Epar / kC) * q[a];
    }
    El[2] = -Elon;
    Bl[2] = -Blon;
}

// the external field in the general case, boosted with E' != 0:
// E = g0 (E' + c beta0 z x B') - (g0 - 1) E'_z z, B = g0 (B' - beta0 z x E' / c) - (g0 - 1) B'_z z
__device__ inline void undulator_field_ext(const RunDev &R, double x, double y, double z, double t, double E[3],
                                           double B[3])
{
    const double g0 = R.gamma0, b0 = R.beta0;
    const double zl = g0 * (z - R.z_ent + b0 * kC * t);
    double El[3] = {0.0, 0.0, 0.0}, Bl[3] = {0.0, 0.0, 0.0};
    if (R.und_type >= 2) {
        const double tl = g0 * (t + b0 * (z - R.z_ent) / kC);
        optical_lab(R, x, y, zl, tl, El, Bl);
    } else if (R.und_type == 1) {
        double tmp[3];
        array_planar(R, x, y, zl, 0.0, tmp);
        for (int a = 0; a < 3; ++a)
            Bl[a] += tmp[a];
        array_planar(R, x, y, zl + 0.25 * R.lam_u, 0.5 * kPi, tmp);
        for (int a = 0; a < 3; ++a)
            Bl[a] += tmp[a];
    } else {
        array_planar(R, x, y, zl, R.theta, Bl);
    }
    E[0] = g0 * (El[0] + kC * b0 * (-Bl[1]));
    E[1] = g0 * (El[1] + kC * b0 * (Bl[0]));
    E[2] = g0 * El[2] - (g0 - 1.0) * El[2];
    B[0] = g0 * (Bl[0] - b0 * (-El[1]) / kC);
    B[1] = g0 * (Bl[1] - b0 * (El[0]) / kC);
    B[2] = g0 * Bl[2] - (g0 - 1.0) * Bl[2];
}

// the external field of a run: the single static module on its own path
// (EXT = false: the benchmark's push), arrays and optical undulators on the
// general one
template <bool EXT>
__device__ inline void external_field(const RunDev &R, double x, double y, double z, double t, double E[3], double B[3])
{
    if constexpr (EXT)
        undulator_field_ext(R, x, y, z, t, E, B);
    else
        undulator_field(R, x, y, z, t, E, B);
}

__device__ inline void boris(double u[3], const double E[3], const double B[3], double dtb)
{
    const double ek = kQe * dtb / (2.0 * kMe * kC);
    double t1[3];
    for (int a = 0; a < 3; ++a)
        t1[a] = u[a] - ek * E[a];
    const double alpha = -kQe * dtb / (2.0 * kMe * sqrt(1.0 + t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]));
    double t2[3];
    t2[0] = t1[0] + alpha * (t1[1] * B[2] - t1[2] * B[1]);
    t2[1] = t1[1] + alpha * (t1[2] * B[0] - t1[0] * B[2]);
    t2[2] = t1[2] + alpha * (t1[0] * B[1] - t1[1] * B[0]);
    const double f = 2.0 * alpha / (1.0 + alpha * alpha * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]));
    const double s[3] = {f * B[0], f * B[1], f * B[2]};
    u[0] = t1[0] + (t2[1] * s[2] - t2[2] * s[1]) - ek * E[0];
    u[1] = t1[1] + (t2[2] * s[0] - t2[0] * s[2]) - ek * E[1];
    u[2] = t1[2] + (t2[0] * s[1] - t2[1] * s[0]) - ek * E[2];
}

// grid coordinates and active cell (1 <= cell <= n-3 on every axis)
__device__ inline bool cell_of(const RunDev &R, const double r[3], double g[3], int c[3])
{
    g[0] = (r[0] - R.x0) / R.dx;
    g[1] = (r[1] - R.y0) / R.dy;
    g[2] = (r[2] - R.z0) / R.dz;
    const int n[3] = {R.nx, R.ny, R.nz};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double f = floor(g[a]);
        ok = ok && (f >= 1.0) && (f <= (double)(n[a] - 3));
        c[a] = ok ? (int)f : 0;
    }
    return ok;
}

// --- accumulation --------------------------------------------------------

// Global accumulation into source set `set` (J_x J_y J_z rho).  FP64: plain
// atomic add.  FP32: atomic add of the rounded value; with compensation the
// exact error of that addition (two-sum on the returned old value) plus the
// rounding of the FP64 value goes into the second array by another atomic.
template <typename T, bool COMP>
struct GlobalAcc {
    // the four arrays of a source set are contiguous: array c starts at c * nn
    T *A0;
    T *Lo0;
    int64_t nn;
    int nx;
    int64_t nxy;
    // the four components of node `at` (one index for all four: each add is
    // one address add from its array's start); zeros skipped; in the
    // compensated mode all the returning adds are issued before their errors
    // are added
    __device__ inline void add4(const double v[4], int64_t at) const
    {
        if constexpr (sizeof(T) == 8) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v[q] != 0.0)
                    atomicAdd(reinterpret_cast<double *>(A0) + q * nn + at, v[q]);
        } else if (!COMP) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v[q] != 0.0)
                    atomicAdd(reinterpret_cast<float *>(A0) + q * nn + at, (float)v[q]);
        } else {
            float vf[4], old[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                vf[q] = (float)v[q];
                old[q] = 0.0f;
                if (v[q] != 0.0)
                    old[q] = atomicAdd(reinterpret_cast<float *>(A0) + q * nn + at, vf[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (v[q] != 0.0) {
                    const float sm = old[q] + vf[q];
                    const float bv = sm - old[q];
                    const float err = (old[q] - (sm - bv)) + (vf[q] - bv);
                    atomicAdd(reinterpret_cast<float *>(Lo0) + q * nn + at, err + (float)(v[q] - (double)vf[q]));
                }
            }
        }
    }
    // index of node (i, j, k) in one array, the index steps along x, y, z,
    // and the add at an index
    __device__ inline int64_t base(const int c[3]) const { return (int64_t)c[2] * nxy + (int64_t)c[1] * nx + c[0]; }
    __device__ inline int64_t stride(int axis) const { return axis == 0 ? 1 : (axis == 1 ? (int64_t)nx : nxy); }
    __device__ inline void add_idx(int comp, int64_t idx, double v) const
    {
        if constexpr (sizeof(T) == 8) {
            atomicAdd(reinterpret_cast<double *>(A0) + comp * nn + idx, v);
        } else {
            const float vf = (float)v;
            const float old = atomicAdd(reinterpret_cast<float *>(A0) + comp * nn + idx, vf);
            if (COMP) {
                const float sm = old + vf;
                const float bv = sm - old;
                const float err = (old - (sm - bv)) + (vf - bv);
                atomicAdd(reinterpret_cast<float *>(Lo0) + comp * nn + idx, err + (float)(v - (double)vf));
            }
        }
    }
};

template <typename T, bool COMP>
__device__ inline GlobalAcc<T, COMP> make_gacc(const RunDev &R, int set)
{
    GlobalAcc<T, COMP> a;
    a.A0 = src_ptr<T>(R, set, 0);
    a.Lo0 = COMP ? srclo_ptr<T>(R, set, 0) : nullptr;
    a.nn = R.nn;
    a.nx = R.nx;
    a.nxy = (int64_t)R.nx * R.ny;
    return a;
}

// Block-local accumulation in LDS over a node box (FP64, or FP32 where the
// run accumulates in FP32 without compensation).
template <typename AccT = double>
struct LdsAcc {
    AccT *s;
    int lo0, lo1, lo2, ex, ey, vol;
    // index of node (i, j, k) in the box, the index steps along x, y, z,
    // and the add at an index
    __device__ inline int base(const int c[3]) const { return ((c[2] - lo2) * ey + (c[1] - lo1)) * ex + (c[0] - lo0); }
    __device__ inline int stride(int axis) const { return axis == 0 ? 1 : (axis == 1 ? ex : ex * ey); }
    __device__ inline void add_idx(int comp, int idx, double v) const { atomicAdd(&s[comp * vol + idx], (AccT)v); }
};

// Lane order of a particle's adds: lanes of one cell would add to the same
// node at once, and same-address atomics serialize.  So the add that the
// code issues as corner e goes, on lane l, to corner e XOR r (r = l mod 8
// for the eight charge corners, l mod 4 for the four edges of a current
// component): along each axis whose bit of r is set, the corner's two
// weights and its two index offsets trade places.  A lane pays that once per
// particle (a few selects), where an additive rotation picked the value and
// the offsets of every add from all of them.

// Current of the move g1 (cell c1) -> g2 (cell c2), grid units: the zigzag
// splits it at the relay point gr (the crossed cell face on an axis whose
// cell changes, the midpoint on the others) into segment A (g1 -> gr, in c1)
// and segment B (gr -> g2, in c2); each carries the exact current of a
// straight move inside its cell under linear weights.  For component l, the
// edge at offsets (s1, s2) along the two other axes (m1, m2) gets
// F (p1[s1] p2[s2] + x) when s1 == s2 and F (p1[s1] p2[s2] - x) otherwise,
// with p[0] = 1 - u, p[1] = u (u: the segment's mean offset along that
// axis), x = d_m1 d_m2 / 12 and F = q d_l / (dt V).  Every lane runs the
// same code: when the move stays in one cell, B's values ride on A's adds
// (12 adds instead of 24); otherwise B adds on its own edges.
template <class Acc>
__device__ inline void deposit_move(const RunDev &R, const Acc &acc, const double g1[3], const int c1[3],
                                    const double g2[3], const int c2[3])
{
    double gr[3];
    for (int l = 0; l < 3; ++l) {
        const double lo = (double)min(c1[l], c2[l]) + 1.0;
        const double hi = (double)max(c1[l], c2[l]);
        gr[l] = fmin(lo, fmax(hi, 0.5 * (g1[l] + g2[l])));
    }
    const bool same = c1[0] == c2[0] && c1[1] == c2[1] && c1[2] == c2[2];
    const double sm = same ? 1.0 : 0.0;
    const auto b1 = acc.base(c1), b2 = acc.base(c2);
    double dA[3], dB[3], WA[3], WB[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        dA[l] = gr[l] - g1[l];
        dB[l] = g2[l] - gr[l];
        WA[l] = 0.5 * (g1[l] + gr[l]) - (double)c1[l];
        WB[l] = 0.5 * (gr[l] + g2[l]) - (double)c2[l];
    }
    const bool r0 = (threadIdx.x & 1) != 0, r1 = (threadIdx.x & 2) != 0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int m1 = (l + 1) % 3, m2 = (l + 2) % 3;
        const double FA = dA[l] * R.qvh_dt[l], FB = dB[l] * R.qvh_dt[l];
        // x with the sign of the edges whose issued offsets are equal
        const double xA = (r0 == r1 ? 1.0 : -1.0) * (dA[m1] * dA[m2] * (1.0 / 12.0));
        const double xB = (r0 == r1 ? 1.0 : -1.0) * (dB[m1] * dB[m2] * (1.0 / 12.0));
        // p[e ^ r] for issued offset e
        const double pA1[2] = {r0 ? WA[m1] : 1.0 - WA[m1], r0 ? 1.0 - WA[m1] : WA[m1]};
        const double pA2[2] = {r1 ? WA[m2] : 1.0 - WA[m2], r1 ? 1.0 - WA[m2] : WA[m2]};
        const double pB1[2] = {r0 ? WB[m1] : 1.0 - WB[m1], r0 ? 1.0 - WB[m1] : WB[m1]};
        const double pB2[2] = {r1 ? WB[m2] : 1.0 - WB[m2], r1 ? 1.0 - WB[m2] : WB[m2]};
        const auto st1 = acc.stride(m1), st2 = acc.stride(m2);
        const decltype(st1) o1[2] = {r0 ? st1 : 0, r0 ? 0 : st1}, o2[2] = {r1 ? st2 : 0, r1 ? 0 : st2};
        double wB[2][2];
#pragma unroll
        for (int e1 = 0; e1 < 2; ++e1)
#pragma unroll
            for (int e2 = 0; e2 < 2; ++e2) {
                const double wA = FA * (pA1[e1] * pA2[e2] + (e1 == e2 ? xA : -xA));
                wB[e1][e2] = FB * (pB1[e1] * pB2[e2] + (e1 == e2 ? xB : -xB));
                acc.add_idx(l, b1 + o1[e1] + o2[e2], wA + sm * wB[e1][e2]);
            }
        if (!same) {
#pragma unroll
            for (int e1 = 0; e1 < 2; ++e1)
#pragma unroll
                for (int e2 = 0; e2 < 2; ++e2)
                    acc.add_idx(l, b2 + o1[e1] + o2[e2], wB[e1][e2]);
        }
    }
}

// Cloud-in-cell charge on the eight corners of cell c.
template <class Acc>
__device__ inline void deposit_charge(const RunDev &R, const Acc &acc, const double g[3], const int c[3])
{
    const double dx = g[0] - c[0], dy = g[1] - c[1], dz = g[2] - c[2];
    const bool r0 = (threadIdx.x & 1) != 0, r1 = (threadIdx.x & 2) != 0, r2 = (threadIdx.x & 4) != 0;
    // weight and index offset of issued offset e along each axis: those of e ^ r
    const double wx[2] = {r0 ? dx : 1.0 - dx, r0 ? 1.0 - dx : dx};
    const double wy[2] = {r1 ? dy : 1.0 - dy, r1 ? 1.0 - dy : dy};
    const double wz[2] = {r2 ? dz : 1.0 - dz, r2 ? 1.0 - dz : dz};
    const auto sy = acc.stride(1), sz = acc.stride(2);
    const decltype(sy) ox[2] = {r0 ? 1 : 0, r0 ? 0 : 1}, oy[2] = {r1 ? sy : 0, r1 ? 0 : sy},
                       oz[2] = {r2 ? sz : 0, r2 ? 0 : sz};
    const auto b = acc.base(c);
#pragma unroll
    for (int K = 0; K < 2; ++K)
#pragma unroll
        for (int J = 0; J < 2; ++J)
#pragma unroll
            for (int I = 0; I < 2; ++I)
                acc.add_idx(3, b + ox[I] + oy[J] + oz[K], R.qV * wx[I] * wy[J] * wz[K]);
}

// floor(n / d) for 0 <= n < 2^52 and d >= 1, from inv_d = 1 / d rounded to
// FP64: (n + 1/2) / d lies at least 1/(2d) from an integer, and the two
// roundings move it by less than 2.3e-16 (n + 1/2) / d, which is smaller
// for every n here; three instructions instead of an integer division.
__device__ inline int64_t small_div(int64_t n, double inv_d)
{
    return (int64_t)(((double)n + 0.5) * inv_d);
}

// the same for 0 <= n < 2^31 in 32-bit registers (four instructions)
__device__ inline int small_div(int n, double inv_d)
{
    return (int)(((double)n + 0.5) * inv_d);
}

// Minimum / maximum over the 64 lanes of a wavefront (every lane active):
// prefix reductions inside each row of 16 lanes with DPP row shifts (a lane
// whose source lies outside its row keeps its own value), then the rows'
// last lanes combined through readlane.  No LDS crossbar traffic, unlike a
// shuffle, which the deposit's atomics compete with.
__device__ inline int wave_min(int v)
{
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    return min(min(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
               min(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}

__device__ inline int wave_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xf, 0xf, false));
    return max(max(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
               max(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}

}  // namespace mithra
