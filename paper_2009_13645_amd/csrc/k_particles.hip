// k_particles.hip -- particle phase of the boosted-frame PIC step.
//
//  * gather of the vertex E and B (trilinear, eq. fieldInterpolation with
//    the linear weights 1 - d, d);
//  * external static undulator field: lab-frame field at the position
//    z' = gamma0 (z - z_entrance + beta0 c t) with entrance and exit fringes,
//    boosted with E' = 0 (eqs. undulatorField, fringingField,
//    LorentzTransformR2L, LorentzTransformElectric/Magnetic); helical = the
//    planar pattern plus its 90-degree rotation a quarter period upstream;
//  * N_b Boris sub-steps (eq. BorisScheme) with the grid field held at
//    t_{n+1/2} and the undulator field re-evaluated per sub-step;
//  * charge-conserving deposit: zigzag split at the printed relay point,
//    each segment carrying the exact current of a straight move inside one
//    cell under linear weights; cloud-in-cell charge.  Accumulation is by
//    device-scope atomics into the source set of the next step; in the
//    compensated FP32 mode every atomic add is followed by an atomic add of
//    its exact rounding error (two-sum) into a second array.
// Particles are processed in the order of the last sort (by cell tile).
#include "mithra_dev.hpp"

namespace mithra {

__device__ inline void lab_planar(const RunDev &R, double x, double y, double zl, double cth, double sth,
                                  double Bl[3])
{
    const double eta = x * sth + y * cth;
    double g, hh;
    if (zl < 0.0) {
        const double a = R.ku * zl;
        const double e = exp(-0.5 * a * a);
        g = a * e;
        hh = e;
    } else if (zl > R.Lu) {
        const double a = R.ku * (zl - R.Lu);
        const double e = exp(-0.5 * a * a);
        g = a * e;
        hh = e;
    } else {
        sincos(R.ku * zl, &g, &hh);
    }
    const double ke = R.ku * eta;
    const double bp = R.B0 * cosh(ke) * g;
    Bl[0] = bp * sth;
    Bl[1] = bp * cth;
    Bl[2] = R.B0 * sinh(ke) * hh;
}

__device__ inline void undulator_field(const RunDev &R, double x, double y, double z, double t, double E[3],
                                       double B[3])
{
    const double zl = R.gamma0 * (z - R.z_ent + R.beta0 * kC * t);
    double Bl[3];
    if (R.und_type == 1) {
        double b2[3];
        lab_planar(R, x, y, zl, 1.0, 0.0, Bl);
        lab_planar(R, x, y, zl + 0.25 * (2.0 * kPi / R.ku), 0.0, 1.0, b2);
        for (int a = 0; a < 3; ++a)
            Bl[a] += b2[a];
    } else {
        double sth, cth;
        sincos(R.theta, &sth, &cth);
        lab_planar(R, x, y, zl, cth, sth, Bl);
    }
    const double gbc = R.gamma0 * R.beta0 * kC;
    E[0] = -gbc * Bl[1];
    E[1] = gbc * Bl[0];
    E[2] = 0.0;
    B[0] = R.gamma0 * Bl[0];
    B[1] = R.gamma0 * Bl[1];
    B[2] = Bl[2];
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
    for (int a = 0; a < 3; ++a) {
        const double f = floor(g[a]);
        ok = ok && (f >= 1.0) && (f <= (double)(n[a] - 3));
        c[a] = ok ? (int)f : 0;
    }
    return ok;
}

// --- accumulation --------------------------------------------------------

__device__ inline void acc_add(double *p, double *, double v) { atomicAdd(p, v); }

template <bool COMP>
__device__ inline void acc_add(float *p, float *lo, double v)
{
    const float vf = (float)v;
    const float old = atomicAdd(p, vf);
    if (COMP) {
        // exact error of old + vf (two-sum) plus the rounding of v to float
        const float sm = old + vf;
        const float bv = sm - old;
        const float err = (old - (sm - bv)) + (vf - bv);
        atomicAdd(lo, err + (float)(v - (double)vf));
    }
}

template <typename T, bool COMP>
struct Acc {
    T *J[3];
    T *Jlo[3];
    T *Q;
    T *Qlo;
    __device__ inline void add(int comp, int64_t idx, double v) const
    {
        if constexpr (sizeof(T) == 8) {
            (void)COMP;
            atomicAdd(reinterpret_cast<double *>(comp < 3 ? J[comp] : Q) + idx, v);
        } else {
            acc_add<COMP>(reinterpret_cast<float *>(comp < 3 ? J[comp] : Q) + idx,
                          COMP ? reinterpret_cast<float *>(comp < 3 ? Jlo[comp] : Qlo) + idx : nullptr, v);
        }
    }
};

template <typename T, bool COMP>
__device__ inline Acc<T, COMP> make_acc(const RunDev &R, int set)
{
    Acc<T, COMP> a;
    for (int c = 0; c < 3; ++c) {
        a.J[c] = src_ptr<T>(R, set, c);
        a.Jlo[c] = COMP ? srclo_ptr<T>(R, set, c) : nullptr;
    }
    a.Q = src_ptr<T>(R, set, 3);
    a.Qlo = COMP ? srclo_ptr<T>(R, set, 3) : nullptr;
    return a;
}

// current of the straight segment a -> b (grid units) inside cell c
template <typename T, bool COMP>
__device__ inline void segment_current(const RunDev &R, const Acc<T, COMP> &acc, const double a[3],
                                       const double b[3], const int c[3])
{
    const int64_t stride[3] = {1, R.nx, (int64_t)R.nx * R.ny};
    const int64_t base = nid(R, c[0], c[1], c[2]);
    double d[3], W[3];
    for (int l = 0; l < 3; ++l) {
        d[l] = b[l] - a[l];
        W[l] = 0.5 * (a[l] + b[l]) - (double)c[l];
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int m1 = (l + 1) % 3, m2 = (l + 2) % 3;
        // J_l = q (displacement in metres) / (dt V) times the edge weights
        const double F = R.qV * d[l] * R.h[l] / R.dt;
        const double x = d[m1] * d[m2] * (1.0 / 12.0);
        const double u1 = W[m1], u2 = W[m2];
        acc.add(l, base, F * ((1.0 - u1) * (1.0 - u2) + x));
        acc.add(l, base + stride[m1], F * (u1 * (1.0 - u2) - x));
        acc.add(l, base + stride[m2], F * ((1.0 - u1) * u2 - x));
        acc.add(l, base + stride[m1] + stride[m2], F * (u1 * u2 + x));
    }
}

struct Box {
    int lo[3], hi[3];
};

template <typename T, bool COMP>
__device__ inline void deposit_move(const RunDev &R, const Acc<T, COMP> &acc, const double g1[3], const int c1[3],
                                    const double g2[3], const int c2[3], Box &bx)
{
    double gr[3];
    for (int l = 0; l < 3; ++l) {
        const double lo = (double)min(c1[l], c2[l]) + 1.0;
        const double hi = (double)max(c1[l], c2[l]);
        gr[l] = fmin(lo, fmax(hi, 0.5 * (g1[l] + g2[l])));
        bx.lo[l] = min(bx.lo[l], min(c1[l], c2[l]));
        bx.hi[l] = max(bx.hi[l], max(c1[l], c2[l]) + 1);
    }
    segment_current<T, COMP>(R, acc, g1, gr, c1);
    segment_current<T, COMP>(R, acc, gr, g2, c2);
}

template <typename T, bool COMP>
__device__ inline void deposit_charge(const RunDev &R, const Acc<T, COMP> &acc, const double g[3], const int c[3],
                                      Box &bx)
{
    const int64_t base = nid(R, c[0], c[1], c[2]);
    const int64_t sy = R.nx, sz = (int64_t)R.nx * R.ny;
    const double dx = g[0] - c[0], dy = g[1] - c[1], dz = g[2] - c[2];
    const double wx[2] = {1.0 - dx, dx}, wy[2] = {1.0 - dy, dy}, wz[2] = {1.0 - dz, dz};
#pragma unroll
    for (int K = 0; K < 2; ++K)
#pragma unroll
        for (int J = 0; J < 2; ++J)
#pragma unroll
            for (int I = 0; I < 2; ++I)
                acc.add(3, base + I + J * sy + K * sz, R.qV * wx[I] * wy[J] * wz[K]);
    for (int l = 0; l < 3; ++l) {
        bx.lo[l] = min(bx.lo[l], c[l]);
        bx.hi[l] = max(bx.hi[l], c[l] + 1);
    }
}

// reduce the per-thread boxes of a block into ctl->dep box `slot`
__device__ inline void box_flush(const RunDev &R, Box &bx, int slot)
{
    __shared__ int sh[6];
    if (threadIdx.x < 3) {
        sh[threadIdx.x] = 0x7fffffff;
        sh[3 + threadIdx.x] = -1;
    }
    __syncthreads();
    for (int l = 0; l < 3; ++l) {
        if (bx.hi[l] >= 0) {
            atomicMin(&sh[l], bx.lo[l]);
            atomicMax(&sh[3 + l], bx.hi[l]);
        }
    }
    __syncthreads();
    if (threadIdx.x < 3 && sh[3 + threadIdx.x] >= 0) {
        atomicMin(&R.ctl->dep_lo[slot][threadIdx.x], sh[threadIdx.x]);
        atomicMax(&R.ctl->dep_hi[slot][threadIdx.x], sh[3 + threadIdx.x]);
    }
}

// K4: gather + undulator + N_b Boris sub-steps + deposit of J^{n+1} and
// rho^{n+3/2} into source set (n+1) & 1.
template <typename T, bool COMP>
__global__ __launch_bounds__(256) void k_push_deposit(RunDev R)
{
    const int64_t s = R.ctl->step;
    const int pb = R.ctl->pbuf;
    const int set = (int)((s + 1) & 1);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Box bx;
    for (int l = 0; l < 3; ++l) {
        bx.lo[l] = 0x7fffffff;
        bx.hi[l] = -1;
    }
    if (p < R.np) {
        double r[3], u[3];
        for (int a = 0; a < 3; ++a) {
            r[a] = R.pr[pb][a][p];
            u[a] = R.pr[pb][3 + a][p];
        }
        double g1[3];
        int c1[3];
        const bool act1 = cell_of(R, r, g1, c1);
        double Eg[3] = {0, 0, 0}, Bg[3] = {0, 0, 0};
        if (act1) {
            const int64_t base = nid(R, c1[0], c1[1], c1[2]);
            const int64_t sy = R.nx, sz = (int64_t)R.nx * R.ny;
            const double dx = g1[0] - c1[0], dy = g1[1] - c1[1], dz = g1[2] - c1[2];
            const double wx[2] = {1.0 - dx, dx}, wy[2] = {1.0 - dy, dy}, wz[2] = {1.0 - dz, dz};
            for (int K = 0; K < 2; ++K)
                for (int J = 0; J < 2; ++J)
                    for (int I = 0; I < 2; ++I) {
                        const double w = wx[I] * wy[J] * wz[K];
                        const int64_t n = base + I + J * sy + K * sz;
                        for (int a = 0; a < 3; ++a) {
                            Eg[a] += w * (double)eb_ptr<T>(R, a)[n];
                            Bg[a] += w * (double)eb_ptr<T>(R, 3 + a)[n];
                        }
                    }
        }
        const double t_half = ((double)s + 0.5) * R.dt;
        for (int sub = 0; sub < R.n_sub; ++sub) {
            double Ee[3], Be[3];
            undulator_field(R, r[0], r[1], r[2], t_half + (double)sub * R.dtb, Ee, Be);
            for (int a = 0; a < 3; ++a) {
                Ee[a] += Eg[a];
                Be[a] += Bg[a];
            }
            boris(u, Ee, Be, R.dtb);
            const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int a = 0; a < 3; ++a)
                r[a] = r[a] + kC * R.dtb * u[a] * ig;
        }
        for (int a = 0; a < 3; ++a) {
            R.pr[pb][a][p] = r[a];
            R.pr[pb][3 + a][p] = u[a];
        }
        double g2[3];
        int c2[3];
        const bool act2 = cell_of(R, r, g2, c2);
        const Acc<T, COMP> acc = make_acc<T, COMP>(R, set);
        if (act1 && act2)
            deposit_move<T, COMP>(R, acc, g1, c1, g2, c2, bx);
        if (act2)
            deposit_charge<T, COMP>(R, acc, g2, c2, bx);
    }
    box_flush(R, bx, set);
}

// Load: first current from the backward drift r - c dt u/gamma -> r and
// charge at r, into source set 0 (particles in buffer 0, id order).
template <typename T, bool COMP>
__global__ __launch_bounds__(256) void k_load_deposit(RunDev R)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Box bx;
    for (int l = 0; l < 3; ++l) {
        bx.lo[l] = 0x7fffffff;
        bx.hi[l] = -1;
    }
    if (p < R.np) {
        double r[3], u[3], r0[3];
        for (int a = 0; a < 3; ++a) {
            r[a] = R.pr[0][a][p];
            u[a] = R.pr[0][3 + a][p];
        }
        const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int a = 0; a < 3; ++a)
            r0[a] = r[a] - kC * R.dt * u[a] * ig;
        double g1[3], g2[3];
        int c1[3], c2[3];
        const bool act1 = cell_of(R, r0, g1, c1);
        const bool act2 = cell_of(R, r, g2, c2);
        const Acc<T, COMP> acc = make_acc<T, COMP>(R, 0);
        if (act1 && act2)
            deposit_move<T, COMP>(R, acc, g1, c1, g2, c2, bx);
        if (act2)
            deposit_charge<T, COMP>(R, acc, g2, c2, bx);
    }
    box_flush(R, bx, 0);
}

// |sum exp(i k_r z)| over active particles, in two partial sums per block
__global__ __launch_bounds__(256) void k_bunching(RunDev R, double *part)
{
    __shared__ double sr[256], si[256], sn[256];
    const int pb = R.ctl->pbuf;
    const double kr = R.ku * R.gamma0 * R.beta0;
    double re = 0, im = 0, n = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < R.np; p += (int64_t)gridDim.x * blockDim.x) {
        double r[3] = {R.pr[pb][0][p], R.pr[pb][1][p], R.pr[pb][2][p]}, g[3];
        int c[3];
        if (cell_of(R, r, g, c)) {
            double sv, cv;
            sincos(kr * r[2], &sv, &cv);
            re += cv;
            im += sv;
            n += 1.0;
        }
    }
    sr[threadIdx.x] = re;
    si[threadIdx.x] = im;
    sn[threadIdx.x] = n;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
            sn[threadIdx.x] += sn[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = sr[0];
        part[3 * blockIdx.x + 1] = si[0];
        part[3 * blockIdx.x + 2] = sn[0];
    }
}

// ---------------------------------------------------------------------------

hipError_t launch_push_deposit(const RunDev &R, hipStream_t st)
{
    if (R.np <= 0)
        return hipSuccess;
    const unsigned blocks = (unsigned)((R.np + 255) / 256);
    if (R.precision == 64)
        hipLaunchKernelGGL((k_push_deposit<double, false>), dim3(blocks), dim3(256), 0, st, R);
    else if (R.compensated)
        hipLaunchKernelGGL((k_push_deposit<float, true>), dim3(blocks), dim3(256), 0, st, R);
    else
        hipLaunchKernelGGL((k_push_deposit<float, false>), dim3(blocks), dim3(256), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_load_deposit(const RunDev &R, hipStream_t st)
{
    const unsigned blocks = (unsigned)((R.np + 255) / 256);
    if (R.precision == 64)
        hipLaunchKernelGGL((k_load_deposit<double, false>), dim3(blocks), dim3(256), 0, st, R);
    else if (R.compensated)
        hipLaunchKernelGGL((k_load_deposit<float, true>), dim3(blocks), dim3(256), 0, st, R);
    else
        hipLaunchKernelGGL((k_load_deposit<float, false>), dim3(blocks), dim3(256), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_bunching(const RunDev &R, double *part, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_bunching, dim3(blocks), dim3(256), 0, st, R, part);
    return hipGetLastError();
}

}  // namespace mithra
