// k_tiles.hip -- tile-owned particle step.
//
// After each sort the particles of an occupied sort tile are contiguous.
// `k_tile_items` cuts the sorted active prefix into work items: one per tile,
// or several chunks of at most kTileChunk particles for crowded tiles.  The
// persistent kernel `k_tile_step` takes items from a device-side counter;
// for each item it
//   1. evaluates E and B at the tile's (T+1)^3 vertices straight from the
//      potentials into LDS (E = -(A^{n+1} - A^n)/dt - grad phi, B = mean of
//      curl A^n and curl A^{n+1}; MITHRA 2.0 manual, sec. "Field
//      Evaluation"),
//   2. pushes its particles: trilinear gather from LDS, undulator field,
//      N_b Boris sub-steps, new sort key,
//   3. deposits the zigzag currents and CIC charge of each move into an LDS
//      box covering the tile plus one node on every side (a particle moves
//      less than one cell per step), and
//   4. adds the non-zero LDS entries to HBM: one atomic per touched node and
//      array instead of one per particle contribution.
// Particles outside the active region (sorted last) take the undulator
// field only, in `k_push_inactive`.
#include "particle_dev.hpp"

namespace mithra {

constexpr int kTileThreads = 256;
constexpr int kTileChunk = 512;
constexpr int kEBCap = 729;    // vertices of the largest tile staged: (Tx+1)(Ty+1)(Tz+1)
constexpr int kAccCap = 1331;  // nodes of its deposit box: (Tx+3)(Ty+3)(Tz+3)

bool tile_kernel_fits(const int tile[3])
{
    return (tile[0] + 1) * (tile[1] + 1) * (tile[2] + 1) <= kEBCap &&
           (tile[0] + 3) * (tile[1] + 3) * (tile[2] + 3) <= kAccCap;
}

// items from the sorted keys of the active prefix [0, n_active)
__global__ __launch_bounds__(256) void k_tile_items(RunDev R)
{
    const int64_t n = R.ctl->n_active;
    const uint32_t tvol = (uint32_t)(R.tile[0] * R.tile[1] * R.tile[2]);
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = R.key_sorted[r] / tvol;
        if (r > 0 && R.key_sorted[r - 1] / tvol == t)
            continue;
        int64_t lo = r + 1, hi = n;  // first index whose tile is beyond t
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (R.key_sorted[mid] / tvol <= t)
                lo = mid + 1;
            else
                hi = mid;
        }
        const int64_t end = lo;
        const int nch = (int)((end - r + kTileChunk - 1) / kTileChunk);
        const int slot = atomicAdd(&R.ctl->n_items, nch);
        for (int c = 0; c < nch && slot + c < R.item_cap; ++c) {
            int32_t *it = R.items + 4 * (int64_t)(slot + c);
            it[0] = (int32_t)t;
            it[1] = (int32_t)(r + (int64_t)c * kTileChunk);
            it[2] = (int32_t)min(end, r + (int64_t)(c + 1) * kTileChunk);
            it[3] = 0;
        }
    }
}

template <typename T>
__device__ inline void tile_vertex_eb(const RunDev &R, int64_t s, int i, int j, int k, double E[3], double B[3])
{
    const T *An[3], *Ap[3];
    for (int c = 0; c < 3; ++c) {
        An[c] = pot_ptr<T>(R, slot_cur(s), c);
        Ap[c] = pot_ptr<T>(R, slot_next(s), c);
    }
    const int64_t c0 = nid(R, i, j, k);
    const int64_t sx = 1, sy = R.nx, sz = (int64_t)R.nx * R.ny;
    const double i2x = 0.5 / R.dx, i2y = 0.5 / R.dy, i2z = 0.5 / R.dz;
    auto dif = [&](const T *a, int64_t st) { return (double)a[c0 + st] - (double)a[c0 - st]; };
    B[0] = 0.5 * ((dif(An[2], sy) + dif(Ap[2], sy)) * i2y - (dif(An[1], sz) + dif(Ap[1], sz)) * i2z);
    B[1] = 0.5 * ((dif(An[0], sz) + dif(Ap[0], sz)) * i2z - (dif(An[2], sx) + dif(Ap[2], sx)) * i2x);
    B[2] = 0.5 * ((dif(An[1], sx) + dif(Ap[1], sx)) * i2x - (dif(An[0], sy) + dif(Ap[0], sy)) * i2y);
    double g[3] = {0.0, 0.0, 0.0};
    if (R.space_charge) {
        const T *ph = pot_ptr<T>(R, slot_cur(s), 3);
        g[0] = dif(ph, sx) * i2x;
        g[1] = dif(ph, sy) * i2y;
        g[2] = dif(ph, sz) * i2z;
    }
    for (int c = 0; c < 3; ++c)
        E[c] = -((double)Ap[c][c0] - (double)An[c][c0]) / R.dt - g[c];
}

// MODE 0: step; MODE 1: load deposit (backward-drift move, source set 0).
// T: field storage; AccT: LDS accumulator (float only for FP32 without
// compensation).
template <typename T, typename AccT, bool COMP, int MODE>
__global__ __launch_bounds__(kTileThreads) void k_tile_step(RunDev R)
{
    __shared__ T ebs[6 * kEBCap];
    __shared__ AccT acc[4 * kAccCap];
    __shared__ int item_s;
    __shared__ int32_t cw[kTileThreads / 64][7];

    const int64_t s = R.ctl->step;
    const int pb = R.ctl->pbuf;
    const int set = MODE == 0 ? (int)((s + 1) & 1) : 0;
    const int Tx = R.tile[0], Ty = R.tile[1], Tz = R.tile[2];
    const int ex = Tx + 1, ey = Ty + 1, ez = Tz + 1, veb = ex * ey * ez;
    const int ax = Tx + 3, ay = Ty + 3, az = Tz + 3, vacc = ax * ay * az;
    const int n[3] = {R.nx, R.ny, R.nz};
    const int n_items = min((int64_t)R.ctl->n_items, R.item_cap);
    const GlobalAcc<T, COMP> gacc = make_gacc<T, COMP>(R, set);

    // block statistics: deposit box (conservative, per item) and active cells
    int dlo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, dhi[3] = {-1, -1, -1};
    int clo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, chi[3] = {-1, -1, -1};
    int nact = 0;

    for (;;) {
        if (threadIdx.x == 0)
            item_s = atomicAdd(&R.ctl->item_next, 1);
        __syncthreads();
        const int it = item_s;
        if (it >= n_items)
            break;
        const int32_t *itm = R.items + 4 * (int64_t)it;
        const int t = itm[0], beg = itm[1], end = itm[2];
        const int c0[3] = {(t % R.ntile[0]) * Tx, ((t / R.ntile[0]) % R.ntile[1]) * Ty,
                           (t / (R.ntile[0] * R.ntile[1])) * Tz};
        // the item's particles are sorted by key, whose slowest local digit
        // is the z plane of the cell inside the tile: they occupy local
        // planes kz0..kz1 only
        const uint32_t tv = (uint32_t)(Tx * Ty * Tz), txy = (uint32_t)(Tx * Ty);
        const int kz0 = (int)((R.key_sorted[beg] % tv) / txy);
        const int kz1 = (int)((R.key_sorted[end - 1] % tv) / txy);
        // 1. vertex fields of the occupied planes (vertex planes kz0..kz1+1)
        if (MODE == 0) {
            const int eb0 = kz0 * ex * ey, eb1 = (kz1 + 2) * ex * ey;
#pragma unroll 1
            for (int e = eb0 + threadIdx.x; e < eb1; e += kTileThreads) {
                const int li = e % ex, lj = (e / ex) % ey, lk = e / (ex * ey);
                const int i = c0[0] + li, j = c0[1] + lj, k = c0[2] + lk;
                double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
                if (i >= 1 && i <= n[0] - 2 && j >= 1 && j <= n[1] - 2 && k >= 1 && k <= n[2] - 2)
                    tile_vertex_eb<T>(R, s, i, j, k, E, B);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    ebs[a * kEBCap + e] = (T)E[a];
                    ebs[(3 + a) * kEBCap + e] = (T)B[a];
                }
            }
        }
        // deposit box planes: cells kz0-1 .. kz1+1 touch node planes
        // kz0-1 .. kz1+2, i.e. local acc planes kz0 .. kz1+3
        const int ap0 = kz0, ap1 = kz1 + 4;  // [ap0, ap1)
        const int aplane = ax * ay;
        for (int comp = 0; comp < 4; ++comp)
            for (int e = ap0 * aplane + threadIdx.x; e < ap1 * aplane; e += kTileThreads)
                acc[comp * vacc + e] = (AccT)0;
        __syncthreads();
        // 2.-3. particles
        const LdsAcc<AccT> lacc{acc, c0[0] - 1, c0[1] - 1, c0[2] - 1, ax, ay, vacc};
#pragma unroll 1
        for (int p = beg + threadIdx.x; p < end; p += kTileThreads) {
            double r[3], u[3], g1[3], g2[3];
            int c1[3], c2[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                r[a] = R.pr[pb][a][p];
                u[a] = R.pr[pb][3 + a][p];
            }
            bool act1, act2;
            if (MODE == 1) {
                const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                double r0[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    r0[a] = r[a] - kC * R.dt * u[a] * ig;
                act1 = cell_of(R, r0, g1, c1);
                act2 = cell_of(R, r, g2, c2);
            } else {
                act1 = cell_of(R, r, g1, c1);  // true: the item holds active particles of this tile
                bool intile = act1;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    intile = intile && c1[a] >= c0[a] && c1[a] < c0[a] + R.tile[a];
                double Eg[3] = {0, 0, 0}, Bg[3] = {0, 0, 0};
                if (intile) {
                const double dx = g1[0] - c1[0], dy = g1[1] - c1[1], dz = g1[2] - c1[2];
                const double wx[2] = {1.0 - dx, dx}, wy[2] = {1.0 - dy, dy}, wz[2] = {1.0 - dz, dz};
                const int b0 = ((c1[2] - c0[2]) * ey + (c1[1] - c0[1])) * ex + (c1[0] - c0[0]);
                // (the sort put this particle in tile t, so its cell is inside)
#pragma unroll
                for (int K = 0; K < 2; ++K)
#pragma unroll
                    for (int J = 0; J < 2; ++J)
#pragma unroll
                        for (int I = 0; I < 2; ++I) {
                            const double w = wx[I] * wy[J] * wz[K];
                            const int e = b0 + I + J * ex + K * ex * ey;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                Eg[a] += w * (double)ebs[a * kEBCap + e];
                                Bg[a] += w * (double)ebs[(3 + a) * kEBCap + e];
                            }
                        }
                }
                const double t_half = ((double)s + 0.5) * R.dt;
                for (int sub = 0; sub < R.n_sub; ++sub) {
                    double Ee[3], Be[3];
                    undulator_field(R, r[0], r[1], r[2], t_half + (double)sub * R.dtb, Ee, Be);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        Ee[a] += Eg[a];
                        Be[a] += Bg[a];
                    }
                    boris(u, Ee, Be, R.dtb);
                    const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        r[a] = r[a] + kC * R.dtb * u[a] * ig;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    R.pr[pb][a][p] = r[a];
                    R.pr[pb][3 + a][p] = u[a];
                }
                act2 = cell_of(R, r, g2, c2);
                const int32_t id = R.pid[pb][p];
                R.key_by_id[id] = act2 ? key_of_cell(R, c2) : R.key_inactive;
                R.slot_of_id[id] = (int32_t)p;
                if (act2) {
                    ++nact;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        clo[a] = min(clo[a], c2[a]);
                        chi[a] = max(chi[a], c2[a]);
                    }
                }
            }
            // the zeroed part of the deposit box holds cells c0-1 .. c0+T
            // across and kz0-1 .. kz1+1 along z (one cell of motion)
            bool inbox = c1[2] >= c0[2] + kz0 - 1 && c1[2] <= c0[2] + kz1 + 1 && c2[2] >= c0[2] + kz0 - 1 &&
                         c2[2] <= c0[2] + kz1 + 1;
#pragma unroll
            for (int a = 0; a < 2; ++a)
                inbox = inbox && c1[a] >= c0[a] - 1 && c1[a] <= c0[a] + R.tile[a] && c2[a] >= c0[a] - 1 &&
                        c2[a] <= c0[a] + R.tile[a];
            if (inbox) {
                if (act1 && act2)
                    deposit_move(R, lacc, g1, c1, g2, c2);
                if (act2)
                    deposit_charge(R, lacc, g2, c2);
            } else {
                if (act1 && act2)
                    deposit_move(R, gacc, g1, c1, g2, c2);
                if (act2)
                    deposit_charge(R, gacc, g2, c2);
                for (int a = 0; a < 3; ++a) {
                    if (act2) {
                        dlo[a] = min(dlo[a], act1 ? min(c1[a], c2[a]) : c2[a]);
                        dhi[a] = max(dhi[a], (act1 ? max(c1[a], c2[a]) : c2[a]) + 1);
                    }
                }
            }
        }
        __syncthreads();
        // 4. add the touched planes of the box to HBM
        const int span = (ap1 - ap0) * aplane;
#pragma unroll 1
        for (int e0 = threadIdx.x; e0 < 4 * span; e0 += 4 * kTileThreads) {
            double v[4];
            int idx[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + q * kTileThreads;
                const int comp = e / span;
                const int r = e - comp * span + ap0 * aplane;
                v[q] = e < 4 * span ? (double)acc[comp * vacc + r] : 0.0;
                idx[q][0] = comp;
                idx[q][1] = c0[0] - 1 + r % ax;
                idx[q][2] = c0[1] - 1 + (r / ax) % ay;
                idx[q][3] = c0[2] - 1 + r / aplane;
            }
            gacc.add4(v, idx);
        }
        dlo[0] = min(dlo[0], max(1, c0[0] - 1));
        dhi[0] = max(dhi[0], min(n[0] - 2, c0[0] + Tx + 1));
        dlo[1] = min(dlo[1], max(1, c0[1] - 1));
        dhi[1] = max(dhi[1], min(n[1] - 2, c0[1] + Ty + 1));
        dlo[2] = min(dlo[2], max(1, c0[2] + kz0 - 1));
        dhi[2] = max(dhi[2], min(n[2] - 2, c0[2] + kz1 + 2));
        __syncthreads();
    }
    // per-block partials: deposit box (boxpart) and active cells (cellpart)
    for (int a = 0; a < 3; ++a) {
        clo[a] = wave_min(clo[a]);
        chi[a] = wave_max(chi[a]);
    }
    for (int o = 32; o > 0; o >>= 1)
        nact += __shfl_xor(nact, o);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 3; ++a) {
            cw[wave][a] = clo[a];
            cw[wave][3 + a] = chi[a];
        }
        cw[wave][6] = nact;
    }
    // deposit box: thread-uniform except for the rare out-of-box moves
    for (int a = 0; a < 3; ++a) {
        dlo[a] = wave_min(dlo[a]);
        dhi[a] = wave_max(dhi[a]);
    }
    __shared__ int32_t dw[kTileThreads / 64][6];
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            dw[wave][a] = dlo[a];
            dw[wave][3 + a] = dhi[a];
        }
    __syncthreads();
    if (threadIdx.x < 7) {
        int32_t v = cw[0][threadIdx.x];
        for (int w = 1; w < kTileThreads / 64; ++w) {
            const int32_t x = cw[w][threadIdx.x];
            v = threadIdx.x < 3 ? min(v, x) : (threadIdx.x < 6 ? max(v, x) : v + x);
        }
        R.cellpart[8 * (int64_t)blockIdx.x + threadIdx.x] = v;
    }
    if (threadIdx.x < 7) {
        int32_t v = threadIdx.x < 6 ? dw[0][threadIdx.x] : 0;
        for (int w = 1; w < kTileThreads / 64 && threadIdx.x < 6; ++w) {
            const int32_t x = dw[w][threadIdx.x];
            v = threadIdx.x < 3 ? min(v, x) : max(v, x);
        }
        R.boxpart[8 * (int64_t)blockIdx.x + threadIdx.x] = v;
    }
}

// particles outside the active region at the last sort: undulator field
// only; a particle that enters the active region deposits its charge (its
// old cell is inactive, so it carries no current this step).  Partials go
// after the tile kernel's.
template <typename T, bool COMP>
__global__ __launch_bounds__(256) void k_push_inactive(RunDev R, int part_base)
{
    __shared__ int32_t cw[4][7];
    __shared__ int32_t dw[4][6];
    const int64_t s = R.ctl->step;
    const int pb = R.ctl->pbuf;
    const GlobalAcc<T, COMP> gacc = make_gacc<T, COMP>(R, (int)((s + 1) & 1));
    int clo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, chi[3] = {-1, -1, -1};
    int dlo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, dhi[3] = {-1, -1, -1};
    int nact = 0;
    const double t_half = ((double)s + 0.5) * R.dt;
    for (int64_t p = R.ctl->sorted_active + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < R.np;
         p += (int64_t)gridDim.x * blockDim.x) {
        double r[3], u[3], g2[3];
        int c2[3];
        for (int a = 0; a < 3; ++a) {
            r[a] = R.pr[pb][a][p];
            u[a] = R.pr[pb][3 + a][p];
        }
        for (int sub = 0; sub < R.n_sub; ++sub) {
            double Ee[3], Be[3];
            undulator_field(R, r[0], r[1], r[2], t_half + (double)sub * R.dtb, Ee, Be);
            boris(u, Ee, Be, R.dtb);
            const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int a = 0; a < 3; ++a)
                r[a] = r[a] + kC * R.dtb * u[a] * ig;
        }
        for (int a = 0; a < 3; ++a) {
            R.pr[pb][a][p] = r[a];
            R.pr[pb][3 + a][p] = u[a];
        }
        const bool act2 = cell_of(R, r, g2, c2);
        const int32_t id = R.pid[pb][p];
        R.key_by_id[id] = act2 ? key_of_cell(R, c2) : R.key_inactive;
        R.slot_of_id[id] = (int32_t)p;
        if (act2) {
            ++nact;
            deposit_charge(R, gacc, g2, c2);
            for (int a = 0; a < 3; ++a) {
                clo[a] = min(clo[a], c2[a]);
                chi[a] = max(chi[a], c2[a]);
                dlo[a] = min(dlo[a], c2[a]);
                dhi[a] = max(dhi[a], c2[a] + 1);
            }
        }
    }
    for (int a = 0; a < 3; ++a) {
        clo[a] = wave_min(clo[a]);
        chi[a] = wave_max(chi[a]);
        dlo[a] = wave_min(dlo[a]);
        dhi[a] = wave_max(dhi[a]);
    }
    for (int o = 32; o > 0; o >>= 1)
        nact += __shfl_xor(nact, o);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 3; ++a) {
            cw[wave][a] = clo[a];
            cw[wave][3 + a] = chi[a];
            dw[wave][a] = dlo[a];
            dw[wave][3 + a] = dhi[a];
        }
        cw[wave][6] = nact;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        int32_t v = cw[0][threadIdx.x];
        int32_t b = threadIdx.x < 6 ? dw[0][threadIdx.x] : 0;
        for (int w = 1; w < 4; ++w) {
            const int32_t x = cw[w][threadIdx.x];
            v = threadIdx.x < 3 ? min(v, x) : (threadIdx.x < 6 ? max(v, x) : v + x);
            if (threadIdx.x < 6)
                b = threadIdx.x < 3 ? min(b, dw[w][threadIdx.x]) : max(b, dw[w][threadIdx.x]);
        }
        R.cellpart[8 * (int64_t)(part_base + blockIdx.x) + threadIdx.x] = v;
        R.boxpart[8 * (int64_t)(part_base + blockIdx.x) + threadIdx.x] = b;
    }
}

// ---------------------------------------------------------------------------

constexpr int kInactiveBlocks = 64;

template <int MODE>
static hipError_t launch_tile_t(const RunDev &R, hipStream_t st)
{
    const dim3 g((unsigned)R.tile_grid), b(kTileThreads);
    if (R.precision == 64)
        hipLaunchKernelGGL((k_tile_step<double, double, false, MODE>), g, b, 0, st, R);
    else if (R.compensated)
        hipLaunchKernelGGL((k_tile_step<float, double, true, MODE>), g, b, 0, st, R);
    else
        hipLaunchKernelGGL((k_tile_step<float, float, false, MODE>), g, b, 0, st, R);
    return hipGetLastError();
}

int tile_partials(const RunDev &R) { return R.tile_grid + kInactiveBlocks; }

hipError_t launch_tile_items(const RunDev &R, hipStream_t st)
{
    int64_t blocks = (R.np + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_tile_items, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_tile_step(const RunDev &R, hipStream_t st)
{
    hipError_t e = launch_tile_t<0>(R, st);
    if (e != hipSuccess)
        return e;
    if (R.precision == 64)
        hipLaunchKernelGGL((k_push_inactive<double, false>), dim3(kInactiveBlocks), dim3(256), 0, st, R, R.tile_grid);
    else if (R.compensated)
        hipLaunchKernelGGL((k_push_inactive<float, true>), dim3(kInactiveBlocks), dim3(256), 0, st, R, R.tile_grid);
    else
        hipLaunchKernelGGL((k_push_inactive<float, false>), dim3(kInactiveBlocks), dim3(256), 0, st, R, R.tile_grid);
    return hipGetLastError();
}

hipError_t launch_tile_load(const RunDev &R, hipStream_t st) { return launch_tile_t<1>(R, st); }

int tile_blocks_per_cu(int precision, int compensated)
{
    int nb = 0;
    hipError_t e;
    if (precision == 64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile_step<double, double, false, 0>, kTileThreads, 0);
    else if (compensated)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile_step<float, double, true, 0>, kTileThreads, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile_step<float, float, false, 0>, kTileThreads, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace mithra
