// k_particles.hip -- the particle step (gather, external field, Boris
// push, deposit), box reductions, the bunching diagnostic and the Halton
// bunch generator.  Particles are processed in the order of the last sort;
// each block sums its deposits in LDS over the node box its particles touch
// and adds that box to HBM once, or adds directly when the box does not
// fit.
#include "particle_dev.hpp"
#include "mur_dev.hpp"

namespace mithra {

// node box capacity of the LDS stage (4 arrays, FP64: 51.6 KiB): the most
// that lets three workgroups share a CU's 160 KiB of LDS (1536 nodes: the
// widest phase of the FEL amplifier's envelope ran 195 against 186 us, its
// blocks' boxes overflowing more often)
constexpr int kLdsNodes = 1650;

// Gather + undulator + N_b Boris sub-steps + deposit (MODE 0), or the load
// deposit of the backward-drift move (MODE 1, set 0).  Rank p handles the
// particle in slot sv[sorted_buf][p] of buffer pbuf (the last sort's order);
// MODE 0 writes the pushed state to rank p of the other buffer (the step's
// last bookkeeping kernel flips pbuf), so the sort never moves the state.
// The block's deposits are summed in LDS over its node box when the box
// fits, then added to HBM once per touched node; otherwise directly.
// EXT selects the general external field (undulator arrays, optical
// undulators); the single static module keeps its own path.
template <typename T, bool COMP, int MODE, bool EXT = false>
struct PushDeposit {
    // The block's box accumulates in FP64 LDS whatever the source precision
    // (an FP32 box measured 367 against 225 us per launch at the FEL
    // amplifier).  Three waves per SIMD: the push needs about 160 VGPRs (at
    // 128 it spills), and the box allows three blocks per CU.  The general
    // external field (arrays, optical undulators) needs about 210: two
    // waves, where three spilled about 50 registers per lane.
    using LT = double;
    static constexpr int kThreads = kDepThreads;
    static constexpr int kWaves = EXT ? 2 : 3;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        __shared__ LT lds[4 * kLdsNodes];
        __shared__ int bb[7];  // node box lo[3], hi[3]; active count
        const int64_t s = R.ctl->step;
        const int pb = R.ctl->pbuf;
        const int set = MODE == 0 ? (int)((s + 1) & 1) : 0;
        const int64_t p = (int64_t)blk.id * blockDim.x + threadIdx.x;
        if (threadIdx.x < 3) {
            bb[threadIdx.x] = 0x7fffffff;
            bb[3 + threadIdx.x] = -1;
        }
        if (threadIdx.x == 3)
            bb[6] = 0;

        double g1[3] = {0, 0, 0}, g2[3] = {0, 0, 0};
        int c1[3] = {0, 0, 0}, c2[3] = {0, 0, 0};
        bool dep_j = false, dep_q = false;
        if (p < R.np) {
            // rank p of the last sort: the slot where the previous push (or
            // the load) left the particle, and its id
            const int sb = R.ctl->sorted_buf;
            const int32_t src = sb < 0 ? (int32_t)p : R.sv[sb][p];
            const int32_t id = R.pid[pb][src];
            double r[3], u[3];
            for (int a = 0; a < 3; ++a) {
                r[a] = R.pr[pb][a][src];
                u[a] = R.pr[pb][3 + a][src];
            }
            if (MODE == 1) {
                const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                double r0[3];
                for (int a = 0; a < 3; ++a)
                    r0[a] = r[a] - kC * R.dt * u[a] * ig;
                const bool a1 = cell_of(R, r0, g1, c1);
                const bool a2 = cell_of(R, r, g2, c2);
                dep_j = a1 && a2;
                dep_q = a2;
                if (a2)  // the vertex fields of this step are needed around this cell
                    R.tile_flag[tile_of_cell(R, c2)] = (uint32_t)s;
            } else {
                const bool act1 = cell_of(R, r, g1, c1);
                double Eg[3] = {0, 0, 0}, Bg[3] = {0, 0, 0};
                if (act1) {
                    const int64_t base = nid(R, c1[0], c1[1], c1[2]);
                    const int64_t sy = R.nx, sz = (int64_t)R.nx * R.ny;
                    const double dx = g1[0] - c1[0], dy = g1[1] - c1[1], dz = g1[2] - c1[2];
                    const double wx[2] = {1.0 - dx, dx}, wy[2] = {1.0 - dy, dy}, wz[2] = {1.0 - dz, dz};
    #pragma unroll
                    for (int K = 0; K < 2; ++K)
    #pragma unroll
                        for (int J = 0; J < 2; ++J)
    #pragma unroll
                            for (int I = 0; I < 2; ++I) {
                                const double w = wx[I] * wy[J] * wz[K];
                                const int64_t n = base + I + J * sy + K * sz;
                                // the corner's six words: 2 (FP32) or 3 (FP64) 16-byte loads
                                constexpr int V = 16 / sizeof(T);
                                const T *q = eb_node<T>(R, n);
                                T f[6 + (V == 4 ? 2 : 0)];
    #pragma unroll
                                for (int h = 0; h < (6 + V - 1) / V; ++h) {
                                    const Vec<T, V> x = vload<T, V>(q + h * V);
    #pragma unroll
                                    for (int e = 0; e < V; ++e)
                                        f[h * V + e] = x.v[e];
                                }
    #pragma unroll
                                for (int a = 0; a < 3; ++a) {
                                    Eg[a] += w * (double)f[a];
                                    Bg[a] += w * (double)f[3 + a];
                                }
                            }
                }
                const double t_half = ((double)s + 0.5) * R.dt;
                for (int sub = 0; sub < R.n_sub; ++sub) {
                    double Ee[3], Be[3];
                    external_field<EXT>(R, r[0], r[1], r[2], t_half + (double)sub * R.dtb, Ee, Be);
                    for (int a = 0; a < 3; ++a) {
                        Ee[a] += Eg[a];
                        Be[a] += Bg[a];
                    }
                    boris(u, Ee, Be, R.dtb);
                    const double ig = 1.0 / sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                    for (int a = 0; a < 3; ++a)
                        r[a] = r[a] + kC * R.dtb * u[a] * ig;
                }
                // the pushed state goes to the other buffer in sort order
                const int nb = pb ^ 1;
                for (int a = 0; a < 3; ++a) {
                    R.pr[nb][a][p] = r[a];
                    R.pr[nb][3 + a][p] = u[a];
                }
                R.pid[nb][p] = id;
                const bool act2 = cell_of(R, r, g2, c2);
                dep_j = act1 && act2;
                dep_q = act2;
                // sort key of the new position at rank p, for the sort after
                // this push (when there is one): the sort is stable, so ties
                // keep this step's order
                if (R.sort_every == 1 || (s + 1) % R.sort_every == 0) {
                    R.key_in[p] = act2 ? key_of_cell(R, c2) : R.key_inactive;
                    R.slot_in[p] = (int32_t)p;
                }
                if (act2)  // the next step's vertex fields are needed around this cell
                    R.tile_flag[tile_of_cell(R, c2)] = (uint32_t)(s + 1);
            }
        }
        // node box of this thread's deposits
        int lo[3], hi[3];
        for (int l = 0; l < 3; ++l) {
            lo[l] = 0x7fffffff;
            hi[l] = -1;
            if (dep_j) {
                lo[l] = min(c1[l], c2[l]);
                hi[l] = max(c1[l], c2[l]) + 1;
            } else if (dep_q) {
                lo[l] = c2[l];
                hi[l] = c2[l] + 1;
            }
            lo[l] = wave_min(lo[l]);
            hi[l] = wave_max(hi[l]);
        }
        // active particles after the push (sort statistics)
        const int nact = MODE == 0 ? (int)__popcll(__ballot(dep_q)) : 0;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            if (hi[0] >= 0)
                for (int l = 0; l < 3; ++l) {
                    atomicMin(&bb[l], lo[l]);
                    atomicMax(&bb[3 + l], hi[l]);
                }
            if (nact != 0)
                atomicAdd(&bb[6], nact);
        }
        __syncthreads();
        // this block's box: the push reduces it into its slot (BoxReduceStep),
        // the load deposit writes its partial (k_box_reduce)
        if (MODE == 0) {
            int32_t *slot = R.boxslot + 16 * (blk.id & (kBoxSlots - 1));
            if (threadIdx.x < 6 && bb[3] >= 0) {
                if (threadIdx.x < 3)
                    atomicMin(&slot[threadIdx.x], bb[threadIdx.x]);
                else
                    atomicMax(&slot[threadIdx.x], bb[threadIdx.x]);
            } else if (threadIdx.x == 6 && bb[6] != 0) {
                atomicAdd(&slot[12], bb[6]);
            }
        } else if (threadIdx.x < 7) {
            R.boxpart[8 * (int64_t)blk.id + threadIdx.x] = threadIdx.x < 6 ? bb[threadIdx.x] : 0;
        }
        const int L0 = bb[0], L1 = bb[1], L2 = bb[2];
        if (bb[3] < 0)
            return;  // nothing deposited by this block (uniform)
        // the rows of this block's node box, grown by one node along every
        // axis, join the source row ranges of the set (read by the sweep)
        {
            const int ry = bb[4] - L1 + 2, rz = bb[5] - L2 + 2;
            int32_t *slo = R.srow_lo + (size_t)set * R.nz * R.ny;
            int32_t *shi = R.srow_hi + (size_t)set * R.nz * R.ny;
            const double iry = 1.0 / (double)ry;
            for (int64_t r = threadIdx.x; r < (int64_t)ry * rz; r += kDepThreads) {
                const int64_t rk = small_div(r, iry), rj = r - rk * ry;
                const int64_t row = (L2 + rk) * R.ny + (L1 + rj);
                atomicMin(&slo[row], L0);
                atomicMax(&shi[row], bb[3] + 1);
            }
        }
        const int ex = bb[3] - L0 + 1, ey = bb[4] - L1 + 1, ez = bb[5] - L2 + 1;
        const int vol = ex * ey * ez;
        const GlobalAcc<T, COMP> gacc = make_gacc<T, COMP>(R, set);
        // Zero an LDS box, deposit into it, then flush its nonzero nodes with
        // global atomics: one node per thread per round, its four components
        // together (so that the returning atomics of the compensated mode are
        // in flight together), the node's (i, j, k) decoded once for the four.
        // first / stride: this thread's share; sync orders the three phases.
        auto lds_deposit = [&](LT *base, int B0, int B1, int B2, int bx, int by, int bv, int first, int stride,
                               auto sync) {
            for (int e = first; e < 4 * bv; e += stride)
                base[e] = (LT)0;
            sync();
            const LdsAcc<LT> acc{base, B0, B1, B2, bx, by, bv};
            if (dep_j)
                deposit_move(R, acc, g1, c1, g2, c2);
            if (dep_q)
                deposit_charge(R, acc, g2, c2);
            sync();
            const double ibx = 1.0 / (double)bx, iby = 1.0 / (double)by;
            for (int e = first; e < bv; e += stride) {
                const int jk = small_div(e, ibx), i = e - jk * bx;
                const int k = small_div(jk, iby), j = jk - k * by;
                double v[4];
    #pragma unroll
                for (int q = 0; q < 4; ++q)
                    v[q] = (double)base[q * bv + e];
                const int c[3] = {B0 + i, B1 + j, B2 + k};
                gacc.add4(v, gacc.base(c));
            }
        };
        if (vol <= kLdsNodes) {
            lds_deposit(lds, L0, L1, L2, ex, ey, vol, threadIdx.x, kDepThreads, [] { __syncthreads(); });
        } else {
            // The block's particles straddle rows of sort tiles, so its box is
            // too large.  Each wavefront then uses a quarter of the LDS for its
            // own box (lo, hi: the wavefront's box, the same in every lane)
            // when that fits, and global atomics when it does not.  LDS
            // accesses of one wavefront complete in order; the fences keep the
            // compiler from moving them across the phases.
            constexpr int kWaveNodes = kLdsNodes / (kDepThreads / 64);
            const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
            if (hi[0] >= 0) {
                const int wx = hi[0] - lo[0] + 1, wy = hi[1] - lo[1] + 1, wz = hi[2] - lo[2] + 1;
                const int wvol = wx * wy * wz;
                if (wvol <= kWaveNodes) {
                    lds_deposit(lds + (size_t)wave * 4 * kWaveNodes, lo[0], lo[1], lo[2], wx, wy, wvol, lane, 64, [] {
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    });
                } else {
                    if (dep_j)
                        deposit_move(R, gacc, g1, c1, g2, c2);
                    if (dep_q)
                        deposit_charge(R, gacc, g2, c2);
                }
            }
        }
    }
};

// sum exp(i k_b z) and the count over active particles, three partial sums
// per block; k_b = gamma0 k_u (1 + beta0), the ponderomotive wavenumber of
// the forward radiation and the backward undulator (microbunches at rest in
// this frame)
__global__ __launch_bounds__(256) void k_bunching(RunDev R, double *part)
{
    __shared__ double sr[256], si[256], sn[256];
    const int pb = R.ctl->pbuf;
    const double kr = R.ku * R.gamma0 * (1.0 + R.beta0);
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
// Halton bunch generation.  Element j of sequence i: 1 minus the radical
// inverse of j in the base of the i-th prime.  One thread per particle;
// the slices of the shot noise are counted in a second pass (integer
// atomics: the counts do not depend on the order) and displaced in a
// third.
// ---------------------------------------------------------------------------

__device__ inline double halton_dev(int i, uint64_t j)
{
    const uint64_t b = (uint64_t)(i == 0 ? 2 : i == 1 ? 3 : i == 2 ? 5 : i == 3 ? 7 : i == 4 ? 11 : i == 5 ? 13
                                  : i == 6 ? 17 : i == 7 ? 19 : i == 8 ? 23 : 29);
    double scale = 1.0, x = 0.0;
    for (uint64_t k = j; k > 0; k /= b) {
        scale /= (double)b;
        x += (double)(k % b) * scale;
    }
    return 1.0 - x;
}

__device__ inline void halton_normal_dev(int ia, int ib, uint64_t j, double &c, double &s)
{
    const double r = sqrt(-2.0 * log(halton_dev(ia, j)));
    const double a = 2.0 * kPi * halton_dev(ib, j);
    c = r * cos(a);
    s = r * sin(a);
}

// pass 0: quiet-start coordinates, momenta and the bunching displacement
__global__ __launch_bounds__(256) void k_gen_bunch(RunDev R, GenParams P)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.n)
        return;
    const uint64_t j = (uint64_t)q;
    double x, y, zl, c, sn;
    if (P.trans_profile == 0) {
        x = P.sx * (halton_dev(0, j) - 0.5);
        y = P.sy * (halton_dev(1, j) - 0.5);
    } else {
        halton_normal_dev(0, 1, j, c, sn);
        x = P.sx * c;
        y = P.sy * sn;
    }
    if (P.long_profile == 1) {
        halton_normal_dev(2, 3, j, c, sn);
        zl = P.L * c;
    } else if (q < P.n_flat) {
        zl = P.L * (halton_dev(2, j) - 0.5);
    } else {
        halton_normal_dev(2, 3, j, c, sn);
        zl = (q & 1) ? 0.5 * P.L + P.sig_t * fabs(c) : -0.5 * P.L - P.sig_t * fabs(c);
    }
    halton_normal_dev(4, 5, j, c, sn);
    const double ge = P.gamma * (1.0 + P.sig_g * c);
    halton_normal_dev(6, 7, j, c, sn);
    const double ux = P.sig_u * c, uy = P.sig_u * sn;
    const double uzl = sqrt(ge * ge - 1.0 - ux * ux - uy * uy);
    double z = P.cz + zl * P.lz;
    if (P.bf != 0.0)
        z = z - (2.0 * P.bf / P.k) * sin(P.k * z + P.bphase);
    R.pr[0][0][q] = P.cx + x;
    R.pr[0][1][q] = P.cy + y;
    R.pr[0][2][q] = z;
    R.pr[0][3][q] = ux;
    R.pr[0][4][q] = uy;
    R.pr[0][5][q] = R.gamma0 * (uzl - R.beta0 * ge);
    R.pid[0][q] = (int32_t)q;
}

// smallest and largest z of the generated bunch (one block, fixed order)
__global__ __launch_bounds__(1024) void k_gen_zrange(RunDev R, int64_t n, double *out)
{
    __shared__ double lo[1024], hi[1024];
    double a = 1e300, b = -1e300;
    for (int64_t q = threadIdx.x; q < n; q += 1024) {
        const double z = R.pr[0][2][q];
        a = fmin(a, z);
        b = fmax(b, z);
    }
    lo[threadIdx.x] = a;
    hi[threadIdx.x] = b;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
            hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = lo[0];
        out[1] = hi[0];
    }
}

// pass 1: particles per shot-noise slice
__global__ __launch_bounds__(256) void k_gen_count(RunDev R, GenParams P)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.n)
        return;
    const int64_t sl = (int64_t)floor((R.pr[0][2][q] - P.zmin) / P.slice);
    atomicAdd(&P.counts[sl], 1);
}

// pass 2: the shot-noise displacement of each particle from its slice
__global__ __launch_bounds__(256) void k_gen_noise(RunDev R, GenParams P)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.n)
        return;
    const double z = R.pr[0][2][q];
    const int64_t sl = (int64_t)floor((z - P.zmin) / P.slice);
    const double ne = fmax((double)P.counts[sl] * P.n_e / (double)P.n, 1.0);
    const double bs = sqrt(-2.0 * log(halton_dev(8, (uint64_t)sl + 1))) / sqrt(ne);
    const double ph = 2.0 * kPi * halton_dev(9, (uint64_t)sl + 1);
    R.pr[0][2][q] = z + (-(2.0 * bs / P.k) * sin(P.k * z + ph));
}

hipError_t launch_gen_bunch(const RunDev &R, const GenParams &P, int pass, double *zrange, hipStream_t st)
{
    const unsigned nb = (unsigned)((P.n + 255) / 256);
    if (pass == 0) {
        hipLaunchKernelGGL(k_gen_bunch, dim3(nb), dim3(256), 0, st, R, P);
        hipLaunchKernelGGL(k_gen_zrange, dim3(1), dim3(1024), 0, st, R, P.n, zrange);
    } else if (pass == 1) {
        hipLaunchKernelGGL(k_gen_count, dim3(nb), dim3(256), 0, st, R, P);
    } else {
        hipLaunchKernelGGL(k_gen_noise, dim3(nb), dim3(256), 0, st, R, P);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

// A single run's push launch followed by the Mur edge and corner
// workgroups.  The edges read the face values of the step's n+1 level and
// write edge and corner nodes only, which neither the vertex fields (axis
// neighbours of interior nodes) nor the push read, so they may run after
// the vertex fields.  They go last: at the front, their workgroups (each
// holding the push's LDS box) delayed the first push workgroups (FEL
// amplifier step 0.4018 -> 0.3987 ms), while at the end they fill the
// slots the push's ragged tail leaves (0.3969 ms).
template <class P, typename T>
struct PushThenEdges {
    static constexpr int kThreads = P::kThreads;
    static constexpr int kWaves = P::kWaves;
    static_assert(P::kThreads == MurEdge<T>::kThreads, "one block size for both bodies");
    static __device__ void run(const RunDev &R, Blk blk)
    {
        const int64_t np_blk = blk.n - mur_edge_blocks_of(R);
        if (blk.id >= np_blk)
            MurEdge<T>::run(R, Blk{blk.id - np_blk, blk.n - np_blk});
        else
            P::run(R, Blk{blk.id, np_blk});
    }
};

template <int MODE>
static hipError_t launch_dep(const RunDev &R, hipStream_t st)
{
    if constexpr (MODE == 0) {
        // a step's push, then the Mur edge and corner workgroups
        const unsigned blocks = (unsigned)((R.np + kDepThreads - 1) / kDepThreads + mur_edge_blocks_of(R));
        if (R.und_ext) {
            if (R.precision == 64)
                hipLaunchKernelGGL((k_run<PushThenEdges<PushDeposit<double, false, 0, true>, double>>), dim3(blocks),
                                   dim3(kDepThreads), 0, st, R);
            else if (R.compensated)
                hipLaunchKernelGGL((k_run<PushThenEdges<PushDeposit<float, true, 0, true>, float>>), dim3(blocks),
                                   dim3(kDepThreads), 0, st, R);
            else
                hipLaunchKernelGGL((k_run<PushThenEdges<PushDeposit<float, false, 0, true>, float>>), dim3(blocks),
                                   dim3(kDepThreads), 0, st, R);
        } else if (R.precision == 64) {
            hipLaunchKernelGGL((k_run<PushThenEdges<PushDeposit<double, false, 0>, double>>), dim3(blocks),
                               dim3(kDepThreads), 0, st, R);
        } else if (R.compensated) {
            hipLaunchKernelGGL((k_run<PushThenEdges<PushDeposit<float, true, 0>, float>>), dim3(blocks),
                               dim3(kDepThreads), 0, st, R);
        } else {
            hipLaunchKernelGGL((k_run<PushThenEdges<PushDeposit<float, false, 0>, float>>), dim3(blocks),
                               dim3(kDepThreads), 0, st, R);
        }
        return hipGetLastError();
    } else {
        // the load's deposit (no push, no boundary)
        if (R.np <= 0)
            return hipSuccess;
        const unsigned blocks = (unsigned)((R.np + kDepThreads - 1) / kDepThreads);
        if (R.precision == 64)
            hipLaunchKernelGGL((k_run<PushDeposit<double, false, MODE>>), dim3(blocks), dim3(kDepThreads), 0, st, R);
        else if (R.compensated)
            hipLaunchKernelGGL((k_run<PushDeposit<float, true, MODE>>), dim3(blocks), dim3(kDepThreads), 0, st, R);
        else
            hipLaunchKernelGGL((k_run<PushDeposit<float, false, MODE>>), dim3(blocks), dim3(kDepThreads), 0, st, R);
        return hipGetLastError();
    }
}

// Reduce the per-block partial boxes (and counts) of `nblocks` blocks into
// lo/hi (and *count if non-null): one block, fixed order.
__device__ inline void box_reduce_blk(const int32_t *part, int64_t nblocks, int32_t *lo, int32_t *hi, int32_t *count)
{
    __shared__ int32_t sh[7][1024];
    int32_t v[7] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -1, -1, -1, 0};
    for (int64_t b = threadIdx.x; b < nblocks; b += 1024) {
        const int32_t *q = part + 8 * b;
        for (int a = 0; a < 3; ++a) {
            v[a] = min(v[a], q[a]);
            v[3 + a] = max(v[3 + a], q[3 + a]);
        }
        v[6] += q[6];
    }
    for (int a = 0; a < 7; ++a)
        sh[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int a = 0; a < 3; ++a) {
                sh[a][threadIdx.x] = min(sh[a][threadIdx.x], sh[a][threadIdx.x + w]);
                sh[3 + a][threadIdx.x] = max(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + w]);
            }
            sh[6][threadIdx.x] += sh[6][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = sh[a][0];
            hi[a] = sh[3 + a][0];
        }
        if (count)
            *count = sh[6][0];
    }
}

__global__ __launch_bounds__(1024) void k_box_reduce(const int32_t *part, int64_t nblocks, int32_t *lo, int32_t *hi,
                                                    int32_t *count)
{
    box_reduce_blk(part, nblocks, lo, hi, count);
}

hipError_t launch_box_reduce(const RunDev &R, int64_t nblocks, const int32_t *part, int32_t *lo, int32_t *hi,
                             int32_t *count, hipStream_t st)
{
    hipLaunchKernelGGL(k_box_reduce, dim3(1), dim3(1024), 0, st, part, nblocks, lo, hi, count);
    return hipGetLastError();
}

int64_t dep_blocks(int64_t np) { return (np + kDepThreads - 1) / kDepThreads; }

hipError_t launch_push_deposit(const RunDev &R, hipStream_t st, bool box, bool end_step)
{
    hipError_t e = launch_dep<0>(R, st);
    if (e != hipSuccess || !box)  // !box: the small sort's workgroup reduces the boxes
        return e;
    // the boxes are written by a kernel that reads the step number on the
    // device, like every other stage
    if (end_step)
        hipLaunchKernelGGL((k_run<BoxReduceEndStep>), dim3(1), dim3(BoxReduceEndStep::kThreads), 0, st, R);
    else if (R.np > 0)
        hipLaunchKernelGGL((k_run<BoxReduceStep>), dim3(1), dim3(BoxReduceStep::kThreads), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_load_deposit(const RunDev &R, hipStream_t st)
{
    hipError_t e = launch_dep<1>(R, st);
    if (e != hipSuccess)
        return e;
    return launch_box_reduce(R, dep_blocks(R.np), R.boxpart, CTL_ADDR(R.ctl, dep_lo), CTL_ADDR(R.ctl, dep_hi), nullptr,
                             st);
}

hipError_t launch_bunching(const RunDev &R, double *part, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_bunching, dim3(blocks), dim3(256), 0, st, R, part);
    return hipGetLastError();
}

}  // namespace mithra

// ---------------------------------------------------------------------------
// grouped launches (several runs per launch; see k_group)
// ---------------------------------------------------------------------------
namespace mithra {

hipError_t launch_push_group(const Group &g, int64_t total, int precision, int compensated, hipStream_t st)
{
    if (total <= 0)
        return hipSuccess;
    if (precision == 64)
        hipLaunchKernelGGL((k_group<PushDeposit<double, false, 0>>), dim3((unsigned)total), dim3(kDepThreads), 0, st, g);
    else if (compensated)
        hipLaunchKernelGGL((k_group<PushDeposit<float, true, 0>>), dim3((unsigned)total), dim3(kDepThreads), 0, st, g);
    else
        hipLaunchKernelGGL((k_group<PushDeposit<float, false, 0>>), dim3((unsigned)total), dim3(kDepThreads), 0, st, g);
    return hipGetLastError();
}

// one workgroup per member each
hipError_t launch_box_group(const Group &g, int64_t total, hipStream_t st)
{
    if (total <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_group<BoxReduceStep>), dim3((unsigned)total), dim3(BoxReduceStep::kThreads), 0, st, g);
    return hipGetLastError();
}

}  // namespace mithra
