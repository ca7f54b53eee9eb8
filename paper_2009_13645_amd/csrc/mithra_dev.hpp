// mithra_dev.hpp -- device-side run description and helpers shared by the
// HIP kernels of the boosted-frame PIC step (NSFD sweep, Mur, vertex fields,
// push/deposit, sort, diagnostics).  Host code fills `RunDev` once per run;
// kernels receive it by value and read the step counter from `Ctl`, so a
// captured step can be replayed without changing any launch argument.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <type_traits>

namespace mithra {

// CODATA 2018
constexpr double kC = 299792458.0;
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

// Device-resident step bookkeeping.  Written only by the kernels of the
// step pipeline (and zeroed at init).
struct Ctl {
    int64_t step;          // completed field steps
    int32_t pbuf;          // particle buffer holding the current sorted state
    int32_t nsort;         // sorts done
    int32_t dep_lo[2][3];  // node bounding box of the nonzero entries of source set s
    int32_t dep_hi[2][3];
    int32_t cell_lo[3];    // bounding box of active particle cells at the last sort
    int32_t cell_hi[3];
    int32_t nan_flag;      // set when a diagnostic sees a non-finite value
    int32_t n_active;      // particles in active cells after the last push (or the load)
    int64_t target;        // step count at which a batched run stops (grouped launches only)
    uint32_t key_base;     // sort keys of the current sort are offset by this (active keys >= it)
    uint32_t key_span;     // active keys lie in [key_base, key_base + key_span); inactive sort as key_span
    int32_t npass;         // radix passes the current sort needs (8-bit digits of key_span)
    int32_t sorted_buf;    // sv[sorted_buf] holds the particles' slots in the order of the last sort;
                           // -1: no sort after the last push, the order is the buffer order
};

constexpr int kMaxBatch = 1;  // one run per RunDev

// floor(t / d) by a multiply-high with m = ceil(2^32 / d): exact whenever
// t * d < 2^32 (the error of m is below 1, so t m / 2^32 stays below the
// next integer); for index decoding by a divisor that is uniform per launch.
struct FastDiv {
    uint32_t d, m;
};

__host__ __device__ inline FastDiv fast_div(uint32_t d) { return FastDiv{d, d == 1 ? 0u : 0xFFFFFFFFu / d + 1u}; }

__device__ inline uint32_t fdiv(uint32_t t, FastDiv f) { return f.d == 1 ? t : __umulhi(t, f.m); }

struct RunDev {
    // mesh
    int nx, ny, nz;
    int64_t nn;
    double dx, dy, dz, x0, y0, z0;
    double inv_dx, inv_dy, inv_dz;  // only used where a product is not compared bitwise
    // time
    double dt, dtb;
    int n_sub;
    int sort_every;  // sort after every sort_every-th push (>= 1)
    // frame and undulator
    double gamma0, beta0;
    double ku, B0, Lu, z_ent, theta;
    int und_type;     // 0 planar, 1 helical, 2 optical plane wave, 3 optical Gaussian beam
    int und_ext;      // 1: the external field needs the general path (arrays or optical)
    double Kund, lam_u; // undulator parameter (optical: a0) and period (optical: half the wavelength)
    int n_modules;    // static array: modules, K_m = K + m dK, gaps between them
    double gap, dK;
    int opt_signal;   // optical pulse: signal type, length, offset (c t, lab), CEP (rad)
    double opt_ctau, opt_ct0, opt_cep, opt_w0[2], opt_zf;
    // TF/SF seed (planes k = 1 and 2)
    int seed_on, seed_type, seed_signal;
    double seed_a0, seed_lambda, seed_ctau, seed_ct0, seed_cep, seed_pol, seed_w0, seed_zf;
    // spectral power: nfreq frequencies nu = nu_min + (nu_max - nu_min) f / (nfreq - 1) times omega_r
    int nfreq;
    double nu_min, nu_max, omega_r;
    double *spec;     // [nfreq][8][nx*ny] running transforms (re/im of Ex' Ey' Bx' By')
    int solver;       // 0 NSFD, 1 FD
    // NSFD interior update: next = a1 cur + a2 (bar_x+ + bar_x-) + a4 (bar_y+ + bar_y-)
    //                              + a6 (cur_k+ + cur_k-) - prev + S
    double A, a1, a2, a4, a6;
    double rx2, ry2, rz2;  // (c dt / d_l)^2: the difference form of the FP32 sweeps
    double qvh_dt[3];      // q / (dx dy dz) * d_l / dt: edge current per unit grid displacement
    double sfac_A;    // (c dt)^2 mu0, multiplies the node-averaged J
    double sfac_phi;  // (c dt)^2 / eps0, multiplies rho
    int space_charge;
    int order;        // Mur order
    // Mur coefficients per normal axis a (faces of axis a), transverse axes
    // t1 = (a+1)%3 and t2 = (a+2)%3:
    //   first order:  be0 (xi0^{n-1} + xi1^{n+1}) + be1 (xi0^n + xi1^n) - xi1^{n-1}
    //   second order: be0 (...) + g1 (xi0^n + xi1^n) - xi1^{n-1}
    //                 + ga (t1 neighbours on planes 0 and 1) + gb (t2 neighbours)
    double mur_be0[3], mur_be1[3], mur_g1[3], mur_ga[3], mur_gb[3];
    double h[3];      // dx dy dz
    double cdt;       // c dt
    int xface_fused;  // 1: the (vector) sweep also updates the x-face nodes
    int precision;    // 32 or 64
    int compensated;
    // particles
    double q, qV;     // macro charge and q / (dx dy dz)
    int64_t np;
    int64_t np_cap;
    int tile[3];
    int ntile[3];
    uint32_t key_inactive;  // sort key of particles outside the active region
    // storage (element type T = float or double for the field arrays)
    void *pot;        // [3 slots][4 comps][nn]
    void *src;        // [2 sets][4: Jx Jy Jz rho][nn]
    void *src_lo;     // compensation terms (same layout) or null
    void *eb;         // [6: Ex Ey Ez Bx By Bz][nn]
    double *pr[2][6]; // particle buffers: x y z ux uy uz
    int32_t *pid[2];
    uint32_t *key_in;     // sort input: key of rank p of the previous order
    int32_t *slot_in;     // sort input: the slot that holds it
    uint32_t *tile_flag;  // per sort tile: the step whose vertex fields the tile's particles gather
    // per source set and (z plane, y row), [2][nz][ny]: the x range of nodes
    // whose sources the last deposit into the set may have made nonzero,
    // grown by one node along every axis (so that it also covers the
    // neighbour each node-averaged source reads); empty when lo > hi
    int32_t *srow_lo, *srow_hi;
    uint32_t *sk[2];
    int32_t *sv[2];
    uint32_t *hist;
    int64_t sort_blocks;
    int32_t *boxpart;  // per-block partial boxes (load deposit, key pass): [block][8] = lo[3], hi[3], count, pad
    int32_t *boxslot;  // kBoxSlots x 16 boxes of the per-block push, reduced with atomics (layout: BoxReduceStep)
    FastDiv tdiv[3];   // division by the sort tile dims (exact: cell index x tile dim < 2^32)
    double *ppart;     // partial sums of the plane-power kernel
    double *power_hist;
    int64_t power_cap;
    int k_plane;
    int record_power;
    Ctl *ctl;
};

// Parameters of the Halton bunch generator (k_particles.hip), filled on the host.
struct GenParams {
    int long_profile, trans_profile, shot_noise;
    int64_t n, n_flat;
    double cx, cy, cz, sx, sy, L;
    double gamma, sig_g, sig_u, bf, bphase, n_e;
    double lz, k, sig_t;
    double zmin, slice;  // shot noise: first z and slice length (third pass)
    int32_t *counts;     // slice counts (second and third passes)
};


// Device address of a Ctl member, formed on the host without dereferencing.
#define CTL_ADDR(ctl, member) ((int32_t *)((char *)(ctl) + offsetof(::mithra::Ctl, member)))

__host__ __device__ inline int64_t nid(const RunDev &R, int i, int j, int k)
{
    return ((int64_t)k * R.ny + j) * R.nx + i;
}

template <typename T>
__device__ inline T *pot_ptr(const RunDev &R, int slot, int comp)
{
    return reinterpret_cast<T *>(R.pot) + ((int64_t)slot * 4 + comp) * R.nn;
}

template <typename T>
__device__ inline T *src_ptr(const RunDev &R, int set, int comp)
{
    return reinterpret_cast<T *>(R.src) + ((int64_t)set * 4 + comp) * R.nn;
}

template <typename T>
__device__ inline T *srclo_ptr(const RunDev &R, int set, int comp)
{
    return reinterpret_cast<T *>(R.src_lo) + ((int64_t)set * 4 + comp) * R.nn;
}

// V consecutive values moved as one 16-byte access when sizeof(T) V == 16.
template <typename T, int V>
struct Vec {
    T v[V];
};

template <typename T, int V>
__device__ inline Vec<T, V> vload(const T *p)
{
    Vec<T, V> r;
    if constexpr (sizeof(T) * V == 16) {
        const uint4 x = *reinterpret_cast<const uint4 *>(p);
        memcpy(&r, &x, 16);
    } else {
        for (int e = 0; e < V; ++e)
            r.v[e] = p[e];
    }
    return r;
}

template <typename T, int V>
__device__ inline void vstore(T *p, const Vec<T, V> &a)
{
    if constexpr (sizeof(T) * V == 16) {
        uint4 x;
        memcpy(&x, &a, 16);
        *reinterpret_cast<uint4 *>(p) = x;
    } else {
        for (int e = 0; e < V; ++e)
            p[e] = a.v[e];
    }
}


// E and B at the vertices are stored node-interleaved: node n holds
// Ex Ey Ez Bx By Bz and two pad words at eb[8 n .. 8 n + 7] (32 bytes in FP32,
// 64 in FP64), so that a corner of the gather is two or four 16-byte loads.
template <typename T>
__device__ inline T *eb_node(const RunDev &R, int64_t n)
{
    return reinterpret_cast<T *>(R.eb) + 8 * n;
}

// Time-level slots of the three rotating potential arrays during step s:
// prev (n-1), cur (n), next (n+1).
__host__ __device__ inline int slot_prev(int64_t s) { return (int)(s % 3); }
__host__ __device__ inline int slot_cur(int64_t s) { return (int)((s + 1) % 3); }
__host__ __device__ inline int slot_next(int64_t s) { return (int)((s + 2) % 3); }

// XCD-aware block order: the hardware deals consecutive workgroups round-
// robin over the 8 XCDs; remap so that each XCD receives a contiguous range
// of logical tiles (which share halos through that XCD's L2).
__device__ inline int64_t xcd_swizzle(int64_t bid, int64_t nblocks)
{
    const int64_t nx = 8;
    int64_t full = (nblocks / nx) * nx;
    if (bid >= full)
        return bid;
    int64_t per = full / nx;
    return (bid % nx) * per + bid / nx;
}

// ---------------------------------------------------------------------------
// Kernel bodies and their two entries.  A body is a struct F with
//   static constexpr int kThreads;
//   static __device__ void run(const RunDev &R, Blk b, args...);
// where Blk replaces blockIdx.x / gridDim.x.  k_run launches it for one run
// (R passed by value); k_group launches it for several runs at once: the
// grid is the concatenation of the members' grids, each member's part
// starting on a multiple of 8 workgroups so that the XCD-aware block order
// holds inside it.  A member whose step counter has reached its target
// does no work (a batch of runs with different lengths replays one graph).
struct Blk {
    int64_t id, n;
};

struct Group {
    const RunDev *runs;    // member descriptors (device memory)
    const int64_t *boff;   // nmem+1 workgroup offsets, multiples of 8
    const int64_t *nblk;   // workgroups each member needs (<= its slice)
    int nmem;
};

__device__ inline int group_find(const Group &G, int64_t b)
{
    int lo = 0, hi = G.nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (G.boff[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Minimum waves per SIMD a body asks the register allocator for
// (F::kWaves when present): a body limited by latency rather than issue
// rate trades a few registers for occupancy.
template <class F, class = void>
struct WavesOf {
    static constexpr int value = 1;
};
template <class F>
struct WavesOf<F, std::void_t<decltype(F::kWaves)>> {
    static constexpr int value = F::kWaves;
};

template <class F, class... A>
__global__ __launch_bounds__(F::kThreads) __attribute__((amdgpu_waves_per_eu(WavesOf<F>::value))) void k_run(RunDev R,
                                                                                                          A... a)
{
    F::run(R, Blk{(int64_t)blockIdx.x, (int64_t)gridDim.x}, a...);
}

// How k_group reaches its member's descriptor.  Through a plain reference a
// field read after a store to device memory cannot be shown unchanged, so
// it is reloaded into vector registers.  Two remedies:
//  * stages with F::kCopyRun take a by-value copy before any store (the
//    sweeps: 6-15 fewer VGPRs, a fourth wave per SIMD at FP64); stages that
//    index the descriptor's arrays at run time would put such a copy in
//    scratch memory, so it is opt-in;
//  * the others read it through a restrict pointer: the table is never
//    written by a kernel, so its loads stay scalar (vertex fields: 107 -> 96
//    VGPRs at FP32).
template <class F, class = void>
struct CopyRunOf {
    static constexpr bool value = false;
};
template <class F>
struct CopyRunOf<F, std::void_t<decltype(F::kCopyRun)>> {
    static constexpr bool value = F::kCopyRun;
};

template <class F, class... A>
__device__ __attribute__((always_inline)) inline void group_stage(const RunDev *__restrict__ runs, int m, Blk blk,
                                                                  A... a)
{
    const RunDev &R = runs[m];
    if (R.ctl->step >= R.ctl->target)
        return;
    F::run(R, blk, a...);
}

template <class F, class... A>
__global__ __launch_bounds__(F::kThreads) __attribute__((amdgpu_waves_per_eu(WavesOf<F>::value))) void k_group(
    Group G, A... a)
{
    const int m = group_find(G, (int64_t)blockIdx.x);
    const int64_t id = (int64_t)blockIdx.x - G.boff[m];
    if (id >= G.nblk[m])
        return;
    if constexpr (CopyRunOf<F>::value) {
        // a copy taken before any store: the fields the stage uses load
        // through the scalar cache once, as from the argument of k_run
        const RunDev R = G.runs[m];
        if (R.ctl->step >= R.ctl->target)
            return;
        F::run(R, Blk{id, G.nblk[m]}, a...);
    } else {
        group_stage<F>(G.runs, m, Blk{id, G.nblk[m]}, a...);
    }
}

// Plane-power workgroups (partial sums in ppart, fixed node partition).
constexpr int kPowerBlocks = 64;

// The radiated power of step s from the sum of the plane-power partial sums
// (lab-frame Poynting flux times the node area), stored to *out or to the
// run's power history; with end_step, the step's bookkeeping follows
// (particle buffer, sort count, step counter).  One thread.
__device__ inline void plane_power_store(const RunDev &R, int64_t s, double sum, double *out, int end_step)
{
    const double mu0 = 1.0 / (kEps0 * kC * kC);
    const double P = sum * R.dx * R.dy / mu0;
    if (out)
        *out = P;
    else if (s >= 0 && s < R.power_cap)
        R.power_hist[s] = P;
    if (!isfinite(P))
        R.ctl->nan_flag = 1;
    if (end_step) {
        R.ctl->pbuf ^= 1;
        R.ctl->nsort += 1;
        R.ctl->step += 1;
    }
}

// The same with the partial sums added by the calling wavefront (lane l
// loads partial l, a fixed butterfly adds them, lane 0 stores).  The whole
// first wavefront of the block must call it.
__device__ inline void plane_power_final(const RunDev &R, int64_t s, double *out, int end_step)
{
    static_assert(kPowerBlocks == 64, "one partial sum per lane");
    const int lane = threadIdx.x & 63;
    double x = R.ppart[lane];
    for (int o = 1; o < 64; o <<= 1)
        x += __shfl_xor(x, o);
    if (lane == 0)
        plane_power_store(R, s, x, out, end_step);
}

// Linear index of the sort tile of an active cell c (tile-major order).
// (cells are non-negative; the tile divisions are exact multiply-highs)
__device__ inline uint32_t tile_of_cell(const RunDev &R, const int c[3])
{
    return (fdiv((uint32_t)c[2], R.tdiv[2]) * (uint32_t)R.ntile[1] + fdiv((uint32_t)c[1], R.tdiv[1])) *
               (uint32_t)R.ntile[0] +
           fdiv((uint32_t)c[0], R.tdiv[0]);
}

// Tile-major sort key of an active cell c (see k_sort.hip for the order).
__device__ inline uint32_t key_of_cell(const RunDev &R, const int c[3])
{
    const uint32_t Tx = (uint32_t)R.tile[0], Ty = (uint32_t)R.tile[1], Tz = (uint32_t)R.tile[2];
    uint32_t q[3], m[3];
    for (int a = 0; a < 3; ++a) {
        q[a] = fdiv((uint32_t)c[a], R.tdiv[a]);
        m[a] = (uint32_t)c[a] - q[a] * (uint32_t)R.tile[a];
    }
    const uint32_t tl = (q[2] * (uint32_t)R.ntile[1] + q[1]) * (uint32_t)R.ntile[0] + q[0];
    const uint32_t loc = (m[2] * Ty + m[1]) * Tx + m[0];
    return tl * (Tx * Ty * Tz) + loc;
}

// Offset and pass count of the current sort, from the box of the active
// cells: active keys lie between the first key of the box's first tile and
// the key of the box's high corner (the key is increasing in each tile
// coordinate and in each offset inside a tile).  Inactive particles sort as
// one past that range.  One thread.
// may_skip: the sort after the push of step ctl->step, which runs only
// after every sort_every-th push; a skipped sort leaves the order as it is
// (no passes, and the push reads the state in buffer order).  The sort at
// load always runs.
__device__ inline void sort_range(const RunDev &R, bool may_skip)
{
    Ctl *c = R.ctl;
    if (may_skip && R.sort_every > 1 && (c->step + 1) % R.sort_every != 0) {
        c->npass = 0;
        c->sorted_buf = -1;
        return;
    }
    uint32_t base = 0, span = 0;
    if (c->cell_hi[0] >= c->cell_lo[0] && c->cell_hi[1] >= c->cell_lo[1] && c->cell_hi[2] >= c->cell_lo[2]) {
        const uint32_t vol = (uint32_t)(R.tile[0] * R.tile[1] * R.tile[2]);
        uint32_t t0[3];
        for (int a = 0; a < 3; ++a)
            t0[a] = (uint32_t)(c->cell_lo[a] / R.tile[a]);
        const uint32_t l0 = (t0[2] * (uint32_t)R.ntile[1] + t0[1]) * (uint32_t)R.ntile[0] + t0[0];
        base = l0 * vol;
        // the box's largest key is that of its high corner (the corner's
        // tile and its offset inside that tile are the largest in each axis)
        const int hi[3] = {c->cell_hi[0], c->cell_hi[1], c->cell_hi[2]};
        span = key_of_cell(R, hi) + 1u - base;
    }
    int bits = 0;
    while (bits < 32 && (span >> bits) != 0)
        ++bits;
    const int np = bits <= 8 ? 1 : (bits + 7) / 8;
    c->key_base = base;
    c->key_span = span;
    c->npass = np;
    c->sorted_buf = (np - 1) & 1;
}

// particles per workgroup of the push (one per thread)
constexpr int kDepThreads = 256;
__host__ __device__ inline int64_t dep_blocks_dev(int64_t np) { return (np + kDepThreads - 1) / kDepThreads; }

// After a per-block push: the deposit box of set (s+1)&1, the active-cell
// box (from the deposit box) and the active count, then the key range of
// the sort that follows;
// the tile work item counter is reset.  The push's workgroups reduce their
// boxes into kBoxSlots slots with integer atomics (min, max, add: the order
// does not change the result); here the first wavefront reduces the slots,
// leaves them empty for the next push, and one thread stores the result.
// Slot layout (16 words): dep lo[3], dep hi[3], unused[6] (left empty),
// active count, pad[3].  Every thread of the block must call it (barriers).
constexpr int kBoxSlots = 64;

__host__ __device__ inline void box_slot_empty(int32_t q[16])
{
    for (int a = 0; a < 16; ++a)
        q[a] = (a < 3 || (a >= 6 && a < 9)) ? 0x7fffffff : ((a < 12) ? -1 : 0);
}

struct BoxReduceStep {
    static constexpr int kThreads = 64;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        const int set = (int)((R.ctl->step + 1) & 1);
        Ctl *c = R.ctl;
        if (threadIdx.x < (unsigned)kBoxSlots) {
            static_assert(kBoxSlots == 64, "one slot per lane of the first wavefront");
            int4 *q = (int4 *)(R.boxslot + 16 * threadIdx.x);
            const int4 a0 = q[0], a1 = q[1], a2 = q[2], a3 = q[3];
            int32_t v[13] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w, a2.x, a2.y, a2.z, a2.w, a3.x};
            int32_t e[16];
            box_slot_empty(e);
            q[0] = make_int4(e[0], e[1], e[2], e[3]);
            q[1] = make_int4(e[4], e[5], e[6], e[7]);
            q[2] = make_int4(e[8], e[9], e[10], e[11]);
            q[3] = make_int4(e[12], e[13], e[14], e[15]);
#pragma unroll
            for (int a = 0; a < 13; ++a) {
                const int kind = a == 12 ? 2 : ((a / 3) & 1);  // 0 min, 1 max, 2 sum
                for (int o = 32; o > 0; o >>= 1) {
                    const int32_t x = __shfl_xor(v[a], o);
                    v[a] = kind == 0 ? min(v[a], x) : (kind == 1 ? max(v[a], x) : v[a] + x);
                }
            }
            if (threadIdx.x == 0) {
                // the box of the active cells after the push is taken as the
                // node box of the deposits less its upper layer: it holds
                // every active cell, and the cells it adds (those left by
                // the push) lie within one cell of it
                for (int a = 0; a < 3; ++a) {
                    c->dep_lo[set][a] = v[a];
                    c->dep_hi[set][a] = v[3 + a];
                    c->cell_lo[a] = v[a];
                    c->cell_hi[a] = v[3 + a] - 1;
                }
                c->n_active = v[12];
                sort_range(R, true);  // the offset and pass count of this step's sort
            }
        }
        __syncthreads();
    }
};

// The box reductions, then the end of the step: the step's radiated power
// from the vertex launch's partial sums (when the run records it) and the
// bookkeeping (particle buffer, step counter).  For a single run whose sort,
// when the step has one, runs as separate pass kernels: those read the sort
// range and the slots, not the step counter or the buffer index, so the
// step may end before them and no launch follows the sort.  Grouped steps
// keep the separate end: there a member on its last step skips the stages
// that come after its step counter has reached the target.
struct BoxReduceEndStep {
    static constexpr int kThreads = 64;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        BoxReduceStep::run(R, blk);
        if (R.record_power) {
            plane_power_final(R, R.ctl->step, nullptr, 1);
        } else if (threadIdx.x == 0) {
            R.ctl->pbuf ^= 1;
            R.ctl->nsort += 1;
            R.ctl->step += 1;
        }
    }
};

}  // namespace mithra
