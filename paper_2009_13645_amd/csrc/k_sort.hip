// k_sort.hip -- bin and sort of the macro-particles by cell.
//
// Key of a particle: the tile-major index of its cell (i,j,k) = floor of
// its grid coordinates, for tile dims (Tx,Ty,Tz):
//   key = tile_lin * (Tx Ty Tz) + local_lin,
//   tile_lin  = ((k/Tz) nTy + j/Ty) nTx + i/Tx,
//   local_lin = ((k%Tz) Ty + j%Ty) Tx + i%Tx,
// and particles outside the active region (cell outside 1..n-3 on some
// axis) get the key one past the largest tile-major index.  The order is
// ascending key with ties broken by particle id; it is unique, so the
// result is bit-exact whatever the previous order was.
//
// Method: keys are scattered to id order, then an LSD radix sort with
// 8-bit digits and stable passes runs on (key, id) pairs starting from the
// identity order, which makes ties come out in id order.  Each pass is a
// per-block digit histogram, one exclusive scan over (digit, block), and a
// stable scatter that ranks equal digits within a wavefront with ballots.
// Finally the particle state is gathered into the other buffer in sorted
// order.  No library sort and no memset: every pass is a plain kernel, so
// the pipeline can be captured in a graph.
#include "mithra_dev.hpp"

namespace mithra {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortChunk = kSortThreads * kSortItems;  // elements per block

__device__ inline uint32_t particle_key(const RunDev &R, double x, double y, double z, int c[3], bool &act)
{
    const double g[3] = {(x - R.x0) / R.dx, (y - R.y0) / R.dy, (z - R.z0) / R.dz};
    const int n[3] = {R.nx, R.ny, R.nz};
    act = true;
    for (int a = 0; a < 3; ++a) {
        const double f = floor(g[a]);
        act = act && (f >= 1.0) && (f <= (double)(n[a] - 3));
        c[a] = act ? (int)f : 0;
    }
    if (!act)
        return R.key_inactive;
    const int Tx = R.tile[0], Ty = R.tile[1], Tz = R.tile[2];
    const uint32_t tl = ((uint32_t)(c[2] / Tz) * (uint32_t)R.ntile[1] + (uint32_t)(c[1] / Ty)) * (uint32_t)R.ntile[0] +
                        (uint32_t)(c[0] / Tx);
    const uint32_t loc = ((uint32_t)(c[2] % Tz) * Ty + (uint32_t)(c[1] % Ty)) * Tx + (uint32_t)(c[0] % Tx);
    return tl * (uint32_t)(Tx * Ty * Tz) + loc;
}

// keys to id order, slot of every id, box of active cells, active count
__global__ __launch_bounds__(256) void k_sort_keys(RunDev R)
{
    __shared__ int sh[7];
    if (threadIdx.x < 3) {
        sh[threadIdx.x] = 0x7fffffff;
        sh[3 + threadIdx.x] = -1;
    }
    if (threadIdx.x == 0)
        sh[6] = 0;
    __syncthreads();
    const int pb = R.ctl->pbuf;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < R.np) {
        int c[3];
        bool act;
        const uint32_t key = particle_key(R, R.pr[pb][0][p], R.pr[pb][1][p], R.pr[pb][2][p], c, act);
        const int32_t id = R.pid[pb][p];
        R.key_by_id[id] = key;
        R.slot_of_id[id] = (int32_t)p;
        if (act) {
            for (int a = 0; a < 3; ++a) {
                atomicMin(&sh[a], c[a]);
                atomicMax(&sh[3 + a], c[a]);
            }
            atomicAdd(&sh[6], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < 3 && sh[3 + threadIdx.x] >= 0) {
        atomicMin(&R.ctl->cell_lo[threadIdx.x], sh[threadIdx.x]);
        atomicMax(&R.ctl->cell_hi[threadIdx.x], sh[3 + threadIdx.x]);
    }
    if (threadIdx.x == 0 && sh[6] > 0)
        atomicAdd(&R.ctl->n_active, sh[6]);
}

// per-block digit histogram, stored digit-major: hist[d * nblocks + b]
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *keys, int64_t n, int shift, uint32_t *hist,
                                                          int64_t nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t e = base + (int64_t)it * kSortThreads + threadIdx.x;
        if (e < n)
            atomicAdd(&h[(keys[e] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan in place over `total` counters, one block of 1024 threads
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t *a, int64_t total)
{
    __shared__ uint32_t part[1024];
    const int64_t per = (total + 1023) / 1024;
    const int64_t b = (int64_t)threadIdx.x * per;
    const int64_t e = min(b + per, total);
    uint32_t s = 0;
    for (int64_t x = b; x < e; ++x)
        s += a[x];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int64_t x = b; x < e; ++x) {
        const uint32_t v = a[x];
        a[x] = run;
        run += v;
    }
}

// stable scatter of one pass.  vals_in == nullptr means identity values.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t *keys_in, const int32_t *vals_in,
                                                             uint32_t *keys_out, int32_t *vals_out, int64_t n,
                                                             int shift, const uint32_t *offs, int64_t nblocks)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kSortThreads / 64][256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    run[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int it = 0; it < kSortItems; ++it) {
        for (int w = 0; w < kSortThreads / 64; ++w)
            wcnt[w][threadIdx.x] = 0;
        const int64_t e = base + (int64_t)it * kSortThreads + threadIdx.x;
        const bool ok = e < n;
        uint32_t key = 0;
        int32_t val = 0;
        uint32_t d = 0;
        if (ok) {
            key = keys_in[e];
            val = vals_in ? vals_in[e] : (int32_t)e;
            d = (key >> shift) & 0xFF;
        }
        // lanes of this wavefront holding the same digit
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        __syncthreads();
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (ok && rank == 0)
            wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (ok) {
            uint32_t pos = run[d] + rank;
            for (int w = 0; w < wave; ++w)
                pos += wcnt[w][d];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / 64; ++w)
            add += wcnt[w][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

// gather particle state into the other buffer in sorted order
__global__ __launch_bounds__(256) void k_sort_gather(RunDev R, const uint32_t *keys, const int32_t *ids)
{
    const int pb = R.ctl->pbuf;
    const int nb = pb ^ 1;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R.np)
        return;
    const int32_t id = ids[r];
    const int32_t src = R.slot_of_id[id];
    for (int a = 0; a < 6; ++a)
        R.pr[nb][a][r] = R.pr[pb][a][src];
    R.pid[nb][r] = id;
    R.key_sorted[r] = keys[r];
}

// ---------------------------------------------------------------------------

int sort_passes(uint32_t key_inactive)
{
    int bits = 0;
    while (bits < 32 && (key_inactive >> bits) != 0)
        ++bits;
    return bits <= 8 ? 1 : (bits + 7) / 8;
}

int64_t sort_blocks(int64_t n) { return (n + kSortChunk - 1) / kSortChunk; }

hipError_t launch_sort(const RunDev &R, hipStream_t st)
{
    if (R.np <= 0)
        return hipSuccess;
    const unsigned pblocks = (unsigned)((R.np + 255) / 256);
    hipLaunchKernelGGL(k_sort_keys, dim3(pblocks), dim3(256), 0, st, R);
    const int passes = sort_passes(R.key_inactive);
    const int64_t nb = R.sort_blocks;
    const uint32_t *kin = R.key_by_id;
    const int32_t *vin = nullptr;
    for (int ps = 0; ps < passes; ++ps) {
        uint32_t *kout = R.sk[ps & 1];
        int32_t *vout = R.sv[ps & 1];
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, st, kin, R.np, 8 * ps, R.hist, nb);
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, R.hist, 256 * nb);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, st, kin, vin, kout, vout, R.np,
                           8 * ps, R.hist, nb);
        kin = kout;
        vin = vout;
    }
    hipLaunchKernelGGL(k_sort_gather, dim3(pblocks), dim3(256), 0, st, R, kin, vin);
    return hipGetLastError();
}

}  // namespace mithra
