// k_sort.hip -- bin and sort of the macro-particles by cell.
//
// Key of a particle: the tile-major index of its cell (i,j,k) = floor of
// its grid coordinates, for tile dims (Tx,Ty,Tz):
//   key = tile_lin * (Tx Ty Tz) + local_lin,
//   tile_lin  = ((k/Tz) nTy + j/Ty) nTx + i/Tx,
//   local_lin = ((k%Tz) Ty + j%Ty) Tx + i%Tx,
// and particles outside the active region (cell outside 1..n-3 on some
// axis) get the key one past the largest tile-major index.  The order is
// ascending key with ties in the previous order: a stable sort of the
// previous order (the last sort's ranks; at load, the buffer order, which
// is the particle ids).
//
// Method: the keys are written in the previous order (the push writes the
// key of rank p at p, coalesced), then an LSD radix sort with 8-bit digits
// and stable passes runs on (key, slot) pairs.  The value carried is the
// particle's slot in the buffer the next push reads (slot_in), so the
// push reaches the state without looking the slot up.  Each pass is a
// per-block digit histogram, 256 independent per-digit scans over the
// blocks, and a stable scatter that ranks equal digits within a wavefront
// with ballots.  Finally the particle state is gathered into the other
// buffer in sorted order.  No library sort and no memset: every pass is a
// plain kernel, so the pipeline can be captured in a graph.
#include "mithra_dev.hpp"

namespace mithra {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
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
    return key_of_cell(R, c);
}

__device__ inline int wmin(int v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ inline int wmax(int v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, __shfl_xor(v, o));
    return v;
}

// keys and slots in buffer order, box of active cells, active count
__global__ __launch_bounds__(256) void k_sort_keys(RunDev R)
{
    const int pb = R.ctl->pbuf;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, hi[3] = {-1, -1, -1};
    bool act = false;
    if (p < R.np) {
        int c[3];
        const uint32_t key = particle_key(R, R.pr[pb][0][p], R.pr[pb][1][p], R.pr[pb][2][p], c, act);
        R.key_in[p] = key;
        R.slot_in[p] = (int32_t)p;
        if (act)
            for (int a = 0; a < 3; ++a)
                lo[a] = hi[a] = c[a];
    }
    __shared__ int32_t wv[4][7];
    const int nact = __popcll(__ballot(act));
    for (int a = 0; a < 3; ++a) {
        lo[a] = wmin(lo[a]);
        hi[a] = wmax(hi[a]);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 3; ++a) {
            wv[wave][a] = lo[a];
            wv[wave][3 + a] = hi[a];
        }
        wv[wave][6] = nact;
    }
    __syncthreads();
    // block partial (reduced over blocks by k_box_reduce)
    if (threadIdx.x < 7) {
        int32_t v = wv[0][threadIdx.x];
        for (int w = 1; w < 4; ++w) {
            const int32_t x = wv[w][threadIdx.x];
            v = threadIdx.x < 3 ? min(v, x) : (threadIdx.x < 6 ? max(v, x) : v + x);
        }
        R.boxpart[8 * (int64_t)blockIdx.x + threadIdx.x] = v;
    }
}

// per-block digit histogram, stored digit-major: hist[d * nblocks + b]
// Digit d of pass ps is taken from the offset key: key - key_base for
// active particles, key_span for inactive ones (same order as the keys; the
// offset needs only the bits of key_span, so passes beyond ctl->npass are
// skipped).
__device__ inline uint32_t sort_digit(const Ctl *ctl, uint32_t inactive, uint32_t key, int shift)
{
    const uint32_t x = key == inactive ? ctl->key_span : key - ctl->key_base;
    return (x >> shift) & 0xFF;
}

// Lanes of the calling wavefront whose digit equals this lane's (all lanes
// must call it; lanes with ok == false match nothing and are matched by
// nothing).
__device__ inline uint64_t digit_peers(uint32_t d, bool ok)
{
    uint64_t peers = __ballot(ok);
    for (int b = 0; b < 8; ++b) {
        const uint64_t m = __ballot((d >> b) & 1);
        peers &= ((d >> b) & 1) ? m : ~m;
    }
    return peers;
}

// Each wavefront of a block takes a contiguous quarter of the block's
// chunk, 64 consecutive elements per iteration, and counts digits in a
// histogram of its own with LDS atomics whose results nothing waits for.
__device__ inline void radix_hist_blk(const uint32_t *keys, int64_t n, int shift, uint32_t *hist, int64_t nblocks,
                                      int64_t bid, const Ctl *ctl, uint32_t inactive)
{
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t wh[kWaves][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < kWaves; ++w)
        wh[w][threadIdx.x] = 0;
    const int64_t wbase = (int64_t)bid * kSortChunk + (int64_t)wave * (kSortChunk / kWaves);
    uint32_t k[kSortItems];
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t e = wbase + 64 * it + lane;
        k[it] = e < n ? keys[e] : 0u;
    }
    __syncthreads();
    for (int it = 0; it < kSortItems; ++it) {
        if (wbase + 64 * it + lane < n)
            atomicAdd(&wh[wave][sort_digit(ctl, inactive, k[it], shift)], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
    for (int w = 0; w < kWaves; ++w)
        c += wh[w][threadIdx.x];
    hist[(int64_t)threadIdx.x * nblocks + bid] = c;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *keys, int64_t n, int shift, uint32_t *hist,
                                                          int64_t nblocks, const Ctl *ctl, uint32_t inactive, int ps)
{
    if (ps >= ctl->npass)
        return;
    radix_hist_blk(keys, n, shift, hist, nblocks, blockIdx.x, ctl, inactive);
}

// Per digit d (one block each): exclusive scan of hist[d][0..nblocks) in
// place, and the digit total into tot[d].
__device__ inline void digit_scan_blk(uint32_t *hist, int64_t nblocks, uint32_t *tot, int64_t bid)
{
    __shared__ uint32_t ws[4];
    uint32_t *a = hist + (int64_t)bid * nblocks;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t base = 0; base < nblocks; base += 4 * 256) {
        const int64_t e0 = base + 4 * (int64_t)threadIdx.x;
        uint32_t v[4];
        for (int q = 0; q < 4; ++q)
            v[q] = (e0 + q < nblocks) ? a[e0 + q] : 0u;
        const uint32_t ts = v[0] + v[1] + v[2] + v[3];
        uint32_t inc = ts;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o);
            if (lane >= o)
                inc += t;
        }
        if (lane == 63)
            ws[wave] = inc;
        __syncthreads();
        uint32_t wbase = 0, btot = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wave)
                wbase += ws[w];
            btot += ws[w];
        }
        uint32_t run = carry + wbase + inc - ts;
        for (int q = 0; q < 4; ++q) {
            if (e0 + q < nblocks)
                a[e0 + q] = run;
            run += v[q];
        }
        carry += btot;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        tot[bid] = carry;
}

__global__ __launch_bounds__(256) void k_digit_scan(uint32_t *hist, int64_t nblocks, uint32_t *tot, const Ctl *ctl, int ps)
{
    if (ps >= ctl->npass)
        return;
    digit_scan_blk(hist, nblocks, tot, blockIdx.x);
}

// stable scatter of one pass.  vals_in == nullptr means identity values.
// Forced inline: called from two kernels, it was otherwise compiled as a
// function with its own register budget (253 VGPRs, 2 waves per SIMD);
// inlined it takes 138 (3 waves).
__device__ __attribute__((always_inline)) inline void radix_scatter_blk(const uint32_t *keys_in, const int32_t *vals_in, uint32_t *keys_out,
                                         int32_t *vals_out, int64_t n, int shift, const uint32_t *offs, int64_t nblocks,
                                         const uint32_t *tot, int64_t bid, const Ctl *ctl, uint32_t inactive)
{
    // The block's kSortChunk elements are held in registers, each wavefront
    // a contiguous quarter of the chunk.  A wavefront ranks its elements
    // among equal digits with ballots and a digit counter of its own, which
    // needs no barrier; the counters of the four wavefronts then give each
    // wavefront its start inside every digit's run of the block, in element
    // order.  The elements go to LDS in block-local sorted order and are
    // written out in that order: each digit run is one contiguous range of
    // the output, so consecutive threads write consecutive addresses.
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t gbase[256];       // output position of the block's first element of each digit
    __shared__ uint32_t lstart[256];      // local position of the same
    __shared__ uint32_t wc[kWaves][256];  // per-wavefront digit counts, then starts
    __shared__ uint32_t scan_tmp[2][kWaves];
    __shared__ uint32_t skey[kSortChunk];
    __shared__ int32_t sval[kSortChunk];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)bid * kSortChunk;
    const int64_t cnt = min((int64_t)kSortChunk, n - base);
    const int64_t wbase = base + (int64_t)wave * (kSortChunk / kWaves);
    uint32_t k[kSortItems];
    int32_t v[kSortItems];
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t e = wbase + 64 * it + lane;
        const bool ok = e < n;
        k[it] = ok ? keys_in[e] : 0u;
        v[it] = ok ? (vals_in ? vals_in[e] : (int32_t)e) : 0;
    }
    for (int w = 0; w < kWaves; ++w)
        wc[w][threadIdx.x] = 0;
    {
        const int d = threadIdx.x;
        const uint32_t o = offs[(int64_t)d * nblocks + bid];
        const uint32_t o1 = bid + 1 < nblocks ? offs[(int64_t)d * nblocks + bid + 1] : tot[d];
        const uint32_t mine = o1 - o;  // this block's count of digit d
        // digit bases (inclusive wave scans of the totals and of the counts)
        const uint32_t t = tot[d];
        uint32_t inc = t, linc = mine;
        for (int q = 1; q < 64; q <<= 1) {
            const uint32_t u = __shfl_up(inc, q), lu = __shfl_up(linc, q);
            if (lane >= q) {
                inc += u;
                linc += lu;
            }
        }
        if (lane == 63) {
            scan_tmp[0][wave] = inc;
            scan_tmp[1][wave] = linc;
        }
        __syncthreads();
        uint32_t wb = 0, lwb = 0;
        for (int w = 0; w < wave; ++w) {
            wb += scan_tmp[0][w];
            lwb += scan_tmp[1][w];
        }
        gbase[d] = wb + inc - t + o;
        lstart[d] = lwb + linc - mine;
    }
    // Rank within the wavefront: position among the wavefront's earlier
    // elements of the same digit.  The lowest lane of each group of equal
    // digits adds the group's size to the wavefront's counter and gets the
    // count before it; LDS executes one wavefront's atomics in issue order,
    // so all of them can be in flight before the first result is used.
    // dp: digit (bits 0-7), leader lane (8-13), rank in the group (14-20).
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint32_t dp[kSortItems], before[kSortItems];
    for (int it = 0; it < kSortItems; ++it) {
        const bool ok = wbase + 64 * it + lane < n;
        const uint32_t d = ok ? sort_digit(ctl, inactive, k[it], shift) : 0u;
        const uint64_t peers = digit_peers(d, ok);
        const uint32_t r = (uint32_t)__popcll(peers & lt);
        const uint32_t leader = peers ? (uint32_t)__builtin_ctzll(peers) : 0u;
        before[it] = 0;
        if (ok && r == 0)
            before[it] = atomicAdd(&wc[wave][d], (uint32_t)__popcll(peers));
        dp[it] = (r << 14) | (leader << 8) | d;
    }
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t b = (uint32_t)__shfl((int)before[it], (int)((dp[it] >> 8) & 63));
        dp[it] = ((b + (dp[it] >> 14)) << 8) | (dp[it] & 0xFF);
    }
    __syncthreads();
    {
        // per digit: start of each wavefront's elements inside the block's run
        const int d = threadIdx.x;
        uint32_t run = lstart[d];
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = wc[w][d];
            wc[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int it = 0; it < kSortItems; ++it) {
        if (wbase + 64 * it + lane < n) {
            const uint32_t p = wc[wave][dp[it] & 0xFF] + (dp[it] >> 8);
            skey[p] = k[it];
            sval[p] = v[it];
        }
    }
    __syncthreads();
    // block-local sorted order -> output, digit runs contiguous
    for (int64_t i = threadIdx.x; i < cnt; i += kSortThreads) {
        const uint32_t key = skey[i];
        const uint32_t d = sort_digit(ctl, inactive, key, shift);
        const int64_t pos = (int64_t)gbase[d] + (i - (int64_t)lstart[d]);
        keys_out[pos] = key;
        vals_out[pos] = sval[i];
    }
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t *keys_in, const int32_t *vals_in,
                                                             uint32_t *keys_out, int32_t *vals_out, int64_t n,
                                                             int shift, const uint32_t *offs, int64_t nblocks,
                                                             const uint32_t *tot, const Ctl *ctl, uint32_t inactive,
                                                             int ps)
{
    if (ps >= ctl->npass)
        return;
    radix_scatter_blk(keys_in, vals_in, keys_out, vals_out, n, shift, offs, nblocks, tot, blockIdx.x, ctl, inactive);
}

// The whole sort in one workgroup when every particle fits one chunk: each
// pass ranks the keys in LDS exactly as the scatter does (wavefront slices
// in element order, ballots, per-wavefront digit counters), with the
// workgroup's own digit counts as the only offsets.  One launch replaces
// three per pass, which is most of a small run's sort time; 1024 threads
// hold four keys each.
constexpr int kSmallThreads = 1024;
constexpr int kSmallChunk = 4096;  // particles the one-workgroup sort takes
constexpr int kSmallItems = kSmallChunk / kSmallThreads;

// With step_tail, the workgroup is the whole tail of a step after the push:
// first the box reductions (BoxReduceStep, which the push launcher then
// skips), then the sort, then the end of the step (the power of the step
// from the vertex launch's partial sums when the run records it, and the
// bookkeeping).  A small run's push is then followed by this launch only.
__global__ __launch_bounds__(kSmallThreads) void k_sort_small(RunDev R, int step_tail)
{
    static_assert(kSmallThreads >= kBoxSlots, "the box reductions run in this workgroup");
    constexpr int kWaves = kSmallThreads / 64;
    __shared__ uint32_t skey[2][kSmallChunk];
    __shared__ int32_t sval[2][kSmallChunk];
    __shared__ uint32_t wc[kWaves][256];
    __shared__ uint32_t scan_tmp[4];
    const int n = (int)R.np;  // 1..kSmallChunk (checked by the launcher)
    const Ctl *ctl = R.ctl;
    if (step_tail) {
        BoxReduceStep::run(R, Blk{0, 1});
        __syncthreads();  // the sort range is in the control block
    }
    const int npass = ctl->npass;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int i = t; i < n; i += kSmallThreads) {
        skey[0][i] = R.key_in[i];
        sval[0][i] = R.slot_in[i];
    }
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int wbase = wave * (kSmallChunk / kWaves);
    for (int ps = 0; ps < npass; ++ps) {
        const int src = ps & 1, dst = src ^ 1;
        for (int i = t; i < kWaves * 256; i += kSmallThreads)
            (&wc[0][0])[i] = 0;
        __syncthreads();  // the input of the pass and the cleared counters
        uint32_t k[kSmallItems], dp[kSmallItems], before[kSmallItems];
        int32_t v[kSmallItems];
        for (int it = 0; it < kSmallItems; ++it) {
            const int e = wbase + 64 * it + lane;
            const bool ok = e < n;
            k[it] = ok ? skey[src][e] : 0u;
            v[it] = ok ? sval[src][e] : 0;
        }
        for (int it = 0; it < kSmallItems; ++it) {
            const bool ok = wbase + 64 * it + lane < n;
            const uint32_t d = ok ? sort_digit(ctl, R.key_inactive, k[it], 8 * ps) : 0u;
            const uint64_t peers = digit_peers(d, ok);
            const uint32_t r = (uint32_t)__popcll(peers & lt);
            const uint32_t leader = peers ? (uint32_t)__builtin_ctzll(peers) : 0u;
            before[it] = 0;
            if (ok && r == 0)
                before[it] = atomicAdd(&wc[wave][d], (uint32_t)__popcll(peers));
            dp[it] = (r << 14) | (leader << 8) | d;
        }
        for (int it = 0; it < kSmallItems; ++it) {
            const uint32_t b = (uint32_t)__shfl((int)before[it], (int)((dp[it] >> 8) & 63));
            dp[it] = ((b + (dp[it] >> 14)) << 8) | (dp[it] & 0xFF);
        }
        __syncthreads();
        // digit d (threads 0..255): its start in the pass's output (exclusive
        // scan of the digit totals), then each wavefront's start inside it
        uint32_t tot = 0, inc = 0;
        if (t < 256) {
            for (int w = 0; w < kWaves; ++w)
                tot += wc[w][t];
            inc = tot;
            for (int q = 1; q < 64; q <<= 1) {
                const uint32_t u = __shfl_up(inc, q);
                if (lane >= q)
                    inc += u;
            }
            if (lane == 63)
                scan_tmp[wave] = inc;
        }
        __syncthreads();
        if (t < 256) {
            uint32_t run = inc - tot;
            for (int w = 0; w < wave; ++w)
                run += scan_tmp[w];
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wc[w][t];
                wc[w][t] = run;
                run += c;
            }
        }
        __syncthreads();
        for (int it = 0; it < kSmallItems; ++it) {
            if (wbase + 64 * it + lane < n) {
                const uint32_t p = wc[wave][dp[it] & 0xFF] + (dp[it] >> 8);
                skey[dst][p] = k[it];
                sval[dst][p] = v[it];
            }
        }
        __syncthreads();  // every read of the starts is done before they are cleared
    }
    // the result goes where the multi-workgroup passes would leave it
    const int fin = npass & 1, ob = (npass - 1) & 1;
    for (int i = t; i < n; i += kSmallThreads) {
        R.sk[ob][i] = skey[fin][i];
        R.sv[ob][i] = sval[fin][i];
    }
    if (step_tail) {
        __syncthreads();  // every read of the control block is done
        if (t < 64) {
            if (R.record_power)
                plane_power_final(R, R.ctl->step, nullptr, 1);  // the first wavefront adds the partial sums
            else if (t == 0) {
                R.ctl->pbuf ^= 1;
                R.ctl->nsort += 1;
                R.ctl->step += 1;
            }
        }
    }
}

bool sort_ends_step(const RunDev &R) { return R.np > 0 && R.np <= kSmallChunk; }

// the sort range as a kernel of its own (after a generic box reduction)
struct SortRange {
    static constexpr int kThreads = 1;
    static __device__ void run(const RunDev &R, Blk) { sort_range(R, false); }
};

// The same passes with every pointer derived from the run, for grouped
// launches over runs of different sizes and key ranges: pass ps of a run
// that needs fewer passes does nothing, and the gather reads the output of
// the run's own last pass.
__host__ __device__ inline int sort_passes_of(uint32_t key_inactive)
{
    int bits = 0;
    while (bits < 32 && (key_inactive >> bits) != 0)
        ++bits;
    return bits <= 8 ? 1 : (bits + 7) / 8;
}

struct RadixHistRun {
    static constexpr int kThreads = kSortThreads;
    static __device__ void run(const RunDev &R, Blk blk, int ps)
    {
        if (ps >= R.ctl->npass || R.np <= 0)
            return;
        const uint32_t *kin = ps == 0 ? R.key_in : R.sk[(ps - 1) & 1];
        radix_hist_blk(kin, R.np, 8 * ps, R.hist, R.sort_blocks, blk.id, R.ctl, R.key_inactive);
    }
};

struct DigitScanRun {
    static constexpr int kThreads = 256;
    static __device__ void run(const RunDev &R, Blk blk, int ps)
    {
        if (ps >= R.ctl->npass || R.np <= 0)
            return;
        digit_scan_blk(R.hist, R.sort_blocks, R.hist + 256 * R.sort_blocks, blk.id);
    }
};

struct RadixScatterRun {
    static constexpr int kThreads = kSortThreads;
    static __device__ void run(const RunDev &R, Blk blk, int ps)
    {
        if (ps >= R.ctl->npass || R.np <= 0)
            return;
        const uint32_t *kin = ps == 0 ? R.key_in : R.sk[(ps - 1) & 1];
        const int32_t *vin = ps == 0 ? R.slot_in : R.sv[(ps - 1) & 1];
        radix_scatter_blk(kin, vin, R.sk[ps & 1], R.sv[ps & 1], R.np, 8 * ps, R.hist, R.sort_blocks,
                          R.hist + 256 * R.sort_blocks, blk.id, R.ctl, R.key_inactive);
    }
};

// ---------------------------------------------------------------------------

hipError_t launch_box_reduce(const RunDev &R, int64_t nblocks, const int32_t *part, int32_t *lo, int32_t *hi,
                             int32_t *count, hipStream_t st);

int sort_passes(uint32_t key_inactive) { return sort_passes_of(key_inactive); }

int64_t sort_blocks(int64_t n) { return (n + kSortChunk - 1) / kSortChunk; }

// keys_ready: the push has already written the keys and the slots, and the
// box reduction after it has set the active-cell box, the count and the
// sort range.  Otherwise (the load) the keys, the box and the range are
// computed here.
hipError_t launch_sort(const RunDev &R, hipStream_t st, bool keys_ready, int step_tail)
{
    if (R.np <= 0)
        return hipSuccess;
    const unsigned pblocks = (unsigned)((R.np + 255) / 256);
    if (!keys_ready)
        hipLaunchKernelGGL(k_sort_keys, dim3(pblocks), dim3(256), 0, st, R);
    if (!keys_ready) {
        hipError_t e = launch_box_reduce(R, pblocks, R.boxpart, CTL_ADDR(R.ctl, cell_lo), CTL_ADDR(R.ctl, cell_hi),
                                         CTL_ADDR(R.ctl, n_active), st);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL((k_run<SortRange>), dim3(1), dim3(1), 0, st, R);
    }
    if (R.np <= kSmallChunk) {
        hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(kSmallThreads), 0, st, R, step_tail);
    } else {
        // as many passes as the widest key range needs; the ones the current
        // range does not need return at once
        const int passes = sort_passes(R.key_inactive);
        const int64_t nb = R.sort_blocks;
        const uint32_t *kin = R.key_in;
        const int32_t *vin = R.slot_in;
        for (int ps = 0; ps < passes; ++ps) {
            uint32_t *kout = R.sk[ps & 1];
            int32_t *vout = R.sv[ps & 1];
            hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, st, kin, R.np, 8 * ps,
                               R.hist, nb, R.ctl, R.key_inactive, ps);
            hipLaunchKernelGGL(k_digit_scan, dim3(256), dim3(256), 0, st, R.hist, nb, R.hist + 256 * nb, R.ctl, ps);
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, st, kin, vin, kout, vout,
                               R.np, 8 * ps, R.hist, nb, R.hist + 256 * nb, R.ctl, R.key_inactive, ps);
            kin = kout;
            vin = vout;
        }
    }
    // the push reads the state through sv[ctl->sorted_buf]
    return hipGetLastError();
}

}  // namespace mithra

// ---------------------------------------------------------------------------
// grouped launches (several runs per launch; see k_group)
// ---------------------------------------------------------------------------
namespace mithra {

// gs: members with sort_blocks workgroups; gd: 256 workgroups each (one
// per digit); the key range was set by the box reduction before (gp unused)
hipError_t launch_sort_group(const Group &gs, int64_t total_s, const Group &gd, int64_t total_d, const Group &gp,
                             int64_t total_p, int max_passes, hipStream_t st)
{
    if (total_p <= 0)
        return hipSuccess;
    (void)gp;
    (void)total_p;
    for (int ps = 0; ps < max_passes; ++ps) {
        hipLaunchKernelGGL((k_group<RadixHistRun, int>), dim3((unsigned)total_s), dim3(kSortThreads), 0, st, gs, ps);
        hipLaunchKernelGGL((k_group<DigitScanRun, int>), dim3((unsigned)total_d), dim3(256), 0, st, gd, ps);
        hipLaunchKernelGGL((k_group<RadixScatterRun, int>), dim3((unsigned)total_s), dim3(kSortThreads), 0, st, gs, ps);
    }
    return hipGetLastError();
}

}  // namespace mithra
