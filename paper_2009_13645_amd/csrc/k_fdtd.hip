// k_fdtd.hip -- field kernels of the boosted-frame PIC step.
//
//  * Sweep / SweepVec: NSFD update of A_x, A_y, A_z and phi at interior
//    nodes (MITHRA 2.0 manual, sec. "FDTD for Wave Equation", eqs. NSFDtrick
//    and updateEquation; sec. "FDTD for Scalar Potential").  HBM-bound
//    15-point stencil: each thread owns one (i,j) column of a TX x TY tile
//    and marches along z with a register queue of psi^n(k-1..k+1); the
//    z-averaged value psi-bar of every column (plus a one-column halo ring)
//    goes through a double-buffered LDS plane, so psi^n is read from HBM
//    about once.  The source of the step (node-averaged edge current, or
//    rho) is read only inside the bounding box of the last deposit.
//  * Mur: Mur absorbing boundaries (sec. "Boundary Truncation"), one thread
//    per boundary face node.  Faces use the printed first/second-order
//    updates with permuted axes; further workgroups of the face launch clear
//    the other source set inside its own box for the coming deposit.  Edges
//    and corners (MurEdge, mur_dev.hpp) follow in a later launch: they solve
//    the sum of the first-order conditions of their faces discretised at the
//    centre of the 2x2 (2x2x2) node stencil, reading the new face values (a
//    corner recomputes its edge neighbours).  Three time levels make all
//    reads race-free.
//  * VertexFields: E and B at vertices (sec. "Field Evaluation"):
//    E = -(A^{n+1} - A^n)/dt - grad phi, B = mean of curl A^n and curl A^{n+1}.
#include "mithra_dev.hpp"
#include "mur_dev.hpp"
#include <algorithm>
#include <type_traits>

namespace mithra {

// ---------------------------------------------------------------------------
// K1: NSFD sweep
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline T src_value(const RunDev &R, int comp, int set, int64_t c, int64_t back)
{
    // node-averaged edge current along comp, or rho; scaled to the update
    if (comp < 3) {
        const T *J = src_ptr<T>(R, set, comp);
        double s = (double)J[c] + (double)J[c - back];
        if (R.compensated) {
            const T *L = srclo_ptr<T>(R, set, comp);
            s += (double)L[c] + (double)L[c - back];
        }
        return (T)(R.sfac_A * 0.5 * s);
    }
    const T *Q = src_ptr<T>(R, set, 3);
    double s = (double)Q[c];
    if (R.compensated)
        s += (double)srclo_ptr<T>(R, set, 3)[c];
    return (T)(R.sfac_phi * s);
}

// FP32 sweeps use the difference form of the update,
//   psi^{n+1} = psi + [(psi - psi^{n-1}) + rx2 (d_xx psi + d_xx c)
//               + ry2 (d_yy psi + d_yy c) + rz2 d_zz psi + S],
//   c = psi-bar - psi = A ((psi_{k-1} - psi) + (psi_{k+1} - psi)),
// with every second difference formed from neighbour differences: for a
// smooth field those are exact in FP32, and psi enters once per step, so the
// rounding the leapfrog integrates is relative to the increment instead of
// to psi.  It is the same update as eq. updateEquation (its coefficients
// summed); FP64 sweeps keep the coefficient form.
template <typename T>
constexpr bool kDiffForm = sizeof(T) == 4;

template <typename T, int TX, int TY, int TZ>
struct Sweep {
    static constexpr int kThreads = TX * TY;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        __shared__ T sb[2][TY + 2][TX + 2];
        // difference form: psi-bar - psi of the same node
        __shared__ T sbc[kDiffForm<T> ? 2 : 1][kDiffForm<T> ? TY + 2 : 1][TX + 2];

        // tiles start at node 0 so that every row load is 128-byte aligned; the
        // boundary columns load (they are the neighbours of the first interior
        // column) but are not updated
        const int ntx = (R.nx + TX - 1) / TX;
        const int nty = (R.ny + TY - 1) / TY;
        const int nch = (R.nz - 2 + TZ - 1) / TZ;
        int64_t lb = xcd_swizzle(blk.id, blk.n);
        const int tile_x = (int)(lb % ntx);
        lb /= ntx;
        const int tile_y = (int)(lb % nty);
        lb /= nty;
        const int chunk = (int)(lb % nch);
        const int comp = (int)(lb / nch);
        if (comp >= 4)
            return;  // grid larger than the tiling (never for the launchers here)

        const int64_t s = R.ctl->step;
        const int set_r = (int)(s & 1);
        const bool update = (comp < 3) || R.space_charge;

        const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
        const int i = tile_x * TX + lx;
        const int j = tile_y * TY + ly;
        const bool inb = (i < R.nx) && (j < R.ny);
        const bool valid = (i >= 1) && (j >= 1) && (i <= R.nx - 2) && (j <= R.ny - 2);
        const int ic = min(i, R.nx - 1), jc = min(j, R.ny - 1);
        const int64_t plane = (int64_t)R.nx * R.ny;
        const int64_t col = (int64_t)jc * R.nx + ic;

        // halo ring: left/right columns (TY each), bottom/top rows (TX each)
        const int H = 2 * (TX + TY);
        const int h = threadIdx.x;
        int hx = 0, hy = 0, hi_ = 0, hj_ = 0;
        bool hval = false;
        if (h < H) {
            if (h < TY) {
                hx = -1; hy = h;
            } else if (h < 2 * TY) {
                hx = TX; hy = h - TY;
            } else if (h < 2 * TY + TX) {
                hy = -1; hx = h - 2 * TY;
            } else {
                hy = TY; hx = h - 2 * TY - TX;
            }
            hi_ = tile_x * TX + hx;
            hj_ = tile_y * TY + hy;
            hval = (hi_ >= 0) && (hi_ < R.nx) && (hj_ >= 0) && (hj_ < R.ny);
        }
        const int64_t hcol = hval ? ((int64_t)hj_ * R.nx + hi_) : 0;

        const int kb = 1 + chunk * TZ;
        const int ke = min(kb + TZ, R.nz - 1);

        const T *cur = pot_ptr<T>(R, slot_cur(s), comp);
        const T *prev = pot_ptr<T>(R, slot_prev(s), comp);
        T *next = pot_ptr<T>(R, slot_next(s), comp);

        // source box of the set read now (expanded by one node on the high side:
        // a node average reaches the edge below it)
        const int *rlo = R.ctl->dep_lo[set_r];
        const int *rhi = R.ctl->dep_hi[set_r];
        const bool src_col = valid && i >= rlo[0] && i <= rhi[0] + 1 && j >= rlo[1] && j <= rhi[1] + 1;
        const int64_t back = comp == 0 ? 1 : (comp == 1 ? R.nx : plane);

        const T cA = (T)R.A, c1A = (T)(1.0 - 2.0 * R.A);
        const T a1 = (T)R.a1, a2 = (T)R.a2, a4 = (T)R.a4, a6 = (T)R.a6;
        const T rx2 = (T)R.rx2, ry2 = (T)R.ry2, rz2 = (T)R.rz2;

        T qm = 0, q0 = 0, qp = 0, hqm = 0, hq0 = 0, hqp = 0;
        if (inb) {
            qm = cur[(int64_t)(kb - 1) * plane + col];
            q0 = cur[(int64_t)kb * plane + col];
            qp = cur[(int64_t)(kb + 1) * plane + col];
        }
        if (hval) {
            hqm = cur[(int64_t)(kb - 1) * plane + hcol];
            hq0 = cur[(int64_t)kb * plane + hcol];
            hqp = cur[(int64_t)(kb + 1) * plane + hcol];
        }

        for (int k = kb; k < ke; ++k) {
            const int64_t c = (int64_t)k * plane + col;
            // issue the loads of this iteration before the barrier
            T pf = 0, hpf = 0;
            if (k + 1 < ke) {
                if (inb)
                    pf = cur[c + 2 * plane];
                if (hval)
                    hpf = cur[(int64_t)(k + 2) * plane + hcol];
            }
            T pm = 0, sv = 0;
            if (valid && update) {
                pm = prev[c];
                if (src_col && k >= rlo[2] && k <= rhi[2] + 1)
                    sv = src_value<T>(R, comp, set_r, c, back);
            }
            T(*buf)[TX + 2] = sb[k & 1];
            if constexpr (kDiffForm<T>) {
                T(*cbuf)[TX + 2] = sbc[k & 1];
                buf[ly + 1][lx + 1] = q0;
                cbuf[ly + 1][lx + 1] = cA * ((qm - q0) + (qp - q0));
                if (h < H) {
                    buf[hy + 1][hx + 1] = hq0;
                    cbuf[hy + 1][hx + 1] = cA * ((hqm - hq0) + (hqp - hq0));
                }
            } else {
                buf[ly + 1][lx + 1] = cA * (qm + qp) + c1A * q0;
                if (h < H)
                    buf[hy + 1][hx + 1] = cA * (hqm + hqp) + c1A * hq0;
            }
            __syncthreads();
            if (valid && update) {
                if constexpr (kDiffForm<T>) {
                    T(*cbuf)[TX + 2] = sbc[k & 1];
                    const T c0 = cbuf[ly + 1][lx + 1];
                    const T dxx = ((buf[ly + 1][lx] - q0) + (buf[ly + 1][lx + 2] - q0)) +
                                  ((cbuf[ly + 1][lx] - c0) + (cbuf[ly + 1][lx + 2] - c0));
                    const T dyy = ((buf[ly][lx + 1] - q0) + (buf[ly + 2][lx + 1] - q0)) +
                                  ((cbuf[ly][lx + 1] - c0) + (cbuf[ly + 2][lx + 1] - c0));
                    const T dzz = (qm - q0) + (qp - q0);
                    next[c] = q0 + ((q0 - pm) + rx2 * dxx + ry2 * dyy + rz2 * dzz + sv);
                } else {
                    T v = a1 * q0 + a2 * (buf[ly + 1][lx + 2] + buf[ly + 1][lx]) +
                          a4 * (buf[ly + 2][lx + 1] + buf[ly][lx + 1]) + a6 * (qp + qm) - pm + sv;
                    next[c] = v;
                }
            }
            qm = q0;
            q0 = qp;
            qp = pf;
            hqm = hq0;
            hq0 = hqp;
            hqp = hpf;
        }
    }
};

// Vectorised sweep: each thread owns V consecutive x-nodes (16-byte loads
// and stores), a tile is TXV*V nodes wide and TY rows high.  psi-bar of the
// tile plus a one-node halo ring goes through a double-buffered LDS plane
// whose interior starts on a 16-byte boundary; a thread reads its two outer
// x-neighbours and its y-neighbour vectors from LDS.  Needs nx % V == 0 so
// that every row starts aligned.
// Streaming (non-temporal) 16-byte accesses: data touched once per sweep
// (psi^{n-1} and psi^{n+1}) bypass cache retention so
// that the psi^n stencil planes stay in L2.
typedef unsigned int nt_u32x4 __attribute__((ext_vector_type(4)));

template <typename T, int V>
__device__ inline void vstore_nt(T *p, const Vec<T, V> &a)
{
    static_assert(sizeof(T) * V == 16, "16-byte vectors only");
    nt_u32x4 w;
    memcpy(&w, &a, 16);
    __builtin_nontemporal_store(w, reinterpret_cast<nt_u32x4 *>(p));
}

template <typename T, int V>
__device__ inline Vec<T, V> vload_nt(const T *p)
{
    static_assert(sizeof(T) * V == 16, "16-byte vectors only");
    const nt_u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const nt_u32x4 *>(p));
    Vec<T, V> r;
    memcpy(&r, &w, 16);
    return r;
}

// Sources of one thread's V nodes on one plane: own edge/node values (a),
// the edge one step back along the component's axis (b, vector) or the
// left neighbour of the first node (lf, x component), with the two-sum low
// parts when compensated.
template <typename T, int V, bool LO>
struct PlaneSrc {
    Vec<T, V> pm, a, al, b, bl;
    T lf, lfl;
};

template <typename T, int V, int TXV, int TY, int TZ, bool LO>
struct SweepVec {
    static constexpr int kThreads = TXV * TY;
    static constexpr bool kCopyRun = true;  // see CopyRunOf
    static_assert(TZ % 4 == 0, "planes are processed four at a time");
    static constexpr int TW = TXV * V;                          // tile width in nodes
    static constexpr int ROW = ((V + TW + 1) + V - 1) / V * V;  // LDS row: pad(V-1), left halo, tile, right halo
    // source sums: FP64 for FP64 fields and for compensated FP32 (hi + lo)
    using ST = typename std::conditional<LO || sizeof(T) == 8, double, T>::type;
    struct Lds {
        __attribute__((aligned(16))) T sb[2][TY + 2][ROW];
        // difference form (FP32): psi-bar - psi of the same node
        __attribute__((aligned(16))) T sbc[kDiffForm<T> ? 2 : 1][kDiffForm<T> ? TY + 2 : 1][ROW];
        // psi^n at the two outermost nodes of each row end (x-face update)
        T rawe[2][TY + 2][4];
        // source row ranges of the tile's rows for the chunk's planes
        int2 sr[TZ][TY];
    };

    static __device__ __attribute__((always_inline)) void run(const RunDev &R, Blk blk)
    {
        __shared__ Lds L;
        const int ntx = (R.nx + TW - 1) / TW;
        const int nty = (R.ny + TY - 1) / TY;
        const int nch = (R.nz - 2 + TZ - 1) / TZ;
        int64_t lb = xcd_swizzle(blk.id, blk.n);
        const int tile_x = (int)(lb % ntx);
        lb /= ntx;
        const int tile_y = (int)(lb % nty);
        lb /= nty;
        const int chunk = (int)(lb % nch);
        const int comp = (int)(lb / nch);
        if (comp >= 4)
            return;  // grid larger than the tiling (never for the launchers here)
        if (comp == 3 && !R.space_charge)
            return;  // phi is not advanced without space charge (uniform per workgroup)
        // the component is a compile-time constant inside the body, so the
        // source loads of the other components do not exist there
        switch (comp) {
        case 0: body<0>(R, L, tile_x, tile_y, chunk); break;
        case 1: body<1>(R, L, tile_x, tile_y, chunk); break;
        case 2: body<2>(R, L, tile_x, tile_y, chunk); break;
        default: body<3>(R, L, tile_x, tile_y, chunk); break;
        }
    }

    template <int COMP>
    static __device__ __attribute__((always_inline)) void body(const RunDev &R, Lds &L, int tile_x, int tile_y,
                                                               int chunk)
    {
        const int64_t s = R.ctl->step;
        const int set_r = (int)(s & 1);

        const int lx = threadIdx.x % TXV, ly = threadIdx.x / TXV;
        const int i0 = tile_x * TW + lx * V;  // first node of this thread
        const int j = tile_y * TY + ly;
        const bool inb = (i0 < R.nx) && (j < R.ny);
        const bool work = inb && j >= 1 && j <= R.ny - 2;
        const int64_t plane = (int64_t)R.nx * R.ny;
        const int64_t col = inb ? ((int64_t)j * R.nx + i0) : 0;

        // Halo: bottom/top rows (TXV threads each), left/right columns (TY
        // threads each).  Every thread issues one aligned 16-byte halo load
        // per plane, so that no load is conditional: a column thread loads
        // the vector holding its node (element hsel), a thread without a
        // halo node reloads its own vector.
        const int t = threadIdx.x;
        int hrole = -1, hx = 0, hy = 0, hsel = 0;
        int64_t hv = col;
        bool hval = false;
        if (t < 2 * TXV) {
            hrole = 0;
            hx = (t % TXV) * V;
            hy = t < TXV ? -1 : TY;
            const int hi_ = tile_x * TW + hx, hj_ = tile_y * TY + hy;
            hval = hj_ >= 0 && hj_ < R.ny && hi_ < R.nx;
            if (hval)
                hv = (int64_t)hj_ * R.nx + hi_;
        } else if (t < 2 * TXV + 2 * TY) {
            hrole = 1;
            const int u = t - 2 * TXV;
            hy = u % TY;
            hx = u < TY ? -1 : TW;
            const int hi_ = tile_x * TW + hx, hj_ = tile_y * TY + hy;
            hval = hi_ >= 0 && hi_ < R.nx && hj_ < R.ny;
            hsel = hx < 0 ? V - 1 : 0;
            if (hval)
                hv = (int64_t)hj_ * R.nx + hi_ - hsel;
        }

        const int kb = 1 + chunk * TZ;
        const int ke = min(kb + TZ, R.nz - 1);
        const T *cur = pot_ptr<T>(R, slot_cur(s), COMP);
        const T *prev = pot_ptr<T>(R, slot_prev(s), COMP);
        T *next = pot_ptr<T>(R, slot_next(s), COMP);

        const int *rlo = R.ctl->dep_lo[set_r];
        const int *rhi = R.ctl->dep_hi[set_r];
        const bool src_col = work && i0 + V - 1 >= rlo[0] && i0 <= rhi[0] + 1 && j >= rlo[1] && j <= rhi[1] + 1;
        const int sk_lo = rlo[2], sk_hi = rhi[2] + 1;
        // the source row ranges of the set for the tile's rows and the
        // chunk's planes, through LDS (rows and planes clamped into the grid;
        // a clamped entry is never used for a stored node)
        {
            const int32_t *srl = R.srow_lo + (size_t)set_r * R.nz * R.ny;
            const int32_t *srh = R.srow_hi + (size_t)set_r * R.nz * R.ny;
            for (int e = threadIdx.x; e < TZ * TY; e += kThreads) {
                const int pz = e / TY, py = e - pz * TY;
                const int64_t row = (int64_t)min(kb + pz, R.nz - 1) * R.ny + min(tile_y * TY + py, R.ny - 1);
                L.sr[pz][py] = make_int2(srl[row], srh[row]);
            }
            __syncthreads();
        }
        const T *J = src_ptr<T>(R, set_r, COMP);
        const T *Jl = LO ? srclo_ptr<T>(R, set_r, COMP) : nullptr;
        const ST sfac = (ST)(COMP < 3 ? 0.5 * R.sfac_A : R.sfac_phi);

        const T cA = (T)R.A, c1A = (T)(1.0 - 2.0 * R.A);
        const T a1 = (T)R.a1, a2 = (T)R.a2, a4 = (T)R.a4, a6 = (T)R.a6;
        const T rx2 = (T)R.rx2, ry2 = (T)R.ry2, rz2 = (T)R.rz2;
        const int kmax = R.nz - 1;

        // psi^n of plane kk (own vector and halo vector); every plane index
        // is clamped into the array, so the loads need no guard
        auto load_cur = [&](int kk, Vec<T, V> &q, Vec<T, V> &h) {
            const int64_t o = (int64_t)min(kk, kmax) * plane;
            q = vload<T, V>(cur + o + col);
            h = vload<T, V>(cur + o + hv);
        };
        // psi^{n-1} and the sources of plane kk (kk <= nz - 1).  Outside the
        // source box the source loads read node 0, which no deposit reaches
        // and which therefore holds zero; the z component's back edge is the
        // previous plane's own edge, carried in registers.
        auto fetch = [&](int kk, const PlaneSrc<T, V, LO> &prv, PlaneSrc<T, V, LO> &r) {
            const int64_t c = (int64_t)kk * plane + col;
            r.pm = vload_nt<T, V>(prev + c);
            // planes at or beyond ke are not stored: no source needed
            const int2 rg = L.sr[min(kk - kb, TZ - 1)][ly];
            const bool in = src_col && kk >= sk_lo && kk <= sk_hi && kk < ke && i0 + V - 1 >= rg.x && i0 <= rg.y;
            const int64_t ca = in ? c : 0;
            r.a = vload<T, V>(J + ca);
            if constexpr (LO)
                r.al = vload<T, V>(Jl + ca);
            if constexpr (COMP == 0) {
                const int64_t cl = in ? c - 1 : 0;
                r.lf = J[cl];
                if constexpr (LO)
                    r.lfl = Jl[cl];
            } else if constexpr (COMP == 1) {
                const int64_t cb = in ? c - R.nx : 0;
                r.b = vload<T, V>(J + cb);
                if constexpr (LO)
                    r.bl = vload<T, V>(Jl + cb);
            } else if constexpr (COMP == 2) {
                if (kk > kb) {
                    r.b = prv.a;
                    if constexpr (LO)
                        r.bl = prv.al;
                } else {
                    const int64_t cb = in ? c - plane : 0;
                    r.b = vload<T, V>(J + cb);
                    if constexpr (LO)
                        r.bl = vload<T, V>(Jl + cb);
                }
            }
        };

        // Plane k from the psi^n planes k-1, k, k+1 (qm, q0, qp; halo hm,
        // h0, hp) and the psi^{n-1} / source plane ps; the loads of plane
        // k+2 (pf, hpf) and of plane k+1 (pn) are issued first.  The caller
        // rotates the roles of the variables instead of copying them, so a
        // prefetch stays in flight across planes.  Planes at or beyond ke
        // (only in a chunk's last group of four) are computed and not stored.
        auto plane_step = [&](int k, const Vec<T, V> &qm, const Vec<T, V> &q0, const Vec<T, V> &qp, Vec<T, V> &pf,
                              const Vec<T, V> &hm, const Vec<T, V> &h0, const Vec<T, V> &hp, Vec<T, V> &hpf,
                              const PlaneSrc<T, V, LO> &ps, PlaneSrc<T, V, LO> &pn) {
            const int64_t c = (int64_t)k * plane + col;
            load_cur(k + 2, pf, hpf);
            fetch(min(k + 1, kmax), ps, pn);
            ST sv[V];
            if constexpr (COMP == 3) {
                for (int e = 0; e < V; ++e)
                    sv[e] = (ST)ps.a.v[e] + (LO ? (ST)ps.al.v[e] : (ST)0);
            } else if constexpr (COMP == 0) {
                ST left = (ST)ps.lf + (LO ? (ST)ps.lfl : (ST)0);
                for (int e = 0; e < V; ++e) {
                    const ST own = (ST)ps.a.v[e] + (LO ? (ST)ps.al.v[e] : (ST)0);
                    sv[e] = own + left;
                    left = own;
                }
            } else {
                for (int e = 0; e < V; ++e)
                    sv[e] = LO ? ((ST)ps.a.v[e] + (ST)ps.al.v[e]) + ((ST)ps.b.v[e] + (ST)ps.bl.v[e])
                               : (ST)ps.a.v[e] + (ST)ps.b.v[e];
            }
            T(*buf)[ROW] = L.sb[k & 1];
            // a column thread's halo node is element hsel of its vector
            const bool hl = hsel != 0;
            const T h0s = hl ? h0.v[V - 1] : h0.v[0], hms = hl ? hm.v[V - 1] : hm.v[0], hps = hl ? hp.v[V - 1] : hp.v[0];
            Vec<T, V> bar;  // psi-bar, or (difference form) psi-bar - psi
            if constexpr (kDiffForm<T>) {
                T(*cbuf)[ROW] = L.sbc[k & 1];
                for (int e = 0; e < V; ++e)
                    bar.v[e] = cA * ((qm.v[e] - q0.v[e]) + (qp.v[e] - q0.v[e]));
                vstore<T, V>(&buf[ly + 1][V + lx * V], q0);
                vstore<T, V>(&cbuf[ly + 1][V + lx * V], bar);
                if (hrole == 0) {
                    Vec<T, V> hb;
                    for (int e = 0; e < V; ++e)
                        hb.v[e] = cA * ((hm.v[e] - h0.v[e]) + (hp.v[e] - h0.v[e]));
                    vstore<T, V>(&buf[hy + 1][V + hx], h0);
                    vstore<T, V>(&cbuf[hy + 1][V + hx], hb);
                } else if (hrole == 1) {
                    buf[hy + 1][V + hx] = h0s;
                    cbuf[hy + 1][V + hx] = cA * ((hms - h0s) + (hps - h0s));
                }
            } else {
                for (int e = 0; e < V; ++e)
                    bar.v[e] = cA * (qm.v[e] + qp.v[e]) + c1A * q0.v[e];
                vstore<T, V>(&buf[ly + 1][V + lx * V], bar);
                if (hrole == 0) {
                    Vec<T, V> hb;
                    for (int e = 0; e < V; ++e)
                        hb.v[e] = cA * (hm.v[e] + hp.v[e]) + c1A * h0.v[e];
                    vstore<T, V>(&buf[hy + 1][V + hx], hb);
                } else if (hrole == 1) {
                    buf[hy + 1][V + hx] = cA * (hms + hps) + c1A * h0s;
                }
            }
            {
                T(*raw)[4] = L.rawe[k & 1];
                if (inb && i0 == 0) {
                    raw[ly + 1][0] = q0.v[0];
                    raw[ly + 1][1] = q0.v[1];
                }
                if (inb && i0 + V == R.nx) {
                    raw[ly + 1][2] = q0.v[V - 2];
                    raw[ly + 1][3] = q0.v[V - 1];
                }
                if (hrole == 0 && hval) {
                    const int hi_ = tile_x * TW + hx;
                    if (hi_ == 0) {
                        raw[hy + 1][0] = h0.v[0];
                        raw[hy + 1][1] = h0.v[1];
                    }
                    if (hi_ + V == R.nx) {
                        raw[hy + 1][2] = h0.v[V - 2];
                        raw[hy + 1][3] = h0.v[V - 1];
                    }
                }
            }
            __syncthreads();
            if (work && k < ke) {
                const T left = buf[ly + 1][V + lx * V - 1];
                const T right = buf[ly + 1][V + lx * V + V];
                const Vec<T, V> dn = vload<T, V>(&buf[ly][V + lx * V]);
                const Vec<T, V> up = vload<T, V>(&buf[ly + 2][V + lx * V]);
                Vec<T, V> out;
                if constexpr (kDiffForm<T>) {
                    T(*cbuf)[ROW] = L.sbc[k & 1];
                    const T cleft = cbuf[ly + 1][V + lx * V - 1];
                    const T cright = cbuf[ly + 1][V + lx * V + V];
                    const Vec<T, V> cdn = vload<T, V>(&cbuf[ly][V + lx * V]);
                    const Vec<T, V> cup = vload<T, V>(&cbuf[ly + 2][V + lx * V]);
                    for (int e = 0; e < V; ++e) {
                        const T p0 = q0.v[e], c0 = bar.v[e];
                        const T ql = e == 0 ? left : q0.v[e - 1], qr = e == V - 1 ? right : q0.v[e + 1];
                        const T cl = e == 0 ? cleft : bar.v[e - 1], cr = e == V - 1 ? cright : bar.v[e + 1];
                        const T dxx = ((ql - p0) + (qr - p0)) + ((cl - c0) + (cr - c0));
                        const T dyy = ((dn.v[e] - p0) + (up.v[e] - p0)) + ((cdn.v[e] - c0) + (cup.v[e] - c0));
                        const T dzz = (qm.v[e] - p0) + (qp.v[e] - p0);
                        out.v[e] = p0 + ((p0 - ps.pm.v[e]) + rx2 * dxx + ry2 * dyy + rz2 * dzz + (T)(sfac * sv[e]));
                    }
                } else {
                    for (int e = 0; e < V; ++e) {
                        const T xl = e == 0 ? left : bar.v[e - 1];
                        const T xr = e == V - 1 ? right : bar.v[e + 1];
                        out.v[e] = a1 * q0.v[e] + a2 * (xl + xr) + a4 * (dn.v[e] + up.v[e]) +
                                   a6 * (qp.v[e] + qm.v[e]) - ps.pm.v[e] + (T)(sfac * sv[e]);
                    }
                }
                // the x-face nodes of the row: Mur update (faces of the x
                // axis, transverse y and z), from this thread's own columns,
                // the neighbouring rows' values in LDS and the new inner
                // value.  When the Mur kernel also updates the x faces (a
                // scalar shape is the run's own), it runs after this kernel
                // and its values replace these.
                if (i0 == 0 || i0 + V == R.nx) {
                    const T(*raw)[4] = L.rawe[k & 1];
                    for (int side = 0; side < 2; ++side) {
                        if ((side == 0 && i0 != 0) || (side == 1 && i0 + V != R.nx))
                            continue;
                        const int eb = side == 0 ? 0 : V - 1, ei = side == 0 ? 1 : V - 2;
                        const int ro = side == 0 ? 0 : 2;
                        const int rb = side == 0 ? ro : ro + 1, ri = side == 0 ? ro + 1 : ro;
                        const Vec<T, V> &pm = ps.pm;
                        double v = R.mur_be0[0] * ((double)pm.v[eb] + (double)out.v[ei]) - (double)pm.v[ei];
                        if (R.order == 1) {
                            v += R.mur_be1[0] * ((double)q0.v[eb] + (double)q0.v[ei]);
                        } else {
                            v += R.mur_g1[0] * ((double)q0.v[eb] + (double)q0.v[ei]);
                            const double s1 = ((double)raw[ly][rb] + (double)raw[ly][ri]) +
                                              ((double)raw[ly + 2][rb] + (double)raw[ly + 2][ri]);
                            const double s2 = ((double)qm.v[eb] + (double)qm.v[ei]) + ((double)qp.v[eb] + (double)qp.v[ei]);
                            v += R.mur_ga[0] * s1;
                            v += R.mur_gb[0] * s2;
                        }
                        out.v[eb] = (T)v;
                    }
                }
                vstore_nt<T, V>(next + c, out);
            }
        };

        Vec<T, V> qm, q0, qp, pf, hm, h0, hp, hpf;
        load_cur(kb - 1, qm, hm);
        load_cur(kb, q0, h0);
        load_cur(kb + 1, qp, hp);
        PlaneSrc<T, V, LO> ps{}, pn{};
        fetch(kb, pn, ps);
        // four planes per iteration, the variables' roles rotating by one
        // plane each time (a period of four for the psi^n queues, two for
        // the psi^{n-1} / source planes); the last group of a chunk may run
        // up to three planes past ke, computed and not stored
        for (int k = kb; k < ke; k += 4) {
            plane_step(k, qm, q0, qp, pf, hm, h0, hp, hpf, ps, pn);
            plane_step(k + 1, q0, qp, pf, qm, h0, hp, hpf, hm, pn, ps);
            plane_step(k + 2, qp, pf, qm, q0, hp, hpf, hm, h0, ps, pn);
            plane_step(k + 3, pf, qm, q0, qp, hpf, hm, h0, hp, pn, ps);
        }
    }
};

// ---------------------------------------------------------------------------
// K2: Mur boundaries
// ---------------------------------------------------------------------------

// r / d for 0 <= r < half (r = row * d + column of a face): multiply-high
// when exact, else 64-bit division
__device__ inline uint32_t face_div(int64_t r, int64_t half, int d)
{
    if ((uint64_t)half * (uint64_t)d < (1ull << 32))
        return fdiv((uint32_t)r, fast_div((uint32_t)d));
    return (uint32_t)(r / d);
}

// The source set that this step's deposit accumulates into is zeroed on the
// node box of its previous deposit, every component.  The set was last read
// by the previous step's sweep, and the deposit runs after this kernel.
// One wavefront per x-row of the box; row indices are wavefront-uniform.
template <typename T>
__device__ inline void clear_next_sources(const RunDev &R, int64_t b, int64_t nb)
{
    const int64_t s = R.ctl->step;
    const int set_c = (int)((s + 1) & 1);
    const int *lo = R.ctl->dep_lo[set_c];
    const int *hi = R.ctl->dep_hi[set_c];
    const int l0 = lo[0], l1 = lo[1], l2 = lo[2];
    const int ex = hi[0] - l0 + 1, ey = hi[1] - l1 + 1, ez = hi[2] - l2 + 1;
    if (ex <= 0 || ey <= 0 || ez <= 0)
        return;
    // the set's source row ranges, on the rows the deposit's boxes may have
    // grown them to (one more node along y and z)
    {
        int32_t *slo = R.srow_lo + (size_t)set_c * R.nz * R.ny;
        int32_t *shi = R.srow_hi + (size_t)set_c * R.nz * R.ny;
        const int ry = ey + 1, nr = ry * (ez + 1);
        for (int64_t r = b * blockDim.x + threadIdx.x; r < nr; r += nb * blockDim.x) {
            const int64_t row = (int64_t)(l2 + (int)(r / ry)) * R.ny + (l1 + (int)(r % ry));
            slo[row] = 0x7f7f7f7f;
            shi[row] = -1;
        }
    }
    const uint32_t rows = (uint32_t)ey * (uint32_t)ez;
    const uint32_t nw = (uint32_t)nb * (blockDim.x / 64);
    const uint32_t w0 = __builtin_amdgcn_readfirstlane((uint32_t)b * (blockDim.x / 64) + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    // row r = k ey + j; the stride nw advances (j, k) by (nw % ey, nw / ey)
    // with a carry, so only the first row of a wavefront needs a division
    const uint32_t dk = nw / (uint32_t)ey, dj = nw - dk * (uint32_t)ey;
    const uint32_t k0 = w0 / (uint32_t)ey, j0 = w0 - k0 * (uint32_t)ey;
    const int64_t sy = R.nx, sz = (int64_t)R.nx * R.ny;
    for (int comp = 0; comp < 4; ++comp) {
        T *dst = src_ptr<T>(R, set_c, comp) + nid(R, l0, l1, l2);
        T *dlo = R.compensated ? srclo_ptr<T>(R, set_c, comp) + nid(R, l0, l1, l2) : nullptr;
        uint32_t j = j0, k = k0;
        for (uint32_t r = w0; r < rows; r += nw) {
            const int64_t row = (int64_t)k * sz + (int64_t)j * sy;
            for (int i = lane; i < ex; i += 64) {
                dst[row + i] = (T)0;
                if (dlo)
                    dlo[row + i] = (T)0;
            }
            j += dj;
            k += dk;
            if (j >= (uint32_t)ey) {
                j -= (uint32_t)ey;
                ++k;
            }
        }
    }
}

// workgroups that clear the next source set, after the Mur workgroups
static __host__ __device__ inline int64_t clear_blocks_of(int ny, int nz)
{
    const int64_t r = (int64_t)ny * nz / 64;
    return r < 8 ? 8 : (r > 2048 ? 2048 : r);
}

// Face nodes of the boundary, one thread each (per component): z faces, y
// faces, and the x faces unless the vector sweep updated them, with direct
// strides, laid out x fastest so that their accesses coalesce.  The
// workgroups after the boundary ones clear the next source set
// (clear_next_sources).  Edge and corner nodes follow in MurEdge.
template <typename T>
struct Mur {
    static constexpr int kThreads = 256;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        const int nx = R.nx, ny = R.ny, nz = R.nz;
        const int64_t fz = 2LL * (nx - 2) * (ny - 2);
        const int64_t fy = 2LL * (nx - 2) * (nz - 2);
        const int64_t fx = R.xface_fused ? 0 : 2LL * (ny - 2) * (nz - 2);
        const int64_t nb = fz + fy + fx;
        // ceil(nb / 256) workgroups per component (component uniform per
        // workgroup), then the workgroups that clear the next source set
        const int64_t bpc = (nb + 255) / 256;
        const int64_t nmur = bpc * (R.space_charge ? 4 : 3);
        if (blk.id >= nmur) {
            clear_next_sources<T>(R, blk.id - nmur, blk.n - nmur);
            return;
        }
        const int comp = (int)(blk.id / bpc);
        int64_t r = (blk.id - (int64_t)comp * bpc) * blockDim.x + threadIdx.x;
        if (r >= nb)
            return;
        const int64_t s = R.ctl->step;
        const T *pm = pot_ptr<T>(R, slot_prev(s), comp);
        const T *p0 = pot_ptr<T>(R, slot_cur(s), comp);
        T *pp = pot_ptr<T>(R, slot_next(s), comp);
        int p[3], ax;
        if (r < fz) {
            const int64_t half = (int64_t)(nx - 2) * (ny - 2);
            ax = 2;
            p[2] = r < half ? 0 : nz - 1;
            if (r >= half)
                r -= half;
            const uint32_t q = face_div(r, half, nx - 2);
            p[0] = 1 + (int)(r - (int64_t)q * (nx - 2));
            p[1] = 1 + (int)q;
        } else if (r < fz + fy) {
            r -= fz;
            const int64_t half = (int64_t)(nx - 2) * (nz - 2);
            ax = 1;
            p[1] = r < half ? 0 : ny - 1;
            if (r >= half)
                r -= half;
            const uint32_t q = face_div(r, half, nx - 2);
            p[0] = 1 + (int)(r - (int64_t)q * (nx - 2));
            p[2] = 1 + (int)q;
        } else {
            r -= fz + fy;
            const int64_t half = (int64_t)(ny - 2) * (nz - 2);
            ax = 0;
            p[0] = r < half ? 0 : nx - 1;
            if (r >= half)
                r -= half;
            const uint32_t q = face_div(r, half, ny - 2);
            p[1] = 1 + (int)(r - (int64_t)q * (ny - 2));
            p[2] = 1 + (int)q;
        }
        // strides and coefficients of the normal axis by selects (no array
        // indexed at run time)
        const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
        const int64_t sn = ax == 0 ? sx : (ax == 1 ? sy : sz);
        const int64_t s1 = ax == 0 ? sy : (ax == 1 ? sz : sx), s2 = ax == 0 ? sz : (ax == 1 ? sx : sy);
        auto co = [ax](const double (&a)[3]) { return ax == 0 ? a[0] : (ax == 1 ? a[1] : a[2]); };
        const int pa = ax == 0 ? p[0] : (ax == 1 ? p[1] : p[2]);
        const int side = pa == 0 ? -1 : 1;
        const int64_t c = ((int64_t)p[2] * ny + p[1]) * nx + p[0];
        const int64_t q = c - side * sn;  // first node inside
        double v = co(R.mur_be0) * ((double)pm[c] + (double)pp[q]) - (double)pm[q];
        if (R.order == 1) {
            v += co(R.mur_be1) * ((double)p0[c] + (double)p0[q]);
        } else {
            v += co(R.mur_g1) * ((double)p0[c] + (double)p0[q]);
            const double a1 = ((double)p0[c - s1] + (double)p0[q - s1]) + ((double)p0[c + s1] + (double)p0[q + s1]);
            const double a2 = ((double)p0[c - s2] + (double)p0[q - s2]) + ((double)p0[c + s2] + (double)p0[q + s2]);
            v = v + co(R.mur_ga) * a1 + co(R.mur_gb) * a2;
        }
        pp[c] = (T)v;
    }
};


// ---------------------------------------------------------------------------
// K3: E and B at vertices
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline void vertex_eb(const RunDev &R, int64_t s, int i, int j, int k, double E[3], double B[3])
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
    // curl of A at n and at n+1, averaged
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

// Is node (i, j, k) a corner of an active cell whose sort tile holds a
// particle at step s?  The push of step s-1 (or the load) marks the tiles of
// the cells its particles end in with s; a node's cells are i-1..i on each
// axis, within the active range 1..n-3.
__device__ inline bool node_needed(const RunDev &R, int64_t s, int i, int j, int k)
{
    const uint32_t want = (uint32_t)s;
    const int c0[3] = {max(i - 1, 1), max(j - 1, 1), max(k - 1, 1)};
    const int c1[3] = {min(i, R.nx - 3), min(j, R.ny - 3), min(k, R.nz - 3)};
    const int tx0 = (int)fdiv((uint32_t)c0[0], R.tdiv[0]), tx1 = (int)fdiv((uint32_t)c1[0], R.tdiv[0]);
    const int ty0 = (int)fdiv((uint32_t)c0[1], R.tdiv[1]), ty1 = (int)fdiv((uint32_t)c1[1], R.tdiv[1]);
    const int tz0 = (int)fdiv((uint32_t)c0[2], R.tdiv[2]), tz1 = (int)fdiv((uint32_t)c1[2], R.tdiv[2]);
    for (int tz = tz0; tz <= tz1; ++tz)
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx)
                if (R.tile_flag[((int64_t)tz * R.ntile[1] + ty) * R.ntile[0] + tx] == want)
                    return true;
    return false;
}

// E, B over the active-particle box of the last sort (full == 0) or over
// all interior nodes (full == 1).  step_bias selects the step whose levels
// are used (0 during a step, -1 after it for read-back).
template <typename T>
struct VertexFields {
    static constexpr int kThreads = 256;
    static __device__ void run(const RunDev &R, Blk blk, int step_bias, int full)
    {
        const int64_t s = R.ctl->step + step_bias;
        int lo[3], hi[3];
        const int n[3] = {R.nx, R.ny, R.nz};
        for (int a = 0; a < 3; ++a) {
            if (full) {
                lo[a] = 1;
                hi[a] = n[a] - 2;
            } else {
                lo[a] = max(1, R.ctl->cell_lo[a]);
                hi[a] = min(n[a] - 2, R.ctl->cell_hi[a] + 1);
            }
            if (hi[a] < lo[a])
                return;
        }
        constexpr int V = 16 / sizeof(T);
        const int64_t ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
        const int64_t tot = ex * ey * ez;
        // 32-bit decoding by multiply-high when exact (t * max(ex, ey) < 2^32)
        const bool fast = (uint64_t)tot * (uint64_t)(ex > ey ? ex : ey) < (1ull << 32);
        const FastDiv fx = fast_div((uint32_t)ex), fy = fast_div((uint32_t)ey);
        for (int64_t t = (int64_t)blk.id * blockDim.x + threadIdx.x; t < tot; t += (int64_t)blk.n * blockDim.x) {
            int i, j, k;
            if (fast) {
                const uint32_t t32 = (uint32_t)t, row = fdiv(t32, fx);
                const uint32_t kk = fdiv(row, fy);
                i = lo[0] + (int)(t32 - row * (uint32_t)ex);
                j = lo[1] + (int)(row - kk * (uint32_t)ey);
                k = lo[2] + (int)kk;
            } else {
                i = lo[0] + (int)(t % ex);
                j = lo[1] + (int)((t / ex) % ey);
                k = lo[2] + (int)(t / (ex * ey));
            }
            if (!full && !node_needed(R, s, i, j, k))
                continue;  // no particle of this step gathers at this node
            double E[3], B[3];
            vertex_eb<T>(R, s, i, j, k, E, B);
            Vec<T, V> w[8 / V];
            const T all[8] = {(T)E[0], (T)E[1], (T)E[2], (T)B[0], (T)B[1], (T)B[2], (T)0, (T)0};
            for (int q = 0; q < 8; ++q)
                w[q / V].v[q % V] = all[q];
            T *dst = eb_node<T>(R, nid(R, i, j, k));
            for (int q = 0; q < 8 / V; ++q)
                vstore<T, V>(dst + q * V, w[q]);
        }
    }
};

// Radiated power through node plane k_plane of the fields at t_{s+1/2}
// (lab-frame Poynting flux).  kPowerBlocks blocks write partial sums over
// a fixed node partition; one block adds them in fixed order, so the
// result does not depend on scheduling.  (A single launch whose last block
// adds the partial sums needs a device-scope release fence in every block,
// which writes back the XCD's L2: in a grouped launch of 32 runs that made
// the stage six times slower.)
template <typename T>
struct PlanePower {
    static constexpr int kThreads = 256;
    static __device__ void run(const RunDev &R, Blk blk, int step_bias, int kp_arg)
    {
        __shared__ double red[256];
        const int kp = kp_arg < 0 ? R.k_plane : kp_arg;  // < 0: the run's diagnostic plane
        const int64_t s = R.ctl->step + step_bias;
        const double g0 = R.gamma0, b0 = R.beta0;
        double acc = 0.0;
        const int wx = R.nx - 2, wy = R.ny - 2;
        for (int t = blk.id * 256 + threadIdx.x; t < wx * wy; t += kPowerBlocks * 256) {
            const int i = 1 + t % wx, j = 1 + t / wx;
            double E[3], B[3];
            vertex_eb<T>(R, s, i, j, kp, E, B);
            const double Exl = g0 * (E[0] + b0 * kC * B[1]);
            const double Eyl = g0 * (E[1] - b0 * kC * B[0]);
            const double Bxl = g0 * (B[0] - b0 * E[1] / kC);
            const double Byl = g0 * (B[1] + b0 * E[0] / kC);
            acc += Exl * Byl - Eyl * Bxl;
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            R.ppart[blk.id] = red[0];
    }
};

struct PlanePowerFinal {
    static constexpr int kThreads = 64;
    static __device__ void run(const RunDev &R, Blk blk, int step_bias, double *out, int end_step)
    {
        plane_power_final(R, R.ctl->step + step_bias, out, end_step);
    }
};

// Workgroups of the vertex-field launch (the same count on host and device).
__host__ __device__ inline int64_t vertex_blocks_of(const RunDev &R)
{
    const int64_t inner = (int64_t)(R.nx - 2) * (R.ny - 2) * (R.nz - 2);
    const int64_t b = (inner + 255) / 256;
    return b < 1 ? 1 : (b > 8192 ? 8192 : b);
}

// The step's vertex fields and the plane-power partial sums in one launch:
// both read only the potentials of step s, which the push and the sort do
// not change, so the partial sums equal those of a launch after the sort.
// The power's workgroups come first, so that they do not form the launch's
// tail.  Single-run steps only: in a grouped launch the merged body needs
// 12-15 more VGPRs than the vertex fields alone, one wave per SIMD fewer.
template <typename T>
struct VertexPower {
    static constexpr int kThreads = 256;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        if (blk.id < kPowerBlocks)
            PlanePower<T>::run(R, Blk{blk.id, kPowerBlocks}, 0, -1);
        else
            VertexFields<T>::run(R, Blk{blk.id - kPowerBlocks, vertex_blocks_of(R)}, 0, 0);
    }
};

// ---------------------------------------------------------------------------
// Spectral radiated power: running Fourier transforms over the boosted time
// t_{s+1/2} of the lab-frame E'_x E'_y B'_x B'_y at every interior node of
// the power plane, at omega_f = nu_f omega_r.  One thread per plane node
// owns its accumulators (no atomics); the fields are those of the plane
// power, from the potentials of step s.
// ---------------------------------------------------------------------------

__host__ __device__ inline double spec_nu(const RunDev &R, int f)
{
    return R.nfreq == 1 ? R.nu_min : R.nu_min + (R.nu_max - R.nu_min) * f / (double)(R.nfreq - 1);
}

template <typename T>
struct PlaneSpectrum {
    static constexpr int kThreads = 256;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        const int64_t s = R.ctl->step;
        const int wx = R.nx - 2, wy = R.ny - 2;
        const int t = (int)(blk.id * kThreads + threadIdx.x);
        if (t >= wx * wy)
            return;
        const int i = 1 + t % wx, j = 1 + t / wx;
        double E[3], B[3];
        vertex_eb<T>(R, s, i, j, R.k_plane, E, B);
        const double g0 = R.gamma0, b0 = R.beta0;
        double F[4];
        F[0] = g0 * (E[0] + b0 * kC * B[1]);
        F[1] = g0 * (E[1] - b0 * kC * B[0]);
        F[2] = g0 * (B[0] - b0 * E[1] / kC);
        F[3] = g0 * (B[1] + b0 * E[0] / kC);
        const double tt = ((double)s + 0.5) * R.dt;
        const int64_t plane = (int64_t)R.nx * R.ny, pidx = (int64_t)j * R.nx + i;
        for (int f = 0; f < R.nfreq; ++f) {
            const double om = spec_nu(R, f) * R.omega_r;
            const double c = cos(om * tt) * R.dt, sn = -sin(om * tt) * R.dt;
            double *acc = R.spec + (int64_t)f * 8 * plane + pidx;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc[(2 * q) * plane] += F[q] * c;
                acc[(2 * q + 1) * plane] += F[q] * sn;
            }
        }
    }
};

// dW/domega of frequency f = blockIdx.x: (1/pi) (dx dy / mu0) sum over the
// plane's interior nodes of Re(Ex' By'* - Ey' Bx'*), fixed-order tree sum
__global__ __launch_bounds__(256) void k_spec_reduce(RunDev R, double *out)
{
    __shared__ double red[256];
    const int f = blockIdx.x;
    const int wx = R.nx - 2, wy = R.ny - 2;
    const int64_t plane = (int64_t)R.nx * R.ny;
    const double *acc = R.spec + (int64_t)f * 8 * plane;
    double sum = 0.0;
    for (int t = threadIdx.x; t < wx * wy; t += 256) {
        const int64_t p = (int64_t)(1 + t / wx) * R.nx + 1 + t % wx;
        sum += (acc[0 * plane + p] * acc[6 * plane + p] + acc[1 * plane + p] * acc[7 * plane + p]) -
               (acc[2 * plane + p] * acc[4 * plane + p] + acc[3 * plane + p] * acc[5 * plane + p]);
    }
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu0 = 1.0 / (kEps0 * kC * kC);
        out[f] = red[0] * R.dx * R.dy / (mu0 * kPi);
    }
}

// ---------------------------------------------------------------------------
// TF/SF seed injection on the planes k = 1 (scattered-field boundary) and
// k = 2 (total-field boundary): after the update of A_x and A_y, each node
// gets back the incident-wave part of the terms through which it used the
// other region's values, so that the total-field region holds +f.
// Incident wave (boosted, along +z): A = A0 p s(t - (z - z_2)/c), the lab
// signal Doppler-scaled by gamma0 (1 + beta0); Gaussian seeds add the
// paraxial amplitude, curvature and Gouy phase.
// ---------------------------------------------------------------------------

__device__ inline double seed_signal(int type, double tau, double f, double tp, double t0, double ph)
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

__device__ inline double seed_incident(const RunDev &R, int comp, int i, int j, int k, double t)
{
    const double x = R.x0 + i * R.dx, y = R.y0 + j * R.dy, z = R.z0 + k * R.dz;
    const double pc = comp == 0 ? cos(R.seed_pol) : sin(R.seed_pol);
    const double D = R.gamma0 * (1.0 + R.beta0);
    const double lam = R.seed_lambda * D;
    const double f = kC / lam, tp = R.seed_ctau / kC * D, t0 = R.seed_ct0 / kC * D;
    const double A0 = R.seed_a0 * kMe * kC / kQe;
    const double z2 = R.z0 + 2.0 * R.dz;
    const double tau = t - (z - z2) / kC;
    double amp = 1.0, ph = R.seed_cep;
    if (R.seed_type == 1) {
        const double zR = kPi * R.seed_w0 * R.seed_w0 / lam;
        const double l = z - R.seed_zf;
        const double w = R.seed_w0 * sqrt(1.0 + (l / zR) * (l / zR));
        const double r2 = x * x + y * y;
        amp = (R.seed_w0 / w) * exp(-r2 / (w * w));
        ph += -0.5 * (2.0 * kPi / lam) * r2 * l / (l * l + zR * zR) + atan(l / zR);
    }
    return pc * A0 * amp * seed_signal(R.seed_signal, tau, f, tp, t0, ph);
}

template <typename T>
struct SeedInject {
    static constexpr int kThreads = 256;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        const int64_t s = R.ctl->step;
        const int wx = R.nx - 2, wy = R.ny - 2;
        const int64_t t = blk.id * kThreads + threadIdx.x;
        if (t >= 2 * (int64_t)wx * wy)
            return;
        const int comp = (int)(t / ((int64_t)wx * wy));
        const int r = (int)(t % ((int64_t)wx * wy));
        const int i = 1 + r % wx, j = 1 + r / wx;
        const double tt = (double)s * R.dt;  // time level n of the update
        const double A = R.A;
        auto F = [&](int ii, int jj, int kk) { return seed_incident(R, comp, ii, jj, kk, tt); };
        const double c1 = A * (R.a2 * F(i + 1, j, 2) + R.a2 * F(i - 1, j, 2) + R.a4 * F(i, j + 1, 2) +
                               R.a4 * F(i, j - 1, 2)) + R.a6 * F(i, j, 2);
        const double c2 = A * (R.a2 * F(i + 1, j, 1) + R.a2 * F(i - 1, j, 1) + R.a4 * F(i, j + 1, 1) +
                               R.a4 * F(i, j - 1, 1)) + R.a6 * F(i, j, 1);
        T *pn = pot_ptr<T>(R, slot_next(s), comp);
        const int64_t n1 = nid(R, i, j, 1), n2 = nid(R, i, j, 2);
        pn[n1] = (T)((double)pn[n1] - c1);
        pn[n2] = (T)((double)pn[n2] + c2);
    }
};

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

struct SweepShape {
    int tx, ty, tz;
};

template <typename T, int TX, int TY, int TZ>
static hipError_t launch_sweep_t(const RunDev &R, hipStream_t st)
{
    const int64_t ntx = (R.nx + TX - 1) / TX, nty = (R.ny + TY - 1) / TY;
    const int64_t nch = (R.nz - 2 + TZ - 1) / TZ;
    const int64_t nb = ntx * nty * nch * 4;
    hipLaunchKernelGGL((k_run<Sweep<T, TX, TY, TZ>>), dim3((unsigned)nb), dim3(TX * TY), 0, st, R);
    return hipGetLastError();
}

template <typename T, int V, int TXV, int TY, int TZ>
static hipError_t launch_sweep_vec_t(const RunDev &R, hipStream_t st)
{
    constexpr int TW = TXV * V;
    const int64_t ntx = (R.nx + TW - 1) / TW, nty = (R.ny + TY - 1) / TY;
    const int64_t nch = (R.nz - 2 + TZ - 1) / TZ;
    const int64_t nb = ntx * nty * nch * 4;
    if constexpr (sizeof(T) == 4) {
        if (R.compensated) {
            hipLaunchKernelGGL((k_run<SweepVec<T, V, TXV, TY, TZ, true>>), dim3((unsigned)nb), dim3(TXV * TY), 0, st, R);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_run<SweepVec<T, V, TXV, TY, TZ, false>>), dim3((unsigned)nb), dim3(TXV * TY), 0, st, R);
    return hipGetLastError();
}

int sweep_fuses_xfaces(const RunDev &R, int shape)
{
    const int V = R.precision == 32 ? 4 : 2;
    return (shape >= 8 && R.nx % V == 0) ? 1 : 0;
}

template <typename T>
static hipError_t launch_sweep_shape(const RunDev &R, int shape, hipStream_t st)
{
    constexpr int V = 16 / sizeof(T);
    if (shape >= 8 && R.nx % V != 0)
        shape = 0;  // vector tiles need aligned rows
    switch (shape) {
    case 8: return launch_sweep_vec_t<T, V, 128 / V, 512 * V / 128, 32>(R, st);
    case 9: return launch_sweep_vec_t<T, V, 128 / V, 256 * V / 128, 32>(R, st);
    case 10: return launch_sweep_vec_t<T, V, 64 / V, 512 * V / 64, 32>(R, st);
    case 11: return launch_sweep_vec_t<T, V, 128 / V, 512 * V / 128, 16>(R, st);
    case 12: return launch_sweep_vec_t<T, V, 128 / V, 512 * V / 128, 64>(R, st);
    case 13: return launch_sweep_vec_t<T, V, 32 / V, 256 * V / 32, 32>(R, st);
    case 14: return launch_sweep_vec_t<T, V, 128 / V, 256 * V / 128, 16>(R, st);
    case 15: return launch_sweep_vec_t<T, V, 128 / V, 512 * V / 128, 4>(R, st);
    case 16: return launch_sweep_vec_t<T, V, 128 / V, 1024 * V / 128, 16>(R, st);
    case 17: return launch_sweep_vec_t<T, V, 64 / V, 512 * V / 64, 16>(R, st);
    case 0: return launch_sweep_t<T, 64, 8, 32>(R, st);
    case 1: return launch_sweep_t<T, 64, 4, 32>(R, st);
    case 2: return launch_sweep_t<T, 32, 8, 32>(R, st);
    case 3: return launch_sweep_t<T, 64, 8, 64>(R, st);
    case 4: return launch_sweep_t<T, 128, 4, 32>(R, st);
    case 5: return launch_sweep_t<T, 64, 16, 32>(R, st);
    case 6: return launch_sweep_t<T, 32, 4, 16>(R, st);
    case 7: return launch_sweep_t<T, 64, 8, 16>(R, st);
    default: return hipErrorInvalidValue;
    }
}

int sweep_shape_count() { return 18; }

// Tile of each shape in nodes (x, y, z) for FP32; shapes 8..13 are the
// vector kernels (4 FP32 or 2 FP64 nodes per thread; y rows halve in FP64).
void sweep_shape_dims(int shape, int *tx, int *ty, int *tz)
{
    static const int d[18][3] = {{64, 8, 32},  {64, 4, 32},  {32, 8, 32},  {64, 8, 64},  {128, 4, 32},
                                 {64, 16, 32}, {32, 4, 16},  {64, 8, 16},  {128, 16, 32}, {128, 8, 32},
                                 {64, 32, 32}, {128, 16, 16}, {128, 16, 64}, {32, 32, 32}, {128, 8, 16},
                                 {128, 16, 4}, {128, 32, 16}, {64, 32, 16}};
    *tx = d[shape][0];
    *ty = d[shape][1];
    *tz = d[shape][2];
}

// boundary nodes the Mur kernel updates (see Mur)
// face nodes of the boundary (per component), and edge and corner nodes
static int64_t mur_nodes(const RunDev &R)
{
    const int64_t nx = R.nx, ny = R.ny, nz = R.nz;
    return 2 * (nx - 2) * (ny - 2) + 2 * (nx - 2) * (nz - 2) + (R.xface_fused ? 0 : 2 * (ny - 2) * (nz - 2));
}

hipError_t launch_sweep(const RunDev &R, int shape, hipStream_t st)
{
    return R.precision == 32 ? launch_sweep_shape<float>(R, shape, st) : launch_sweep_shape<double>(R, shape, st);
}

// Mur face workgroups (per component) plus the source-clearing workgroups
int64_t mur_blocks(const RunDev &R)
{
    return ((mur_nodes(R) + 255) / 256) * (R.space_charge ? 4 : 3) + clear_blocks_of(R.ny, R.nz);
}

// Mur edge and corner workgroups (per component)
int64_t mur_edge_blocks(const RunDev &R) { return mur_edge_blocks_of(R); }

// The face workgroups (and the source clearing) only: the step's push
// launch carries the edge workgroups.
hipError_t launch_mur_faces(const RunDev &R, hipStream_t st)
{
    const unsigned blocks = (unsigned)mur_blocks(R);
    if (R.precision == 32)
        hipLaunchKernelGGL((k_run<Mur<float>>), dim3(blocks), dim3(256), 0, st, R);
    else
        hipLaunchKernelGGL((k_run<Mur<double>>), dim3(blocks), dim3(256), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_mur(const RunDev &R, hipStream_t st)
{
    const unsigned blocks = (unsigned)mur_blocks(R), eblocks = (unsigned)mur_edge_blocks(R);
    if (R.precision == 32) {
        hipLaunchKernelGGL((k_run<Mur<float>>), dim3(blocks), dim3(256), 0, st, R);
        hipLaunchKernelGGL((k_run<MurEdge<float>>), dim3(eblocks), dim3(256), 0, st, R);
    } else {
        hipLaunchKernelGGL((k_run<Mur<double>>), dim3(blocks), dim3(256), 0, st, R);
        hipLaunchKernelGGL((k_run<MurEdge<double>>), dim3(eblocks), dim3(256), 0, st, R);
    }
    return hipGetLastError();
}

// workgroups of the vertex fields (a grid-stride loop over the box)
int64_t vertex_blocks(const RunDev &R) { return vertex_blocks_of(R); }

hipError_t launch_vertex_power(const RunDev &R, hipStream_t st)
{
    const int64_t blocks = vertex_blocks_of(R) + kPowerBlocks;
    if (R.precision == 32)
        hipLaunchKernelGGL((k_run<VertexPower<float>>), dim3((unsigned)blocks), dim3(256), 0, st, R);
    else
        hipLaunchKernelGGL((k_run<VertexPower<double>>), dim3((unsigned)blocks), dim3(256), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_vertex_fields(const RunDev &R, int step_bias, int full, hipStream_t st)
{
    const int64_t blocks = vertex_blocks(R);
    if (R.precision == 32)
        hipLaunchKernelGGL((k_run<VertexFields<float>, int, int>), dim3((unsigned)blocks), dim3(256), 0, st, R, step_bias,
                           full);
    else
        hipLaunchKernelGGL((k_run<VertexFields<double>, int, int>), dim3((unsigned)blocks), dim3(256), 0, st, R, step_bias,
                           full);
    return hipGetLastError();
}

hipError_t launch_plane_spectrum(const RunDev &R, hipStream_t st)
{
    if (R.nfreq <= 0)
        return hipSuccess;
    const unsigned nb = (unsigned)(((int64_t)(R.nx - 2) * (R.ny - 2) + 255) / 256);
    if (R.precision == 32)
        hipLaunchKernelGGL((k_run<PlaneSpectrum<float>>), dim3(nb), dim3(256), 0, st, R);
    else
        hipLaunchKernelGGL((k_run<PlaneSpectrum<double>>), dim3(nb), dim3(256), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_spec_reduce(const RunDev &R, double *out, hipStream_t st)
{
    if (R.nfreq <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_spec_reduce, dim3((unsigned)R.nfreq), dim3(256), 0, st, R, out);
    return hipGetLastError();
}

hipError_t launch_seed_inject(const RunDev &R, hipStream_t st)
{
    if (!R.seed_on)
        return hipSuccess;
    const unsigned nb = (unsigned)((2 * (int64_t)(R.nx - 2) * (R.ny - 2) + 255) / 256);
    if (R.precision == 32)
        hipLaunchKernelGGL((k_run<SeedInject<float>>), dim3(nb), dim3(256), 0, st, R);
    else
        hipLaunchKernelGGL((k_run<SeedInject<double>>), dim3(nb), dim3(256), 0, st, R);
    return hipGetLastError();
}

hipError_t launch_plane_power(const RunDev &R, int step_bias, int kp, double *out, hipStream_t st, int end_step)
{
    if (R.precision == 32)
        hipLaunchKernelGGL((k_run<PlanePower<float>, int, int>), dim3(kPowerBlocks), dim3(256), 0, st, R, step_bias, kp);
    else
        hipLaunchKernelGGL((k_run<PlanePower<double>, int, int>), dim3(kPowerBlocks), dim3(256), 0, st, R, step_bias, kp);
    hipLaunchKernelGGL((k_run<PlanePowerFinal, int, double *, int>), dim3(1), dim3(64), 0, st, R, step_bias, out, end_step);
    return hipGetLastError();
}

}  // namespace mithra

// ---------------------------------------------------------------------------
// grouped launches (several runs per launch; see k_group)
// ---------------------------------------------------------------------------
namespace mithra {

int64_t sweep_blocks(const RunDev &R, int shape)
{
    const int V = R.precision == 32 ? 4 : 2;
    if (shape >= 8 && R.nx % V != 0)
        shape = 0;
    int tx, ty, tz;
    sweep_shape_dims(shape, &tx, &ty, &tz);
    if (shape >= 8 && V == 2)
        ty /= 2;  // FP64 vector tiles: same thread count, half the rows
    const int64_t ntx = (R.nx + tx - 1) / tx, nty = (R.ny + ty - 1) / ty;
    const int64_t nch = (R.nz - 2 + tz - 1) / tz;
    return ntx * nty * nch * 4;
}

template <typename T, int TX, int TY, int TZ>
static void grp_sweep_t(const Group &g, int64_t total, hipStream_t st)
{
    hipLaunchKernelGGL((k_group<Sweep<T, TX, TY, TZ>>), dim3((unsigned)total), dim3(TX * TY), 0, st, g);
}

template <typename T, int V, int TXV, int TY, int TZ>
static void grp_sweep_vec_t(const Group &g, int64_t total, bool lo, hipStream_t st)
{
    if constexpr (sizeof(T) == 4) {
        if (lo) {
            hipLaunchKernelGGL((k_group<SweepVec<T, V, TXV, TY, TZ, true>>), dim3((unsigned)total), dim3(TXV * TY), 0,
                               st, g);
            return;
        }
    }
    hipLaunchKernelGGL((k_group<SweepVec<T, V, TXV, TY, TZ, false>>), dim3((unsigned)total), dim3(TXV * TY), 0, st, g);
}

template <typename T>
static hipError_t grp_sweep(const Group &g, int64_t total, int shape, bool lo, hipStream_t st)
{
    constexpr int V = 16 / sizeof(T);
    switch (shape) {
    case 8: grp_sweep_vec_t<T, V, 128 / V, 512 * V / 128, 32>(g, total, lo, st); break;
    case 9: grp_sweep_vec_t<T, V, 128 / V, 256 * V / 128, 32>(g, total, lo, st); break;
    case 10: grp_sweep_vec_t<T, V, 64 / V, 512 * V / 64, 32>(g, total, lo, st); break;
    case 11: grp_sweep_vec_t<T, V, 128 / V, 512 * V / 128, 16>(g, total, lo, st); break;
    case 12: grp_sweep_vec_t<T, V, 128 / V, 512 * V / 128, 64>(g, total, lo, st); break;
    case 13: grp_sweep_vec_t<T, V, 32 / V, 256 * V / 32, 32>(g, total, lo, st); break;
    case 14: grp_sweep_vec_t<T, V, 128 / V, 256 * V / 128, 16>(g, total, lo, st); break;
    case 15: grp_sweep_vec_t<T, V, 128 / V, 512 * V / 128, 4>(g, total, lo, st); break;
    case 16: grp_sweep_vec_t<T, V, 128 / V, 1024 * V / 128, 16>(g, total, lo, st); break;
    case 17: grp_sweep_vec_t<T, V, 64 / V, 512 * V / 64, 16>(g, total, lo, st); break;
    case 0: grp_sweep_t<T, 64, 8, 32>(g, total, st); break;
    case 1: grp_sweep_t<T, 64, 4, 32>(g, total, st); break;
    case 2: grp_sweep_t<T, 32, 8, 32>(g, total, st); break;
    case 3: grp_sweep_t<T, 64, 8, 64>(g, total, st); break;
    case 4: grp_sweep_t<T, 128, 4, 32>(g, total, st); break;
    case 5: grp_sweep_t<T, 64, 16, 32>(g, total, st); break;
    case 6: grp_sweep_t<T, 32, 4, 16>(g, total, st); break;
    case 7: grp_sweep_t<T, 64, 8, 16>(g, total, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// all members share precision, compensation and the (effective) shape
hipError_t launch_sweep_group(const Group &g, int64_t total, int precision, int compensated, int shape,
                              hipStream_t st)
{
    if (total <= 0)
        return hipSuccess;
    return precision == 32 ? grp_sweep<float>(g, total, shape, compensated != 0, st)
                           : grp_sweep<double>(g, total, shape, false, st);
}



// ge: the same members with their edge and corner workgroup counts
hipError_t launch_mur_group(const Group &g, int64_t total, const Group &ge, int64_t total_e, int precision,
                            hipStream_t st)
{
    if (total <= 0)
        return hipSuccess;
    if (precision == 32) {
        hipLaunchKernelGGL((k_group<Mur<float>>), dim3((unsigned)total), dim3(256), 0, st, g);
        hipLaunchKernelGGL((k_group<MurEdge<float>>), dim3((unsigned)total_e), dim3(256), 0, st, ge);
    } else {
        hipLaunchKernelGGL((k_group<Mur<double>>), dim3((unsigned)total), dim3(256), 0, st, g);
        hipLaunchKernelGGL((k_group<MurEdge<double>>), dim3((unsigned)total_e), dim3(256), 0, st, ge);
    }
    return hipGetLastError();
}



hipError_t launch_vertex_group(const Group &g, int64_t total, int precision, hipStream_t st)
{
    if (total <= 0)
        return hipSuccess;
    if (precision == 32)
        hipLaunchKernelGGL((k_group<VertexFields<float>, int, int>), dim3((unsigned)total), dim3(256), 0, st, g, 0, 0);
    else
        hipLaunchKernelGGL((k_group<VertexFields<double>, int, int>), dim3((unsigned)total), dim3(256), 0, st, g, 0, 0);
    return hipGetLastError();
}

int64_t power_blocks() { return kPowerBlocks; }

hipError_t launch_power_group(const Group &g, int64_t total, const Group &gf, int64_t total_f, int precision,
                              hipStream_t st)
{
    if (total <= 0)
        return hipSuccess;
    if (precision == 32)
        hipLaunchKernelGGL((k_group<PlanePower<float>, int, int>), dim3((unsigned)total), dim3(256), 0, st, g, 0, -1);
    else
        hipLaunchKernelGGL((k_group<PlanePower<double>, int, int>), dim3((unsigned)total), dim3(256), 0, st, g, 0, -1);
    hipLaunchKernelGGL((k_group<PlanePowerFinal, int, double *, int>), dim3((unsigned)total_f), dim3(64), 0, st, gf, 0,
                       (double *)nullptr, 0);
    return hipGetLastError();
}

}  // namespace mithra
