// mur_dev.hpp -- Mur absorbing boundary (sec. "Boundary Truncation"): the
// device functions of the edge and corner update, shared by the boundary
// kernels and by the push launch that carries the edge workgroups.  Edges
// and corners impose the summed first-order conditions of their faces.
#pragma once

#include "mithra_dev.hpp"

namespace mithra {

template <typename T>
struct Lv {
    const T *pm;  // n-1
    const T *p0;  // n
    const T *pp;  // n+1 (interior written by the sweep)
};

__device__ inline int bside(const RunDev &R, int a, int v)
{
    const int n = a == 0 ? R.nx : (a == 1 ? R.ny : R.nz);
    return v == 0 ? -1 : (v == n - 1 ? 1 : 0);
}

template <typename T>
__device__ inline double ld(const T *a, const RunDev &R, const int p[3])
{
    return (double)a[nid(R, p[0], p[1], p[2])];
}

// Summed first-order conditions over the 2^m stencil of node p whose
// boundary axes are ax[0..m-1].  Per stencil node X, with sigma_b = +1 on
// the boundary side of axis b and -1 on the inner side, the conditions
// (scaled by 2^m dt) contribute
//   (w1 + w2) X^{n+1} - 2 w2 X^n + (w2 - w1) X^{n-1},
//   w1 = sum_b sigma_b / h_b,  w2 = m / (c dt).
// np1[] holds the n+1 values of the stencil nodes except node 0 (p).
template <typename T>
__device__ double solve_summed(const RunDev &R, const Lv<T> &L, const int p[3], const int *ax,
                               const int *sd, int m, const double *np1)
{
    const double w2 = (double)m / R.cdt;
    double rest = 0.0, cu = 0.0;
    for (int st = 0; st < (1 << m); ++st) {
        int q[3] = {p[0], p[1], p[2]};
        double w1 = 0.0;
        for (int b = 0; b < m; ++b) {
            const bool inner = (st >> b) & 1;
            if (inner)
                q[ax[b]] -= sd[b];
            w1 += (inner ? -1.0 : 1.0) / R.h[ax[b]];
        }
        rest += -2.0 * w2 * ld(L.p0, R, q) + (w2 - w1) * ld(L.pm, R, q);
        if (st == 0)
            cu = w1 + w2;
        else
            rest += (w1 + w2) * np1[st];
    }
    return -rest / cu;
}

// The face and interior nodes of an edge's or a corner's stencil already
// hold their n+1 values when this runs (the sweep and the face kernel come
// first), so they are read; a corner recomputes its three edge neighbours.
template <typename T>
__device__ double edge_np1(const RunDev &R, const Lv<T> &L, const int p[3], const int *ax, const int *sd)
{
    double np1[4];
    for (int st = 1; st < 4; ++st) {
        int q[3] = {p[0], p[1], p[2]};
        for (int b = 0; b < 2; ++b)
            if ((st >> b) & 1)
                q[ax[b]] -= sd[b];
        np1[st] = ld(L.pp, R, q);
    }
    return solve_summed(R, L, p, ax, sd, 2, np1);
}

template <typename T>
__device__ double corner_np1(const RunDev &R, const Lv<T> &L, const int p[3], const int *ax, const int *sd)
{
    double np1[8];
    for (int st = 1; st < 8; ++st) {
        int q[3] = {p[0], p[1], p[2]};
        int eax[3], esd[3], me = 0;
        for (int b = 0; b < 3; ++b) {
            if ((st >> b) & 1)
                q[ax[b]] -= sd[b];
            else {
                eax[me] = ax[b];
                esd[me] = sd[b];
                ++me;
            }
        }
        if (me == 2)
            np1[st] = edge_np1(R, L, q, eax, esd);
        else
            np1[st] = ld(L.pp, R, q);
    }
    return solve_summed(R, L, p, ax, sd, 3, np1);
}

// Edge and corner nodes of the boundary (one thread each, per component):
// the summed first-order conditions of their faces (solve_summed), with the
// face values the face kernel has just written; a corner recomputes its
// three edge neighbours.  Not in the face kernel: this path needs far more
// registers than the face path, and in one kernel it set the face threads'
// occupancy too.  A single run's step carries these workgroups at the end
// of the push launch (PushThenEdges); grouped steps and the sweep-shape
// tuners launch them on their own after the face kernel.
template <typename T>
struct MurEdge {
    static constexpr int kThreads = 256;
    static __device__ void run(const RunDev &R, Blk blk)
    {
        const int nx = R.nx, ny = R.ny, nz = R.nz;
        const int64_t ex = 4LL * nx, ey = 4LL * (ny - 2), ez = 4LL * (nz - 2);
        const int64_t nb = ex + ey + ez;
        const int64_t bpc = (nb + 255) / 256;
        const int comp = (int)(blk.id / bpc);
        if (comp >= (R.space_charge ? 4 : 3))
            return;
        int64_t r = (blk.id - (int64_t)comp * bpc) * blockDim.x + threadIdx.x;
        if (r >= nb)
            return;
        const int64_t s = R.ctl->step;
        const T *pm = pot_ptr<T>(R, slot_prev(s), comp);
        const T *p0 = pot_ptr<T>(R, slot_cur(s), comp);
        T *pp = pot_ptr<T>(R, slot_next(s), comp);
        int p[3];
        if (r < ex) {
            p[0] = (int)(r % nx);
            const int e = (int)(r / nx);
            p[1] = (e & 1) ? ny - 1 : 0;
            p[2] = (e & 2) ? nz - 1 : 0;
        } else if (r < ex + ey) {
            r -= ex;
            p[1] = 1 + (int)(r % (ny - 2));
            const int e = (int)(r / (ny - 2));
            p[0] = (e & 1) ? nx - 1 : 0;
            p[2] = (e & 2) ? nz - 1 : 0;
        } else {
            r -= ex + ey;
            p[2] = 1 + (int)(r % (nz - 2));
            const int e = (int)(r / (nz - 2));
            p[0] = (e & 1) ? nx - 1 : 0;
            p[1] = (e & 2) ? ny - 1 : 0;
        }
        Lv<T> L{pm, p0, pp};
        int axs[3], sd[3], m = 0;
        for (int a = 0; a < 3; ++a) {
            const int v = bside(R, a, p[a]);
            if (v != 0) {
                axs[m] = a;
                sd[m] = v;
                ++m;
            }
        }
        const double v = m == 2 ? edge_np1(R, L, p, axs, sd) : corner_np1(R, L, p, axs, sd);
        pp[nid(R, p[0], p[1], p[2])] = (T)v;
    }
};

// Workgroups of the edge and corner update (per component; the same count
// on host and device).
__host__ __device__ inline int64_t mur_edge_blocks_of(const RunDev &R)
{
    const int64_t nodes = 4LL * R.nx + 4LL * (R.ny - 2) + 4LL * (R.nz - 2);
    return ((nodes + 255) / 256) * (R.space_charge ? 4 : 3);
}

}  // namespace mithra
