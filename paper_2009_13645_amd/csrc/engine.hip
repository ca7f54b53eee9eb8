// engine.hip -- host engine and C ABI (include/mithra.h) of the MI355X
// boosted-frame PIC step.  It validates the run descriptor, derives the
// boost and the NSFD/Mur coefficients, carves the caller's device arena,
// and enqueues the step pipeline on the caller's stream:
//
//   sweep (A, phi; clears the stale source set) -> Mur -> vertex E,B on the
//   active-particle box -> gather/push/deposit -> bin+sort -> radiated
//   power -> bookkeeping (step counter, particle buffer).
//
// Every kernel reads the step number from device memory, so one step is
// captured once into a HIP graph and replayed for the following steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mithra.h"
#include "mithra_dev.hpp"
#include "mur_dev.hpp"

namespace mithra {
hipError_t launch_sweep(const RunDev &R, int shape, hipStream_t st);
int sweep_shape_count();
void sweep_shape_dims(int shape, int *tx, int *ty, int *tz);
hipError_t launch_mur(const RunDev &R, hipStream_t st);
hipError_t launch_mur_faces(const RunDev &R, hipStream_t st);
int sweep_fuses_xfaces(const RunDev &R, int shape);
hipError_t launch_vertex_fields(const RunDev &R, int step_bias, int full, hipStream_t st);
hipError_t launch_plane_power(const RunDev &R, int step_bias, int kp, double *out, hipStream_t st, int end_step = 0);
hipError_t launch_plane_spectrum(const RunDev &R, hipStream_t st);
hipError_t launch_spec_reduce(const RunDev &R, double *out, hipStream_t st);
hipError_t launch_seed_inject(const RunDev &R, hipStream_t st);
hipError_t launch_gen_bunch(const RunDev &R, const GenParams &P, int pass, double *zrange, hipStream_t st);
hipError_t launch_push_deposit(const RunDev &R, hipStream_t st, bool box, bool end_step);
hipError_t launch_load_deposit(const RunDev &R, hipStream_t st);
hipError_t launch_bunching(const RunDev &R, double *part, int blocks, hipStream_t st);
hipError_t launch_sort(const RunDev &R, hipStream_t st, bool keys_ready, int step_tail = 0);
// launch_sort with step_tail runs the box reductions before the sort and
// ends the step after it, in one workgroup, when this holds
bool sort_ends_step(const RunDev &R);
hipError_t launch_box_reduce(const RunDev &R, int64_t nblocks, const int32_t *part, int32_t *lo, int32_t *hi,
                             int32_t *count, hipStream_t st);
int64_t sweep_blocks(const RunDev &R, int shape);
hipError_t launch_sweep_group(const Group &g, int64_t total, int precision, int compensated, int shape,
                              hipStream_t st);
int64_t mur_blocks(const RunDev &R);
int64_t mur_edge_blocks(const RunDev &R);
hipError_t launch_mur_group(const Group &g, int64_t total, const Group &ge, int64_t total_e, int precision,
                            hipStream_t st);
int64_t vertex_blocks(const RunDev &R);
hipError_t launch_vertex_group(const Group &g, int64_t total, int precision, hipStream_t st);
int64_t power_blocks();
hipError_t launch_power_group(const Group &g, int64_t total, const Group &gf, int64_t total_f, int precision,
                              hipStream_t st);
hipError_t launch_vertex_power(const RunDev &R, hipStream_t st);
hipError_t launch_push_group(const Group &g, int64_t total, int precision, int compensated, hipStream_t st);
hipError_t launch_box_group(const Group &g, int64_t total, hipStream_t st);
hipError_t launch_sort_group(const Group &gs, int64_t total_s, const Group &gd, int64_t total_d, const Group &gp,
                             int64_t total_p, int max_passes, hipStream_t st);
int64_t dep_blocks(int64_t np);
int sort_passes(uint32_t key_inactive);
int64_t sort_blocks(int64_t n);

// --- bookkeeping kernels (single thread) -----------------------------------

__device__ inline void book_end(Ctl *ctl, int advance)
{
    ctl->pbuf ^= 1;
    ctl->nsort += 1;
    if (advance)
        ctl->step += 1;
}

struct BookEnd {
    static constexpr int kThreads = 1;
    static __device__ void run(const RunDev &R, Blk) { book_end(R.ctl, 1); }
};

__global__ void k_book_load(Ctl *ctl)
{
    for (int a = 0; a < 3; ++a) {
        ctl->cell_lo[a] = 0x7fffffff;
        ctl->cell_hi[a] = -1;
    }
    ctl->n_active = 0;
}

}  // namespace mithra

using namespace mithra;

static const int64_t kPowerCap = 1 << 16;
static const int kPartials = 8192;  // per-block partial slots (>= persistent blocks + inactive blocks)
static const int kBunchBlocks = 256;

struct Layout {
    size_t ctl, pot, src, src_lo, eb, spec, pr, pid, key_in, slot_in, cell_by_id, sk, sv, hist, boxpart,
        boxslot, ppart, power, scratch, tile_flag, srow, ntiles, total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static Layout make_layout(const mithra_grid_desc *d, int64_t cap)
{
    Layout L{};
    const size_t nn = (size_t)d->nx * d->ny * d->nz;
    const size_t pf = d->field_precision == 32 ? 4 : 8;
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.ctl = take(sizeof(Ctl));
    L.pot = take(12 * nn * pf);
    L.src = take(8 * nn * pf);
    L.src_lo = (d->compensated && d->field_precision == 32) ? take(8 * nn * pf) : (size_t)-1;
    L.eb = take(8 * nn * pf);
    L.spec = take((size_t)(d->n_freq > 0 ? d->n_freq : 0) * 8 * (size_t)d->nx * d->ny * 8);
    L.pr = take(12 * c * 8);
    L.pid = take(2 * c * 4);
    L.key_in = take(c * 4);
    L.slot_in = take(c * 4);
    L.cell_by_id = take(c * 4);
    L.sk = take(2 * c * 4);
    L.sv = take(2 * c * 4);
    L.hist = take((256 * (size_t)sort_blocks((int64_t)c) + 256) * 4);
    const size_t nparts = std::max((size_t)((c + 255) / 256), (size_t)kPartials);
    L.boxpart = take(8 * 4 * nparts);
    L.boxslot = take(16 * 4 * kBoxSlots);
    size_t ntiles = 1;
    for (int a = 0; a < 3; ++a) {
        const size_t cells = (size_t)((a == 0 ? d->nx : (a == 1 ? d->ny : d->nz)) - 1);
        ntiles *= (cells + d->tile[a] - 1) / d->tile[a];
    }
    L.ppart = take(256 * 8);
    L.power = take((size_t)kPowerCap * 8);
    L.scratch = take((size_t)(3 * kBunchBlocks + 8) * 8);
    L.ntiles = ntiles;
    L.tile_flag = take(ntiles * 4);
    L.srow = take(4 * (size_t)d->ny * d->nz * 4);
    L.total = off;
    return L;
}

struct mithra_engine {
    mithra_grid_desc d;
    RunDev R;
    Layout L;
    char *arena = nullptr;
    hipStream_t stream = nullptr;
    int64_t steps = 0;
    bool loaded = false;
    int sweep_shape = 0;
    int32_t *cell_by_id = nullptr;
    // captured steps: one step without and with the sort launches; a run of
    // steps starting at each sort phase (step mod sort_every)
    hipGraphExec_t g1[2] = {nullptr, nullptr};
    std::vector<hipGraphExec_t> gl;
    int use_graph = 1;
    bool batched = false;              // the run belongs to a batch
    hipStream_t ext_stream = nullptr;  // that batch's stream
    std::string err;
};

// the run's own stream and, while it belongs to a batch, the batch's stream
static hipError_t sync_run(mithra_handle h)
{
    if (h->batched) {
        hipError_t e = hipStreamSynchronize(h->ext_stream);
        if (e != hipSuccess)
            return e;
    }
    return hipStreamSynchronize(h->stream);
}

static int fail(mithra_handle h, int code, const char *fmt, ...)
{
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->err = buf;
    }
    return code;
}

#define HIPCHK(h, call)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(h, MITHRA_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

static double gamma0_of(const mithra_grid_desc *d)
{
    return d->und_type == 1 ? d->gamma / std::sqrt(1.0 + d->K * d->K) : d->gamma / std::sqrt(1.0 + 0.5 * d->K * d->K);
}

// field time step: dz / c for NSFD (dispersion-free along z); standard FD
// cannot take it (eq. CFLcondition) and takes 0.99 of its stable step
static double field_dt(const mithra_grid_desc *d)
{
    if (d->solver == 1)
        return 0.99 / (kC * std::sqrt(1.0 / (d->dx * d->dx) + 1.0 / (d->dy * d->dy) + 1.0 / (d->dz * d->dz)));
    return d->dz / kC;
}

static const char *validate(const mithra_grid_desc *d)
{
    if (!d)
        return "null descriptor";
    if (d->nx < 6 || d->ny < 6 || d->nz < 6)
        return "each of nx, ny, nz must be >= 6";
    if ((double)d->nx * d->ny * d->nz > 4.0e9)
        return "grid too large";
    if (d->nx > (1 << 20) || d->ny > (1 << 20) || d->nz > (1 << 20))
        return "each of nx, ny, nz must be <= 2^20";
    if (d->truncation_order != 1 && d->truncation_order != 2)
        return "truncation_order must be 1 or 2";
    if (d->space_charge != 0 && d->space_charge != 1)
        return "space_charge must be 0 or 1";
    if (d->solver != 0 && d->solver != 1)
        return "solver must be 0 (NSFD) or 1 (FD)";
    if (d->n_sub < 1 || d->n_sub > 1024)
        return "n_sub must be in 1..1024";
    if (d->sort_every < 0 || d->sort_every > 1024)
        return "sort_every must be in 0..1024";
    if (d->field_precision != 32 && d->field_precision != 64)
        return "field_precision must be 32 or 64";
    if (d->compensated != 0 && d->compensated != 1)
        return "compensated must be 0 or 1";
    if (d->compensated && d->field_precision != 32)
        return "compensated accumulation applies to field_precision 32 only";
    if (d->und_type < 0 || d->und_type > 3)
        return "und_type must be 0 (planar), 1 (helical), 2 (optical plane wave) or 3 (optical Gaussian beam)";
    if (d->n_freq < 0 || d->n_freq > 64)
        return "n_freq must be in 0..64";
    if (d->n_freq > 0 && !(std::isfinite(d->nu_min) && std::isfinite(d->nu_max)))
        return "non-finite normalised frequency";
    if (d->n_periods < 1)
        return "n_periods must be >= 1";
    if (d->k_plane < 1 || d->k_plane > d->nz - 2)
        return "k_plane must be in 1..nz-2";
    for (int a = 0; a < 3; ++a)
        if (d->tile[a] < 1 || d->tile[a] > 64)
            return "tile dims must be in 1..64";
    if (d->max_particles < 0 || d->max_particles > 0x7fffffffLL)
        return "max_particles out of range";
    const double v[] = {d->dx, d->dy, d->dz, d->x0, d->y0, d->z0, d->gamma, d->K, d->lambda_u, d->pol_angle_deg,
                        d->z_entrance};
    for (double x : v)
        if (!std::isfinite(x))
            return "non-finite descriptor value";
    if (!(d->dx > 0 && d->dy > 0 && d->dz > 0))
        return "mesh spacings must be positive";
    const double q = (d->dz / d->dx) * (d->dz / d->dx) + (d->dz / d->dy) * (d->dz / d->dy);
    if (d->solver == 0 && !(q < 1.0))
        return "NSFD stability needs (dz/dx)^2 + (dz/dy)^2 < 1 (mithra_adapt_mesh adjusts dx, dy)";
    if (!(d->gamma > 1.0 && d->K > 0.0 && d->lambda_u > 0.0))
        return "gamma > 1, K > 0 and lambda_u > 0 are required";
    if (!(gamma0_of(d) > 1.0))
        return "frame Lorentz factor gamma0 must exceed 1";
    if (d->record_power != 0 && d->record_power != 1)
        return "record_power must be 0 or 1";
    // key range: one past the largest tile-major key must fit in 32 bits
    double tiles = 1.0;
    for (int a = 0; a < 3; ++a) {
        const int cells = (a == 0 ? d->nx : (a == 1 ? d->ny : d->nz)) - 1;
        tiles *= (double)((cells + d->tile[a] - 1) / d->tile[a]);
    }
    if (tiles * d->tile[0] * d->tile[1] * d->tile[2] >= 4294967295.0)
        return "tile-major key range exceeds 32 bits";
    return nullptr;
}

extern "C" size_t mithra_footprint_bytes(const mithra_grid_desc *d, int64_t n_particles)
{
    if (validate(d) || n_particles < 0)
        return 0;
    int64_t cap = n_particles > d->max_particles ? n_particles : d->max_particles;
    return make_layout(d, cap).total;
}

extern "C" int mithra_init_grid(const mithra_grid_desc *d, void *dev_arena, size_t arena_bytes, void *hip_stream,
                                mithra_handle *out)
{
    if (!out)
        return MITHRA_EINVAL;
    *out = nullptr;
    static thread_local std::string init_err;
    const char *why = validate(d);
    mithra_handle h = new mithra_engine();
    if (why) {
        fail(h, MITHRA_EINVAL, "%s", why);
        *out = h;  // the handle carries the message; destroy frees it
        return MITHRA_EINVAL;
    }
    h->d = *d;
    h->L = make_layout(d, d->max_particles);
    if (!dev_arena || arena_bytes < h->L.total || ((uintptr_t)dev_arena & 255)) {
        fail(h, MITHRA_ENOMEM, "arena of %zu bytes at %p; need %zu bytes aligned to 256", arena_bytes, dev_arena,
             h->L.total);
        *out = h;
        return MITHRA_ENOMEM;
    }
    h->arena = (char *)dev_arena;
    h->stream = (hipStream_t)hip_stream;
    // from here on a failure returns the handle too, so that its message
    // can be read; the caller destroys it
    *out = h;
    const char *env = getenv("MITHRA_NO_GRAPH");
    h->use_graph = (env && env[0] == '1') ? 0 : 1;

    RunDev &R = h->R;
    memset(&R, 0, sizeof R);
    R.nx = d->nx;
    R.ny = d->ny;
    R.nz = d->nz;
    R.nn = (int64_t)d->nx * d->ny * d->nz;
    R.dx = d->dx;
    R.dy = d->dy;
    R.dz = d->dz;
    R.x0 = d->x0;
    R.y0 = d->y0;
    R.z0 = d->z0;
    R.inv_dx = 1.0 / d->dx;
    R.inv_dy = 1.0 / d->dy;
    R.inv_dz = 1.0 / d->dz;
    // Lorentz boost of mesh and time: dt = dz / c (NSFD) or 0.99 of the
    // stable step of eq. CFLcondition (FD), dt_b = dt / N
    R.solver = d->solver;
    R.dt = field_dt(d);
    R.dtb = R.dt / (double)d->n_sub;
    R.n_sub = d->n_sub;
    R.sort_every = d->sort_every > 1 ? d->sort_every : 1;
    R.gamma0 = gamma0_of(d);
    R.beta0 = std::sqrt(1.0 - 1.0 / (R.gamma0 * R.gamma0));
    R.ku = 2.0 * kPi / d->lambda_u;
    R.B0 = 2.0 * kPi * kMe * kC * d->K / (kQe * d->lambda_u);
    R.Lu = d->n_periods * d->lambda_u;
    R.z_ent = d->z_entrance;
    R.theta = d->pol_angle_deg * kPi / 180.0;
    R.und_type = d->und_type;
    R.Kund = d->K;
    R.lam_u = d->lambda_u;
    R.n_modules = 1;
    R.und_ext = d->und_type >= 2 ? 1 : 0;
    // NSFD: A = 0.25 (1 + 0.02 / ((dz/dx)^2 + (dz/dy)^2)); r_l = c dt / d_l
    const double cdt = kC * R.dt;
    const double rx2 = (cdt / d->dx) * (cdt / d->dx), ry2 = (cdt / d->dy) * (cdt / d->dy),
                 rz2 = (cdt / d->dz) * (cdt / d->dz);
    const double qq = (d->dz / d->dx) * (d->dz / d->dx) + (d->dz / d->dy) * (d->dz / d->dy);
    // standard FD is the same update with no z average (A = 0)
    R.A = d->solver == 0 ? 0.25 * (1.0 + 0.02 / qq) : 0.0;
    R.a1 = 2.0 * (1.0 - (1.0 - 2.0 * R.A) * rx2 - (1.0 - 2.0 * R.A) * ry2 - rz2);
    R.a2 = rx2;
    R.a4 = ry2;
    R.a6 = rz2 - 2.0 * R.A * (rx2 + ry2);
    R.rx2 = rx2;
    R.ry2 = ry2;
    R.rz2 = rz2;
    const double mu0 = 1.0 / (kEps0 * kC * kC);
    R.sfac_A = cdt * cdt * mu0;
    R.sfac_phi = cdt * cdt / kEps0;
    R.space_charge = d->space_charge;
    R.order = d->truncation_order;
    R.cdt = cdt;
    R.h[0] = d->dx;
    R.h[1] = d->dy;
    R.h[2] = d->dz;
    for (int a = 0; a < 3; ++a) {
        const double hn = R.h[a];
        const double r1 = cdt / R.h[(a + 1) % 3], r2 = cdt / R.h[(a + 2) % 3];
        R.mur_be0[a] = (cdt - hn) / (cdt + hn);
        R.mur_be1[a] = 2.0 * hn / (cdt + hn);
        R.mur_g1[a] = hn * (2.0 - r1 * r1 - r2 * r2) / (cdt + hn);
        R.mur_ga[a] = r1 * r1 * hn / (2.0 * (cdt + hn));
        R.mur_gb[a] = r2 * r2 * hn / (2.0 * (cdt + hn));
    }
    R.precision = d->field_precision;
    R.compensated = d->compensated;
    R.np = 0;
    R.np_cap = d->max_particles;
    for (int a = 0; a < 3; ++a) {
        R.tile[a] = d->tile[a];
        R.tdiv[a] = fast_div((uint32_t)d->tile[a]);
        const int cells = (a == 0 ? d->nx : (a == 1 ? d->ny : d->nz)) - 1;
        R.ntile[a] = (cells + d->tile[a] - 1) / d->tile[a];
    }
    {
        // one past the largest active key: the key of the active cell
        // (n-3, n-3, n-3), which lies in the last tile of every axis at the
        // largest local offset (keys grow with each tile and local coordinate);
        // the smallest value keeps the radix sort to the fewest passes
        const int last[3] = {d->nx - 3, d->ny - 3, d->nz - 3};
        uint32_t tl = 0, loc = 0;
        for (int a = 2; a >= 0; --a) {
            tl = tl * (uint32_t)R.ntile[a] + (uint32_t)(last[a] / R.tile[a]);
            loc = loc * (uint32_t)R.tile[a] + (uint32_t)(last[a] % R.tile[a]);
        }
        R.key_inactive = tl * (uint32_t)(R.tile[0] * R.tile[1] * R.tile[2]) + loc + 1;
    }

    char *A = h->arena;
    const Layout &L = h->L;
    const size_t c = (size_t)(d->max_particles > 0 ? d->max_particles : 1);
    R.ctl = (Ctl *)(A + L.ctl);
    R.pot = A + L.pot;
    R.src = A + L.src;
    R.src_lo = L.src_lo == (size_t)-1 ? nullptr : A + L.src_lo;
    R.eb = A + L.eb;
    R.nfreq = d->n_freq;
    R.nu_min = d->nu_min;
    R.nu_max = d->nu_max;
    R.omega_r = 2.0 * kPi * kC * R.gamma0 * R.beta0 / d->lambda_u;
    R.spec = d->n_freq > 0 ? (double *)(A + L.spec) : nullptr;
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 6; ++a)
            R.pr[b][a] = (double *)(A + L.pr) + (size_t)(b * 6 + a) * c;
    R.pid[0] = (int32_t *)(A + L.pid);
    R.pid[1] = R.pid[0] + c;
    R.key_in = (uint32_t *)(A + L.key_in);
    R.slot_in = (int32_t *)(A + L.slot_in);
    h->cell_by_id = (int32_t *)(A + L.cell_by_id);
    R.tile_flag = (uint32_t *)(A + L.tile_flag);
    R.srow_lo = (int32_t *)(A + L.srow);
    R.srow_hi = R.srow_lo + 2 * (size_t)d->ny * d->nz;
    R.sk[0] = (uint32_t *)(A + L.sk);
    R.sk[1] = R.sk[0] + c;
    R.sv[0] = (int32_t *)(A + L.sv);
    R.sv[1] = R.sv[0] + c;
    R.hist = (uint32_t *)(A + L.hist);
    R.boxpart = (int32_t *)(A + L.boxpart);
    R.boxslot = (int32_t *)(A + L.boxslot);
    R.ppart = (double *)(A + L.ppart);
    R.sort_blocks = sort_blocks((int64_t)c);
    R.power_hist = (double *)(A + L.power);
    R.power_cap = kPowerCap;
    R.k_plane = d->k_plane;
    R.record_power = d->record_power;

    // zero fields, sources, vertex fields and the power history; set the boxes empty
    const size_t pf = d->field_precision == 32 ? 4 : 8;
    const size_t nn = (size_t)R.nn;
    HIPCHK(h, hipMemsetAsync(R.pot, 0, 12 * nn * pf, h->stream));
    HIPCHK(h, hipMemsetAsync(R.src, 0, 8 * nn * pf, h->stream));
    if (R.src_lo)
        HIPCHK(h, hipMemsetAsync(R.src_lo, 0, 8 * nn * pf, h->stream));
    HIPCHK(h, hipMemsetAsync(R.eb, 0, 8 * nn * pf, h->stream));
    if (R.spec)
        HIPCHK(h, hipMemsetAsync(R.spec, 0, (size_t)R.nfreq * 8 * (size_t)d->nx * d->ny * 8, h->stream));
    HIPCHK(h, hipMemsetAsync(R.power_hist, 0, (size_t)kPowerCap * 8, h->stream));
    // no tile marked for any step (the load marks those of step 0)
    HIPCHK(h, hipMemsetAsync(R.tile_flag, 0xFF, L.ntiles * 4, h->stream));
    // source row ranges empty: lo = 0x7f7f7f7f, hi = -1
    HIPCHK(h, hipMemsetAsync(R.srow_lo, 0x7F, 2 * (size_t)d->ny * d->nz * 4, h->stream));
    HIPCHK(h, hipMemsetAsync(R.srow_hi, 0xFF, 2 * (size_t)d->ny * d->nz * 4, h->stream));
    Ctl c0;
    memset(&c0, 0, sizeof c0);
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < 3; ++a) {
            c0.dep_lo[s][a] = 0x7fffffff;
            c0.dep_hi[s][a] = -1;
        }
    for (int a = 0; a < 3; ++a) {
        c0.cell_lo[a] = 0x7fffffff;
        c0.cell_hi[a] = -1;
    }
    HIPCHK(h, hipMemcpyAsync(R.ctl, &c0, sizeof c0, hipMemcpyHostToDevice, h->stream));
    std::vector<int32_t> slots(16 * kBoxSlots);  // every push box slot empty
    for (int b = 0; b < kBoxSlots; ++b)
        box_slot_empty(&slots[16 * b]);
    HIPCHK(h, hipMemcpyAsync(R.boxslot, slots.data(), slots.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, sync_run(h));
    // default sweep tile (measured): grids of up to 2^20 nodes take chunks
    // of 4 or 16 planes, so that enough workgroups run (vector tiles when the
    // row length allows 16-byte vectors, else the scalar tiles); larger grids
    // take vector tiles 32 nodes wide for short rows, else 64 nodes wide over
    // 16 planes (the best at 128-node rows)
    const int vec = d->field_precision == 32 ? 4 : 2;
    const bool small = (double)d->nx * d->ny * d->nz <= 1048576.0;
    if (d->nx % vec == 0)
        h->sweep_shape = small ? 15 : (d->nx <= 48 ? 13 : 17);
    else
        h->sweep_shape = small ? 6 : ((d->nx - 2 <= 40) ? 2 : 0);
    const char *sh = getenv("MITHRA_SWEEP_SHAPE");
    if (sh)
        h->sweep_shape = atoi(sh) % sweep_shape_count();
    R.xface_fused = sweep_fuses_xfaces(R, h->sweep_shape);
    *out = h;
    return MITHRA_OK;
}

static int enqueue_sort_with_cells(mithra_handle h);
static int finish_load(mithra_handle h, int64_t n, double q_macro);

extern "C" int mithra_load_bunch(mithra_handle h, int64_t n, const double *xyz, const double *u, double q_macro)
{
    if (!h)
        return MITHRA_EINVAL;
    if (h->steps > 0 || h->loaded)
        return fail(h, MITHRA_ESTATE, "load_bunch is allowed once, before the first step");
    if (n <= 0 || n > h->d.max_particles)
        return fail(h, MITHRA_EINVAL, "n = %lld outside 1..max_particles (%lld)", (long long)n,
                    (long long)h->d.max_particles);
    if (!xyz || !u || !std::isfinite(q_macro))
        return fail(h, MITHRA_EINVAL, "null input or non-finite charge");
    std::vector<double> col((size_t)n);
    for (int64_t p = 0; p < 3 * n; ++p)
        if (!std::isfinite(xyz[p]) || !std::isfinite(u[p]))
            return fail(h, MITHRA_EINVAL, "non-finite particle value at index %lld", (long long)(p / 3));
    RunDev &R = h->R;
    for (int a = 0; a < 3; ++a) {
        for (int64_t p = 0; p < n; ++p)
            col[(size_t)p] = xyz[3 * p + a];
        HIPCHK(h, hipMemcpy(R.pr[0][a], col.data(), (size_t)n * 8, hipMemcpyHostToDevice));
        for (int64_t p = 0; p < n; ++p)
            col[(size_t)p] = u[3 * p + a];
        HIPCHK(h, hipMemcpy(R.pr[0][3 + a], col.data(), (size_t)n * 8, hipMemcpyHostToDevice));
    }
    std::vector<int32_t> ids((size_t)n);
    for (int64_t p = 0; p < n; ++p)
        ids[(size_t)p] = (int32_t)p;
    HIPCHK(h, hipMemcpy(R.pid[0], ids.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    return finish_load(h, n, q_macro);
}

// The particles are in buffer 0 (ids 0..n-1 in slot order): first current
// from the backward drift, charge, sort, boxes.
static int finish_load(mithra_handle h, int64_t n, double q_macro)
{
    RunDev &R = h->R;
    R.np = n;
    R.q = q_macro;
    R.qV = q_macro / (h->d.dx * h->d.dy * h->d.dz);
    for (int a = 0; a < 3; ++a)
        R.qvh_dt[a] = R.qV * R.h[a] / R.dt;
    // sort first so that the first deposit runs in cell order
    hipLaunchKernelGGL(k_book_load, dim3(1), dim3(1), 0, h->stream, R.ctl);
    int rc = enqueue_sort_with_cells(h);
    if (rc)
        return rc;
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, launch_load_deposit(R, h->stream));
    HIPCHK(h, sync_run(h));
    h->loaded = true;
    return MITHRA_OK;
}

// cell index per id, written beside the sort keys (read back on request)
__global__ void k_cells_by_id(RunDev R, int32_t *cell_by_id)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= R.np)
        return;
    const int pb = R.ctl->pbuf;
    const double g[3] = {(R.pr[pb][0][p] - R.x0) / R.dx, (R.pr[pb][1][p] - R.y0) / R.dy,
                         (R.pr[pb][2][p] - R.z0) / R.dz};
    const int n[3] = {R.nx, R.ny, R.nz};
    int c[3];
    bool act = true;
    for (int a = 0; a < 3; ++a) {
        const double f = floor(g[a]);
        act = act && f >= 1.0 && f <= (double)(n[a] - 3);
        c[a] = act ? (int)f : 0;
    }
    cell_by_id[R.pid[pb][p]] = act ? (int32_t)nid(R, c[0], c[1], c[2]) : -1;
}

static int enqueue_sort_with_cells(mithra_handle h)
{
    HIPCHK(h, launch_sort(h->R, h->stream, false));
    return MITHRA_OK;
}

// One step on stream `st`: sweep, Mur, vertex fields (with the power's
// partial sums), push + deposit, bin + sort, step tail.  With `ev` (seven
// events), ev[i] is recorded before stage i and ev[6] after the last one:
// stages 0 sweep, 1 Mur, 2 vertex fields, 3 push + deposit, 4 sort (with
// the box reductions), 5 step tail (power sum, bookkeeping).
static void drop_graphs(mithra_handle h)
{
    for (auto &g : h->g1)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    for (auto &g : h->gl)
        if (g)
            (void)hipGraphExecDestroy(g);
    h->gl.clear();
}

// Step s sorts after its push when (s + 1) is a multiple of sort_every; the
// multi-workgroup sort's launches are left out of the other steps (their
// box reduction sets no passes anyway).  A one-workgroup sort also ends the
// step, so it is always launched.
static bool step_sorts(const mithra_handle h, int64_t s)
{
    return h->R.sort_every <= 1 || (s + 1) % h->R.sort_every == 0 || sort_ends_step(h->R);
}

static int enqueue_step_on(mithra_handle h, hipStream_t st, hipEvent_t *ev, int64_t s)
{
    RunDev &R = h->R;
    auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], st) : hipSuccess; };
    HIPCHK(h, mark(0));
    HIPCHK(h, launch_sweep(R, h->sweep_shape, st));
    if (R.seed_on)  // before Mur: the boundary kernel reads the corrected planes
        HIPCHK(h, launch_seed_inject(R, st));
    HIPCHK(h, mark(1));
    HIPCHK(h, launch_mur_faces(R, st));  // the push launch runs the edge workgroups
    HIPCHK(h, mark(2));
    // no mid-step bookkeeping: the box reductions after the push rewrite the
    // deposit box, the active-cell box and the active count whole
    if (R.record_power)  // the power's partial sums ride on the vertex launch
        HIPCHK(h, launch_vertex_power(R, st));
    else
        HIPCHK(h, launch_vertex_fields(R, 0, 0, st));
    if (R.nfreq > 0)
        HIPCHK(h, launch_plane_spectrum(R, st));
    HIPCHK(h, mark(3));
    // a small run's one-workgroup sort reduces the boxes and ends the step;
    // otherwise the box reduction after the push ends it (the power of the
    // step from the vertex launch's partial sums, then the bookkeeping), and
    // the sort passes, when the step sorts, follow
    const bool small = sort_ends_step(R);
    HIPCHK(h, launch_push_deposit(R, st, !small, !small));
    HIPCHK(h, mark(4));
    if (step_sorts(h, s))
        HIPCHK(h, launch_sort(R, st, true, 1));
    HIPCHK(h, mark(5));
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, mark(6));
    return MITHRA_OK;
}

static int enqueue_step(mithra_handle h, int64_t s) { return enqueue_step_on(h, h->stream, nullptr, s); }

// Capture one step on a private stream (the caller's stream may be the
// legacy default stream, which cannot be captured); the graph is then
// launched on the caller's stream.
// steps per graph of the long replay (fewer graph launches per step)
static const int kGraphSteps = 8;

// the steps s0 .. s0 + nsteps - 1 (only their sort phases matter)
static int build_graph(mithra_handle h, int nsteps, int64_t s0, hipGraphExec_t *out)
{
    hipStream_t cap = nullptr;
    HIPCHK(h, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t user = h->stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    int rc = MITHRA_OK;
    if (e == hipSuccess) {
        h->stream = cap;
        for (int i = 0; i < nsteps && rc == MITHRA_OK; ++i)
            rc = enqueue_step(h, s0 + i);
        h->stream = user;
        e = hipStreamEndCapture(cap, &g);
    }
    (void)hipStreamDestroy(cap);
    if (rc) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return fail(h, MITHRA_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return fail(h, MITHRA_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    return MITHRA_OK;
}

extern "C" int mithra_step(mithra_handle h, int64_t n_steps)
{
    if (!h)
        return MITHRA_EINVAL;
    if (!h->loaded)
        return fail(h, MITHRA_ESTATE, "no bunch loaded");
    if (n_steps < 0)
        return fail(h, MITHRA_EINVAL, "negative step count");
    if (h->batched)
        return fail(h, MITHRA_ESTATE, "the run belongs to a batch: step it with mithra_batch_run");
    int64_t i = 0;
    // replays of a graph of at least kGraphSteps steps, a whole number of
    // sort periods (for periods up to 64 steps), then single steps
    const int64_t se = h->R.sort_every > 1 ? h->R.sort_every : 1;
    const int64_t L = se <= 64 ? se * ((kGraphSteps + se - 1) / se) : 0;
    if (h->use_graph && L > 0 && n_steps >= L) {
        if ((int64_t)h->gl.size() < se)
            h->gl.resize((size_t)se, nullptr);
        for (; i + L <= n_steps; i += L) {
            hipGraphExec_t &g = h->gl[(size_t)(h->steps % se)];
            if (!g) {
                int rc = build_graph(h, (int)L, h->steps, &g);
                if (rc)
                    return rc;
            }
            HIPCHK(h, hipGraphLaunch(g, h->stream));
            h->steps += L;
        }
    }
    for (; i < n_steps; ++i) {
        if (h->use_graph) {
            hipGraphExec_t &g = h->g1[step_sorts(h, h->steps) ? 1 : 0];
            if (!g) {
                int rc = build_graph(h, 1, h->steps, &g);
                if (rc)
                    return rc;
            }
            HIPCHK(h, hipGraphLaunch(g, h->stream));
        } else {
            int rc = enqueue_step(h, h->steps);
            if (rc)
                return rc;
        }
        h->steps += 1;
    }
    return MITHRA_OK;
}

static int check_nan(mithra_handle h)
{
    int32_t flag = 0;
    HIPCHK(h, hipMemcpy(&flag, &h->R.ctl->nan_flag, 4, hipMemcpyDeviceToHost));
    if (flag)
        return fail(h, MITHRA_ENUMERIC, "non-finite value detected by the diagnostics");
    return MITHRA_OK;
}

extern "C" int mithra_read_fields(mithra_handle h, int field_id, int dtype, void *host_out, size_t bytes)
{
    if (!h)
        return MITHRA_EINVAL;
    const size_t nn = (size_t)h->R.nn;
    const size_t esz = dtype == MITHRA_DTYPE_F32 ? 4 : 8;
    if (field_id < 0 || field_id > MITHRA_FIELD_RHO || (dtype != 0 && dtype != 1) || !host_out || bytes != nn * esz)
        return fail(h, MITHRA_EINVAL, "bad field id, dtype, buffer or size");
    HIPCHK(h, sync_run(h));
    int rc = check_nan(h);
    if (rc)
        return rc;
    RunDev &R = h->R;
    const size_t pf = R.precision == 32 ? 4 : 8;
    const int64_t S = h->steps;
    const char *src = nullptr, *lo = nullptr;
    if (field_id <= MITHRA_FIELD_BZ) {
        if (S == 0) {
            memset(host_out, 0, bytes);
            return MITHRA_OK;
        }
        HIPCHK(h, launch_vertex_fields(R, -1, 1, h->stream));
        HIPCHK(h, sync_run(h));
        // node-interleaved: 8 words per node, component field_id
        std::vector<char> all(8 * nn * pf);
        HIPCHK(h, hipMemcpy(all.data(), R.eb, all.size(), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < nn; ++i) {
            const double v = pf == 4 ? (double)((const float *)all.data())[8 * i + field_id]
                                     : ((const double *)all.data())[8 * i + field_id];
            if (esz == 4)
                ((float *)host_out)[i] = (float)v;
            else
                ((double *)host_out)[i] = v;
        }
        return MITHRA_OK;
    } else if (field_id <= MITHRA_FIELD_AZ || field_id == MITHRA_FIELD_PHI) {
        const int comp = field_id == MITHRA_FIELD_PHI ? 3 : field_id - MITHRA_FIELD_AX;
        src = (const char *)R.pot + ((size_t)slot_cur(S) * 4 + comp) * nn * pf;
    } else {
        const int comp = field_id == MITHRA_FIELD_RHO ? 3 : field_id - MITHRA_FIELD_JX;
        const size_t o = ((size_t)(S & 1) * 4 + comp) * nn * pf;
        src = (const char *)R.src + o;
        if (R.src_lo)
            lo = (const char *)R.src_lo + o;
    }
    std::vector<char> raw(nn * pf), rawlo;
    HIPCHK(h, hipMemcpy(raw.data(), src, nn * pf, hipMemcpyDeviceToHost));
    if (lo) {
        rawlo.resize(nn * pf);
        HIPCHK(h, hipMemcpy(rawlo.data(), lo, nn * pf, hipMemcpyDeviceToHost));
    }
    for (size_t i = 0; i < nn; ++i) {
        double v = pf == 4 ? (double)((const float *)raw.data())[i] : ((const double *)raw.data())[i];
        if (lo)
            v += (double)((const float *)rawlo.data())[i];
        if (esz == 4)
            ((float *)host_out)[i] = (float)v;
        else
            ((double *)host_out)[i] = v;
    }
    return MITHRA_OK;
}

extern "C" int mithra_read_particles(mithra_handle h, double *xyz, double *u, int32_t *cell, int32_t *sort_perm)
{
    if (!h)
        return MITHRA_EINVAL;
    if (!h->loaded)
        return fail(h, MITHRA_ESTATE, "no bunch loaded");
    HIPCHK(h, sync_run(h));
    int rc = check_nan(h);
    if (rc)
        return rc;
    RunDev &R = h->R;
    const int64_t n = R.np;
    int32_t pb = 0;
    HIPCHK(h, hipMemcpy(&pb, &R.ctl->pbuf, 4, hipMemcpyDeviceToHost));
    // the state sits in buffer pb in the slots pid[pb]; the order of the
    // last sort is the slot list sv[sorted_buf] (the push does not move the
    // state after sorting)
    std::vector<int32_t> ids((size_t)n);
    HIPCHK(h, hipMemcpy(ids.data(), R.pid[pb], (size_t)n * 4, hipMemcpyDeviceToHost));
    if (sort_perm) {
        int32_t sb = 0;
        HIPCHK(h, hipMemcpy(&sb, &R.ctl->sorted_buf, 4, hipMemcpyDeviceToHost));
        std::vector<int32_t> slots((size_t)n);
        if (sb < 0)  // no sort after the last push: the buffer order
            for (int64_t r = 0; r < n; ++r)
                slots[(size_t)r] = (int32_t)r;
        else
            HIPCHK(h, hipMemcpy(slots.data(), R.sv[sb], (size_t)n * 4, hipMemcpyDeviceToHost));
        for (int64_t r = 0; r < n; ++r)
            sort_perm[r] = ids[(size_t)slots[(size_t)r]];
    }
    std::vector<double> col((size_t)n);
    for (int a = 0; a < 6; ++a) {
        double *dst = a < 3 ? xyz : u;
        if (!dst)
            continue;
        HIPCHK(h, hipMemcpy(col.data(), R.pr[pb][a], (size_t)n * 8, hipMemcpyDeviceToHost));
        for (int64_t r = 0; r < n; ++r)
            dst[3 * (int64_t)ids[(size_t)r] + (a % 3)] = col[(size_t)r];
    }
    if (cell) {
        hipLaunchKernelGGL(k_cells_by_id, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, R,
                           h->cell_by_id);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, sync_run(h));
        HIPCHK(h, hipMemcpy(cell, h->cell_by_id, (size_t)n * 4, hipMemcpyDeviceToHost));
    }
    return MITHRA_OK;
}

extern "C" int mithra_radiated_power(mithra_handle h, int32_t k_plane, double *p_lab_W)
{
    if (!h || !p_lab_W)
        return MITHRA_EINVAL;
    if (k_plane < 1 || k_plane > h->d.nz - 2)
        return fail(h, MITHRA_EINVAL, "k_plane outside 1..nz-2");
    if (!h->loaded)
        return fail(h, MITHRA_ESTATE, "no bunch loaded");
    if (h->steps == 0) {
        *p_lab_W = 0.0;
        return MITHRA_OK;
    }
    double *dev = (double *)(h->arena + h->L.scratch) + 3 * kBunchBlocks;
    HIPCHK(h, launch_plane_power(h->R, -1, k_plane, dev, h->stream));
    HIPCHK(h, sync_run(h));
    HIPCHK(h, hipMemcpy(p_lab_W, dev, 8, hipMemcpyDeviceToHost));
    return MITHRA_OK;
}

extern "C" int64_t mithra_power_history(mithra_handle h, double *out, int64_t n)
{
    if (!h || !out || n < 0)
        return MITHRA_EINVAL;
    HIPCHK(h, sync_run(h));
    int64_t m = h->steps < n ? h->steps : n;
    if (m > kPowerCap)
        m = kPowerCap;
    if (m > 0)
        HIPCHK(h, hipMemcpy(out, h->R.power_hist, (size_t)m * 8, hipMemcpyDeviceToHost));
    return m;
}

extern "C" int mithra_bunching(mithra_handle h, double *b)
{
    if (!h || !b)
        return MITHRA_EINVAL;
    if (!h->loaded)
        return fail(h, MITHRA_ESTATE, "no bunch loaded");
    double *part = (double *)(h->arena + h->L.scratch);
    HIPCHK(h, launch_bunching(h->R, part, kBunchBlocks, h->stream));
    HIPCHK(h, sync_run(h));
    std::vector<double> hp(3 * kBunchBlocks);
    HIPCHK(h, hipMemcpy(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost));
    double re = 0, im = 0, n = 0;
    for (int i = 0; i < kBunchBlocks; ++i) {
        re += hp[3 * i];
        im += hp[3 * i + 1];
        n += hp[3 * i + 2];
    }
    *b = n > 0 ? std::sqrt(re * re + im * im) / n : 0.0;
    return MITHRA_OK;
}

// ---- the allocation-free bunching call -------------------------------------
//
// Its kernel's partial sums (3 doubles for each of the kBunchBlocks blocks,
// whatever the particle count) live in a file-scope device array, one copy
// per device for the life of the process.  Host code never passes the
// array's name to a kernel: the device address of each device's copy is
// taken once (hipGetSymbolAddress, that device current) and kept.
static __device__ __align__(256) double scratch[3 * kBunchBlocks];
static constexpr int kMaxDevices = 64;
static double *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

static int scratch_address(mithra_handle h, double **out)
{
    int dev = -1;
    HIPCHK(h, hipGetDevice(&dev));
    hipPointerAttribute_t attr;
    HIPCHK(h, hipPointerGetAttributes(&attr, h->arena));
    if (attr.device != dev)
        return fail(h, MITHRA_EINVAL, "the run's device (%d) must be the current device (%d)", attr.device, dev);
    if (dev < 0 || dev >= kMaxDevices)
        return fail(h, MITHRA_EINVAL, "device %d beyond the %d devices this call serves", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(h, MITHRA_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return MITHRA_OK;
}

extern "C" int mithra_bunching_noalloc(mithra_handle h, double *b)
{
    if (!h || !b)
        return MITHRA_EINVAL;
    if (!h->loaded)
        return fail(h, MITHRA_ESTATE, "no bunch loaded");
    double *part = nullptr;
    int rc = scratch_address(h, &part);
    if (rc)
        return rc;
    // the partial sums are overwritten whole by the kernel: nothing to clear
    HIPCHK(h, launch_bunching(h->R, part, kBunchBlocks, h->stream));
    HIPCHK(h, sync_run(h));
    double hp[3 * kBunchBlocks];
    HIPCHK(h, hipMemcpy(hp, part, sizeof hp, hipMemcpyDeviceToHost));
    double re = 0, im = 0, n = 0;
    for (int i = 0; i < kBunchBlocks; ++i) {
        re += hp[3 * i];
        im += hp[3 * i + 1];
        n += hp[3 * i + 2];
    }
    *b = n > 0 ? std::sqrt(re * re + im * im) / n : 0.0;
    return MITHRA_OK;
}

extern "C" int64_t mithra_spectral_power(mithra_handle h, double *dW_domega, int64_t n)
{
    if (!h || !dW_domega || n < 0)
        return MITHRA_EINVAL;
    HIPCHK(h, sync_run(h));
    const int64_t m = std::min<int64_t>(n, h->R.nfreq);
    if (m <= 0)
        return 0;
    double *dev = (double *)(h->arena + h->L.scratch);  // nfreq <= 64 results
    HIPCHK(h, launch_spec_reduce(h->R, dev, h->stream));
    HIPCHK(h, sync_run(h));
    HIPCHK(h, hipMemcpy(dW_domega, dev, (size_t)m * 8, hipMemcpyDeviceToHost));
    return m;
}

extern "C" int mithra_set_undulator(mithra_handle h, const mithra_undulator_desc *u)
{
    if (!h || !u)
        return MITHRA_EINVAL;
    if (h->steps > 0)
        return fail(h, MITHRA_ESTATE, "the undulator is fixed once the run has stepped");
    if (h->batched)
        return fail(h, MITHRA_ESTATE, "the run belongs to a batch");
    const double v[] = {u->gap, u->dK, u->ctau, u->ct0, u->cep_deg, u->w0_par, u->w0_perp, u->z_focus};
    for (double x : v)
        if (!std::isfinite(x))
            return fail(h, MITHRA_EINVAL, "non-finite undulator parameter");
    if (u->n_modules < 1 || u->n_modules > 1000)
        return fail(h, MITHRA_EINVAL, "n_modules must be in 1..1000");
    if (u->n_modules > 1 && !(u->gap > 0.0))
        return fail(h, MITHRA_EINVAL, "an undulator array needs gap > 0");
    if (u->signal < 0 || u->signal > 3)
        return fail(h, MITHRA_EINVAL, "signal must be 0..3");
    if (h->d.und_type >= 2 && u->signal != 3 && !(u->ctau > 0.0))
        return fail(h, MITHRA_EINVAL, "an optical pulse needs ctau > 0");
    if (h->d.und_type == 3 && !(u->w0_par > 0.0 && u->w0_perp > 0.0))
        return fail(h, MITHRA_EINVAL, "a Gaussian-beam undulator needs positive waists");
    for (int m = 0; m < u->n_modules; ++m)
        if (!(h->d.K + m * u->dK > 0.0))
            return fail(h, MITHRA_EINVAL, "tapering makes K of module %d non-positive", m);
    RunDev &R = h->R;
    R.n_modules = u->n_modules;
    R.gap = u->gap;
    R.dK = u->dK;
    R.opt_signal = u->signal;
    R.opt_ctau = u->ctau;
    R.opt_ct0 = u->ct0;
    R.opt_cep = u->cep_deg * kPi / 180.0;
    R.opt_w0[0] = u->w0_par;
    R.opt_w0[1] = u->w0_perp;
    R.opt_zf = u->z_focus;
    R.und_ext = (h->d.und_type >= 2 || u->n_modules > 1) ? 1 : 0;
    drop_graphs(h);
    return MITHRA_OK;
}

extern "C" int mithra_set_seed(mithra_handle h, const mithra_seed_desc *sd)
{
    if (!h || !sd)
        return MITHRA_EINVAL;
    if (h->steps > 0)
        return fail(h, MITHRA_ESTATE, "the seed is fixed once the run has stepped");
    if (h->batched)
        return fail(h, MITHRA_ESTATE, "the run belongs to a batch");
    const double v[] = {sd->a0, sd->wavelength, sd->ctau, sd->ct0, sd->cep_deg, sd->pol_deg, sd->w0, sd->z_focus};
    for (double x : v)
        if (!std::isfinite(x))
            return fail(h, MITHRA_EINVAL, "non-finite seed parameter");
    if (sd->type != 0 && sd->type != 1)
        return fail(h, MITHRA_EINVAL, "seed type must be 0 (plane wave) or 1 (Gaussian beam)");
    if (sd->signal < 0 || sd->signal > 3 || !(sd->wavelength > 0.0) || (sd->signal != 3 && !(sd->ctau > 0.0)))
        return fail(h, MITHRA_EINVAL, "seed signal, wavelength or pulse length out of range");
    if (sd->type == 1 && !(sd->w0 > 0.0))
        return fail(h, MITHRA_EINVAL, "a Gaussian seed needs w0 > 0");
    if (h->d.nz < 8)
        return fail(h, MITHRA_EINVAL, "a seeded run needs nz >= 8");
    RunDev &R = h->R;
    R.seed_on = 1;
    R.seed_type = sd->type;
    R.seed_signal = sd->signal;
    R.seed_a0 = sd->a0;
    R.seed_lambda = sd->wavelength;
    R.seed_ctau = sd->ctau;
    R.seed_ct0 = sd->ct0;
    R.seed_cep = sd->cep_deg * kPi / 180.0;
    R.seed_pol = sd->pol_deg * kPi / 180.0;
    R.seed_w0 = sd->w0;
    R.seed_zf = sd->z_focus;
    // the injection corrects planes 1 and 2 after the sweep: the x faces on
    // those planes must then be updated by the boundary kernel, after it
    if (sweep_fuses_xfaces(R, h->sweep_shape)) {
        int sh = 0;
        while (sh < sweep_shape_count() && sweep_fuses_xfaces(R, sh))
            ++sh;
        h->sweep_shape = sh;
    }
    R.xface_fused = sweep_fuses_xfaces(R, h->sweep_shape);
    drop_graphs(h);
    return MITHRA_OK;
}

extern "C" int mithra_adapt_mesh(mithra_grid_desc *d, double bunch_time_step, int32_t *changed)
{
    if (!d || !(d->dx > 0 && d->dy > 0 && d->dz > 0) || !std::isfinite(bunch_time_step))
        return MITHRA_EINVAL;
    int32_t mask = 0;
    if (d->solver == 0) {
        const double q = (d->dz / d->dx) * (d->dz / d->dx) + (d->dz / d->dy) * (d->dz / d->dy);
        if (!(q < 1.0)) {
            // one common factor on dx and dy: q scales by 1/f^2
            const double f = std::sqrt(q / 0.98);
            d->dx *= f;
            d->dy *= f;
            mask |= 1;
        }
    }
    if (bunch_time_step > 0.0) {
        const double dt = field_dt(d);
        int64_t nb = (int64_t)std::llround(dt / bunch_time_step);
        if (nb < 1)
            nb = 1;
        if (nb > 1024)
            nb = 1024;
        if (nb != d->n_sub) {
            d->n_sub = (int32_t)nb;
            mask |= 2;
        }
    }
    if (changed)
        *changed = mask;
    return MITHRA_OK;
}

extern "C" int mithra_generate_bunch(mithra_handle h, const mithra_bunch_desc *b, int64_t n, double q_macro)
{
    if (!h || !b)
        return MITHRA_EINVAL;
    if (h->steps > 0 || h->loaded)
        return fail(h, MITHRA_ESTATE, "the bunch is loaded once, before the first step");
    if (n <= 0 || n > h->d.max_particles)
        return fail(h, MITHRA_EINVAL, "n = %lld outside 1..max_particles (%lld)", (long long)n,
                    (long long)h->d.max_particles);
    const double v[] = {b->center[0], b->center[1], b->center[2], b->size[0], b->size[1], b->size[2],
                        b->gamma, b->sigma_gamma_rel, b->sigma_u_perp, b->bunching, b->bunching_phase,
                        b->n_electrons, q_macro};
    for (double x : v)
        if (!std::isfinite(x))
            return fail(h, MITHRA_EINVAL, "non-finite bunch parameter");
    if ((b->long_profile != 0 && b->long_profile != 1) || (b->trans_profile != 0 && b->trans_profile != 1) ||
        (b->shot_noise != 0 && b->shot_noise != 1) || (b->tapers != 0 && b->tapers != 1))
        return fail(h, MITHRA_EINVAL, "profile and flag fields must be 0 or 1");
    if (!(b->gamma > 1.0) || b->size[2] < 0 || b->size[0] < 0 || b->size[1] < 0 || b->sigma_gamma_rel < 0 ||
        b->sigma_u_perp < 0 || (b->shot_noise && !(b->n_electrons > 0)))
        return fail(h, MITHRA_EINVAL, "bunch sizes, spreads, gamma or electron count out of range");
    RunDev &R = h->R;
    const double g0 = R.gamma0, b0 = R.beta0;
    const double beta = std::sqrt(1.0 - 1.0 / (b->gamma * b->gamma));
    // boosted radiation wavenumber, and the bunching (ponderomotive) one,
    // gamma0 k_u (1 + beta0): microbunches at rest here, half a boosted
    // radiation wavelength apart
    const double kr = 2.0 * kPi * g0 * b0 / h->d.lambda_u;
    const double kb = 2.0 * kPi * g0 * (1.0 + b0) / h->d.lambda_u;
    GenParams P{};
    P.long_profile = b->long_profile;
    P.trans_profile = b->trans_profile;
    P.shot_noise = b->shot_noise;
    P.n = n;
    P.cx = b->center[0];
    P.cy = b->center[1];
    P.cz = b->center[2];
    P.sx = b->size[0];
    P.sy = b->size[1];
    P.L = b->size[2];
    P.gamma = b->gamma;
    P.sig_g = b->sigma_gamma_rel;
    P.sig_u = b->sigma_u_perp;
    P.bf = b->bunching;
    P.bphase = b->bunching_phase;
    P.n_e = b->n_electrons;
    P.lz = 1.0 / (g0 * (1.0 - beta * b0));
    P.k = kb * g0 * g0 * (1.0 - beta * b0) * b0 / beta;
    P.sig_t = (2.0 * kPi / kr) / (g0 * (1.0 + b0));
    P.n_flat = n;
    if (b->long_profile == 0 && b->tapers == 1)
        P.n_flat = (int64_t)std::llround((double)n * P.L / (P.L + std::sqrt(2.0 * kPi) * P.sig_t));
    double *zr = (double *)(h->arena + h->L.scratch);
    HIPCHK(h, launch_gen_bunch(R, P, 0, zr, h->stream));
    if (b->shot_noise) {
        double range[2];
        HIPCHK(h, hipMemcpyAsync(range, zr, 16, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        P.zmin = range[0];
        P.slice = 2.0 * kPi / P.k;
        const double ns = std::floor((range[1] - range[0]) / P.slice) + 1.0;
        const size_t cap = 2 * (size_t)(h->d.max_particles > 0 ? h->d.max_particles : 1);  // sort-key scratch
        if (!(ns >= 1.0) || ns > (double)cap)
            return fail(h, MITHRA_EINVAL, "%.0f shot-noise slices exceed the %zu of the sort scratch", ns, cap);
        P.counts = (int32_t *)R.sk[0];
        HIPCHK(h, hipMemsetAsync(P.counts, 0, (size_t)ns * 4, h->stream));
        HIPCHK(h, launch_gen_bunch(R, P, 1, zr, h->stream));
        HIPCHK(h, launch_gen_bunch(R, P, 2, zr, h->stream));
    }
    return finish_load(h, n, q_macro);
}

extern "C" int mithra_constants(mithra_handle h, double *o)
{
    if (!h || !o)
        return MITHRA_EINVAL;
    o[0] = h->R.gamma0;
    o[1] = h->R.beta0;
    o[2] = h->R.dt;
    o[3] = h->R.dtb;
    o[4] = h->R.A;
    o[5] = h->R.q;
    o[6] = (double)h->steps;
    o[7] = (double)h->R.np;
    return MITHRA_OK;
}

extern "C" const char *mithra_last_error(mithra_handle h)
{
    if (!h)
        return "null handle";
    return h->err.c_str();
}

extern "C" int mithra_destroy(mithra_handle h)
{
    if (!h)
        return MITHRA_EINVAL;
    drop_graphs(h);
    delete h;
    return MITHRA_OK;
}

// ---- internal entry points used by the Python binding for timing/tuning --

extern "C" int mithra_set_sweep_shape(mithra_handle h, int shape)
{
    if (!h || shape < 0 || shape >= sweep_shape_count())
        return MITHRA_EINVAL;
    if (h->batched)
        return fail(h, MITHRA_ESTATE, "the run belongs to a batch: its sweep shape is fixed");
    if (h->R.seed_on && sweep_fuses_xfaces(h->R, shape))
        return fail(h, MITHRA_EINVAL, "a seeded run needs a sweep shape that leaves the x faces to the boundary kernel");
    h->sweep_shape = shape;
    h->R.xface_fused = sweep_fuses_xfaces(h->R, shape);
    drop_graphs(h);
    return MITHRA_OK;
}

extern "C" int mithra_sweep_shape_count(void) { return sweep_shape_count(); }

// Run n steps by direct launches with HIP events between the stages of
// every step (see enqueue_step_on) on the handle's stream, and add the
// summed milliseconds of each stage to stage_ms[0..5] and of the whole
// steps to stage_ms[6].  Same state evolution as mithra_step.
static int step_profile(mithra_handle h, int64_t n, double *stage_ms)
{
    if (!h || !stage_ms || n < 0)
        return MITHRA_EINVAL;
    if (!h->loaded)
        return fail(h, MITHRA_ESTATE, "no bunch loaded");
    if (h->batched)
        return fail(h, MITHRA_ESTATE, "the run belongs to a batch: step it with mithra_batch_run");
    std::vector<hipEvent_t> ev((size_t)(7 * n));
    for (auto &e : ev)
        HIPCHK(h, hipEventCreate(&e));
    int rc = MITHRA_OK;
    for (int64_t i = 0; i < n && rc == MITHRA_OK; ++i) {
        rc = enqueue_step_on(h, h->stream, &ev[(size_t)(7 * i)], h->steps);
        if (rc == MITHRA_OK)
            h->steps += 1;
    }
    if (rc == MITHRA_OK)
        HIPCHK(h, hipStreamSynchronize(h->stream));
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; rc == MITHRA_OK && i < n; ++i) {
        const hipEvent_t *e = &ev[(size_t)(7 * i)];
        for (int st = 0; st < 6; ++st) {
            float ms = 0.f;
            HIPCHK(h, hipEventElapsedTime(&ms, e[st], e[st + 1]));
            acc[st] += ms;
        }
        float tot = 0.f;
        HIPCHK(h, hipEventElapsedTime(&tot, e[0], e[6]));
        acc[6] += tot;
    }
    for (auto &e : ev)
        (void)hipEventDestroy(e);
    if (rc)
        return rc;
    for (int st = 0; st < 7; ++st)
        stage_ms[st] += acc[st];
    return MITHRA_OK;
}

extern "C" int mithra_step_profile(mithra_handle h, int64_t n_steps, double *stage_ms)
{
    return step_profile(h, n_steps, stage_ms);
}

extern "C" int mithra_step_timed(mithra_handle h, int64_t n, double *sweep_ms, double *step_ms)
{
    if (!sweep_ms || !step_ms)
        return MITHRA_EINVAL;
    double st[7] = {0, 0, 0, 0, 0, 0, 0};
    int rc = step_profile(h, n, st);
    if (rc)
        return rc;
    *sweep_ms += st[0];
    *step_ms += st[6];
    return MITHRA_OK;
}

// Time the field sweep alone: `iters` launches for the current step (the
// sweep only rewrites the next time level, so repeating it leaves the run's
// state unchanged).
extern "C" int mithra_time_sweep(mithra_handle h, int shape, int iters, double *ms)
{
    if (!h || !ms || iters < 1 || shape < -1 || shape >= sweep_shape_count())
        return MITHRA_EINVAL;
    if (!h->loaded)
        return fail(h, MITHRA_ESTATE, "no bunch loaded");
    const int sh = shape < 0 ? h->sweep_shape : shape;
    HIPCHK(h, sync_run(h));
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    HIPCHK(h, launch_sweep(h->R, sh, h->stream));  // warm
    HIPCHK(h, hipEventRecord(e0, h->stream));
    for (int i = 0; i < iters; ++i)
        HIPCHK(h, launch_sweep(h->R, sh, h->stream));
    HIPCHK(h, hipEventRecord(e1, h->stream));
    HIPCHK(h, hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(h, hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / iters;
    return MITHRA_OK;
}

// ===========================================================================
// Sweep-shape autotuner
// ===========================================================================

namespace {
struct TuneKey {
    int32_t prec, comp, sc, nx, ny, nz;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(prec, comp, sc, nx, ny, nz) < std::tie(o.prec, o.comp, o.sc, o.nx, o.ny, o.nz);
    }
};
std::map<TuneKey, int> g_tuned;
std::mutex g_tune_mu;
}  // namespace

// Time every distinct effective sweep shape, each together with the Mur
// kernel it implies (the vector shapes update the x faces themselves), and
// keep the fastest.  Results are cached per (precision, compensation, space
// charge, grid) for the process.  Repeating sweep and Mur leaves the run's
// state unchanged.
extern "C" int mithra_autotune_sweep(mithra_handle h, int iters, int *best_shape)
{
    if (!h || iters < 1)
        return MITHRA_EINVAL;
    if (!h->loaded)
        return fail(h, MITHRA_ESTATE, "no bunch loaded");
    if (h->R.seed_on) {  // seeded runs keep their non-fused shape
        if (best_shape)
            *best_shape = h->sweep_shape;
        return MITHRA_OK;
    }
    const TuneKey key{h->d.field_precision, h->d.compensated, h->d.space_charge, h->d.nx, h->d.ny, h->d.nz};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            if (best_shape)
                *best_shape = it->second;
            return mithra_set_sweep_shape(h, it->second);
        }
    }
    HIPCHK(h, sync_run(h));
    const int V = h->R.precision == 32 ? 4 : 2;
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    const int saved_fuse = h->R.xface_fused;
    int best = h->sweep_shape;
    float best_t = 1e30f;
    for (int sh = 0; sh < sweep_shape_count(); ++sh) {
        if (sh >= 8 && h->R.nx % V != 0)
            continue;  // falls back to shape 0, timed already
        RunDev R = h->R;
        R.xface_fused = sweep_fuses_xfaces(R, sh);
        HIPCHK(h, launch_sweep(R, sh, h->stream));
        HIPCHK(h, launch_mur(R, h->stream));
        HIPCHK(h, hipEventRecord(e0, h->stream));
        for (int i = 0; i < iters; ++i) {
            HIPCHK(h, launch_sweep(R, sh, h->stream));
            HIPCHK(h, launch_mur(R, h->stream));
        }
        HIPCHK(h, hipEventRecord(e1, h->stream));
        HIPCHK(h, hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(h, hipEventElapsedTime(&t, e0, e1));
        if (t < best_t) {
            best_t = t;
            best = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->R.xface_fused = saved_fuse;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key] = best;
    }
    if (best_shape)
        *best_shape = best;
    return mithra_set_sweep_shape(h, best);
}

// ===========================================================================
// Batches: several runs stepped together by grouped launches
// ===========================================================================
//
// Every stage of the step is one launch per kernel variant for all member
// runs that use it (precision, compensation, sweep shape); the workgroups
// of a launch are the members' grids laid end to end (k_group).  One
// batched step is captured into a graph.  Each member stops at its own
// target step: its kernels return at once after that, so runs of different
// lengths share the replays.

// Workgroups of a member in a grouped vertex-field launch: an eighth of the
// single run's count.  A member's particle box is a small part of its grid
// (the grid holds the radiation around the bunch), and the workgroups past
// the box find no node to do and return, but in a launch over many members
// they fill the dispatch and the CU slots that the working ones wait for.
// The grid-stride loop still covers a box as large as the grid (eight nodes
// per thread then).
static int64_t vertex_group_blocks(const RunDev &R)
{
    const int64_t b = vertex_blocks(R) / 8;
    return b < 1 ? 1 : b;
}

struct GroupTab {
    Group g{};
    int64_t total = 0;
};

struct mithra_batch_s {
    std::vector<mithra_handle> runs;
    hipStream_t stream = nullptr;
    // the FP64 members' stages run on a second stream (fork and join by
    // events), beside the FP32 members' stages on the batch stream
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0, ws_used = 0;
    struct SweepCls {
        int precision, comp, shape;
        GroupTab t;
    };
    std::vector<SweepCls> sweep;
    GroupTab mur[2], mur_edge[2], vertex[2], power[2], power_final[2], push[3], one, sort_s, sort_d, sort_p;
    int max_passes = 0;
    hipGraphExec_t graph = nullptr;         // one batched step
    hipGraphExec_t graph_nosort = nullptr;  // the same without the sort passes (captured on first use)
    std::vector<int64_t> host_targets;
    std::string err;
};

static int bfail(mithra_batch b, int code, const char *fmt, ...)
{
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return code;
}

#define BHIPCHK(b, call)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return bfail(b, MITHRA_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

static size_t tab_bytes(size_t n)
{
    return align256(n * sizeof(RunDev)) + align256((n + 1) * sizeof(int64_t)) + align256(n * sizeof(int64_t));
}

extern "C" size_t mithra_batch_workspace_bytes(int32_t n_runs)
{
    if (n_runs <= 0)
        return 0;
    const size_t n = (size_t)n_runs;
    // every stage kind holds each member at most once; sweep classes add at
    // most one table per member
    return 11 * tab_bytes(n) + (n + 18) * 3 * 256 + 256;
}

// table of members `mem` (indices into b->runs), nb(member) workgroups each
template <class NB>
static int make_tab(mithra_batch b, const std::vector<int> &mem, NB nb, GroupTab *out)
{
    *out = GroupTab{};
    const size_t n = mem.size();
    if (n == 0)
        return MITHRA_OK;
    std::vector<RunDev> rd(n);
    std::vector<int64_t> boff(n + 1), nblk(n);
    boff[0] = 0;
    for (size_t m = 0; m < n; ++m) {
        rd[m] = b->runs[mem[m]]->R;
        nblk[m] = nb(rd[m]);
        boff[m + 1] = boff[m] + (nblk[m] + 7) / 8 * 8;
    }
    if (boff[n] > 0x7fffffffLL)
        return bfail(b, MITHRA_EINVAL, "grouped launch too large");
    const size_t need = tab_bytes(n);
    if (b->ws_used + need > b->ws_bytes)
        return bfail(b, MITHRA_ENOMEM, "batch workspace too small");
    char *base = b->ws + b->ws_used;
    b->ws_used += need;
    RunDev *d_runs = (RunDev *)base;
    int64_t *d_boff = (int64_t *)(base + align256(n * sizeof(RunDev)));
    int64_t *d_nblk = (int64_t *)((char *)d_boff + align256((n + 1) * sizeof(int64_t)));
    BHIPCHK(b, hipMemcpy(d_runs, rd.data(), n * sizeof(RunDev), hipMemcpyHostToDevice));
    BHIPCHK(b, hipMemcpy(d_boff, boff.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    BHIPCHK(b, hipMemcpy(d_nblk, nblk.data(), n * sizeof(int64_t), hipMemcpyHostToDevice));
    out->g.runs = d_runs;
    out->g.boff = d_boff;
    out->g.nblk = d_nblk;
    out->g.nmem = (int)n;
    out->total = boff[n];
    return MITHRA_OK;
}

static int effective_shape(const mithra_handle h)
{
    const int V = h->R.precision == 32 ? 4 : 2;
    return (h->sweep_shape >= 8 && h->R.nx % V != 0) ? 0 : h->sweep_shape;
}

static int build_tables(mithra_batch b)
{
    const int n = (int)b->runs.size();
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i)
        all[i] = i;
    // sweep classes
    std::map<std::tuple<int, int, int>, std::vector<int>> cls;
    for (int i = 0; i < n; ++i) {
        const mithra_handle h = b->runs[i];
        cls[{h->R.precision, h->R.compensated, effective_shape(h)}].push_back(i);
    }
    for (auto &kv : cls) {
        mithra_batch_s::SweepCls c{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), {}};
        const int shape = c.shape;
        int rc = make_tab(b, kv.second, [shape](const RunDev &R) { return sweep_blocks(R, shape); }, &c.t);
        if (rc)
            return rc;
        b->sweep.push_back(c);
    }
    for (int pi = 0; pi < 2; ++pi) {
        const int prec = pi == 0 ? 32 : 64;
        std::vector<int> mem, memp;
        for (int i = 0; i < n; ++i)
            if (b->runs[i]->R.precision == prec) {
                mem.push_back(i);
                if (b->runs[i]->R.record_power)
                    memp.push_back(i);
            }
        int rc = make_tab(b, mem, [](const RunDev &R) { return mur_blocks(R); }, &b->mur[pi]);
        if (!rc)
            rc = make_tab(b, mem, [](const RunDev &R) { return mur_edge_blocks(R); }, &b->mur_edge[pi]);
        if (!rc)
            rc = make_tab(b, mem, [](const RunDev &R) { return vertex_group_blocks(R); }, &b->vertex[pi]);
        if (!rc)
            rc = make_tab(b, memp, [](const RunDev &) { return power_blocks(); }, &b->power[pi]);
        if (!rc)
            rc = make_tab(b, memp, [](const RunDev &) { return (int64_t)1; }, &b->power_final[pi]);
        if (rc)
            return rc;
    }
    for (int ci = 0; ci < 3; ++ci) {  // FP64, FP32, FP32 compensated
        std::vector<int> mem;
        for (int i = 0; i < n; ++i) {
            const RunDev &R = b->runs[i]->R;
            const int c = R.precision == 64 ? 0 : (R.compensated ? 2 : 1);
            if (c == ci)
                mem.push_back(i);
        }
        int rc = make_tab(b, mem, [](const RunDev &R) { return dep_blocks(R.np); }, &b->push[ci]);
        if (rc)
            return rc;
    }
    int rc = make_tab(b, all, [](const RunDev &) { return (int64_t)1; }, &b->one);
    if (!rc)
        rc = make_tab(b, all, [](const RunDev &R) { return R.sort_blocks; }, &b->sort_s);
    if (!rc)
        rc = make_tab(b, all, [](const RunDev &) { return (int64_t)256; }, &b->sort_d);
    if (!rc)
        rc = make_tab(b, all, [](const RunDev &) { return (int64_t)1; }, &b->sort_p);  // SortRange
    if (rc)
        return rc;
    b->max_passes = 0;
    for (int i = 0; i < n; ++i)
        b->max_passes = std::max(b->max_passes, sort_passes(b->runs[i]->R.key_inactive));
    return MITHRA_OK;
}

// One batched step.  The members of the two precisions share no memory, so
// their stages up to the push form two independent chains: the FP64
// members' on the side stream, the FP32 members' on st; each chain's
// grouped launches then fill the tails of the other's.  The box reductions,
// the sort and the bookkeeping run over all members after the join.
static void batch_free_streams(mithra_batch b)
{
    if (b->side)
        (void)hipStreamDestroy(b->side);
    if (b->fork)
        (void)hipEventDestroy(b->fork);
    if (b->join)
        (void)hipEventDestroy(b->join);
    b->side = nullptr;
    b->fork = b->join = nullptr;
}

static int enqueue_batch_step(mithra_batch b, hipStream_t st, bool sort)
{
    BHIPCHK(b, hipEventRecord(b->fork, st));
    BHIPCHK(b, hipStreamWaitEvent(b->side, b->fork, 0));
    for (int chain = 0; chain < 2; ++chain) {
        hipStream_t cs = chain == 0 ? b->side : st;
        const int prec = chain == 0 ? 64 : 32, pi = chain == 0 ? 1 : 0;
        for (auto &c : b->sweep)
            if (c.precision == prec)
                BHIPCHK(b, launch_sweep_group(c.t.g, c.t.total, c.precision, c.comp, c.shape, cs));
        BHIPCHK(b, launch_mur_group(b->mur[pi].g, b->mur[pi].total, b->mur_edge[pi].g, b->mur_edge[pi].total, prec,
                                    cs));
        BHIPCHK(b, launch_vertex_group(b->vertex[pi].g, b->vertex[pi].total, prec, cs));
        // the plane power reads the potentials of this step only
        BHIPCHK(b, launch_power_group(b->power[pi].g, b->power[pi].total, b->power_final[pi].g,
                                      b->power_final[pi].total, prec, cs));
        for (int ci = 0; ci < 3; ++ci)
            if ((ci == 0) == (chain == 0))
                BHIPCHK(b, launch_push_group(b->push[ci].g, b->push[ci].total, ci == 0 ? 64 : 32, ci == 2, cs));
    }
    BHIPCHK(b, hipEventRecord(b->join, b->side));
    BHIPCHK(b, hipStreamWaitEvent(st, b->join, 0));
    BHIPCHK(b, launch_box_group(b->one.g, b->one.total, st));
    if (sort)
        BHIPCHK(b, launch_sort_group(b->sort_s.g, b->sort_s.total, b->sort_d.g, b->sort_d.total, b->sort_p.g,
                                     b->sort_p.total, b->max_passes, st));
    hipLaunchKernelGGL((k_group<BookEnd>), dim3((unsigned)b->one.total), dim3(1), 0, st, b->one.g);
    BHIPCHK(b, hipGetLastError());
    return MITHRA_OK;
}

static int build_batch_graph(mithra_batch b, bool sort = true)
{
    hipGraphExec_t *out = sort ? &b->graph : &b->graph_nosort;
    hipStream_t cap = nullptr;
    BHIPCHK(b, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    int rc = MITHRA_OK;
    if (e == hipSuccess) {
        rc = enqueue_batch_step(b, cap, sort);
        e = hipStreamEndCapture(cap, &g);
    }
    (void)hipStreamDestroy(cap);
    if (rc) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return bfail(b, MITHRA_EDEVICE, "batch graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return bfail(b, MITHRA_EDEVICE, "batch graph instantiate failed: %s", hipGetErrorString(e));
    return MITHRA_OK;
}

extern "C" int mithra_batch_create(const mithra_handle *runs, int32_t n_runs, void *dev_workspace,
                                   size_t workspace_bytes, void *hip_stream, mithra_batch *out)
{
    if (!out)
        return MITHRA_EINVAL;
    *out = nullptr;
    if (!runs || n_runs <= 0 || !dev_workspace || ((uintptr_t)dev_workspace & 255))
        return MITHRA_EINVAL;
    if (workspace_bytes < mithra_batch_workspace_bytes(n_runs))
        return MITHRA_ENOMEM;
    for (int i = 0; i < n_runs; ++i) {
        if (!runs[i] || !runs[i]->loaded || runs[i]->batched)
            return MITHRA_ESTATE;
        // the grouped stages carry the plain step only
        if (runs[i]->R.seed_on || runs[i]->R.nfreq > 0 || runs[i]->R.und_ext)
            return MITHRA_EINVAL;
        for (int j = 0; j < i; ++j)
            if (runs[j] == runs[i])
                return MITHRA_EINVAL;
    }
    mithra_batch b = new mithra_batch_s;
    b->runs.assign(runs, runs + n_runs);
    b->stream = (hipStream_t)hip_stream;
    if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) {
        batch_free_streams(b);
        delete b;
        return MITHRA_EDEVICE;
    }
    b->ws = (char *)dev_workspace;
    b->ws_bytes = workspace_bytes;
    for (auto h : b->runs) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) {
            batch_free_streams(b);
            delete b;
            return MITHRA_EDEVICE;
        }
    }
    int rc = build_tables(b);
    if (!rc)
        rc = build_batch_graph(b);
    if (rc) {
        if (b->graph)
            (void)hipGraphExecDestroy(b->graph);
        batch_free_streams(b);
        delete b;
        return rc;
    }
    for (auto h : b->runs) {
        h->batched = true;
        h->ext_stream = b->stream;
    }
    *out = b;
    return MITHRA_OK;
}

// Member shape and the x-face flag it implies; the member's own graphs,
// captured with the old shape, are dropped.
static void member_set_shape(mithra_handle h, int shape)
{
    h->sweep_shape = shape;
    h->R.xface_fused = sweep_fuses_xfaces(h->R, shape);
    drop_graphs(h);
}

static int rebuild_tables(mithra_batch b)
{
    b->ws_used = 0;
    b->sweep.clear();
    return build_tables(b);
}

// Per member class (precision, compensation), time every sweep tile shape
// as the class's grouped sweep and Mur launches with the whole batch on the
// device, and keep the fastest.  A small grid timed alone leaves most of the
// GPU idle, so the shape that wins alone is often not the one that wins in a
// full batch.  Sweep and Mur only rewrite the next time level and re-clear
// the next source set, so the runs' state is unchanged.
extern "C" int mithra_batch_autotune_sweep(mithra_batch b, int iters, int32_t *shapes_out)
{
    if (!b || iters < 1)
        return MITHRA_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    const int n = (int)b->runs.size();
    // let every member's kernels run while timing, and none afterwards
    const int64_t open = INT64_MAX;
    for (auto h : b->runs)
        BHIPCHK(b, hipMemcpy(&h->R.ctl->target, &open, sizeof(int64_t), hipMemcpyHostToDevice));
    std::map<std::pair<int, int>, std::vector<int>> cls;
    for (int i = 0; i < n; ++i)
        cls[{b->runs[i]->R.precision, b->runs[i]->R.compensated}].push_back(i);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    int rc = MITHRA_OK;
    for (auto &kv : cls) {
        const int prec = kv.first.first, comp = kv.first.second;
        const int V = prec == 32 ? 4 : 2;
        bool any_vec = false;
        for (int i : kv.second)
            any_vec = any_vec || b->runs[i]->R.nx % V == 0;
        int best = b->runs[kv.second[0]]->sweep_shape;
        float best_t = 1e30f;
        for (int sh = 0; sh < sweep_shape_count() && !rc; ++sh) {
            if (sh >= 8 && !any_vec)
                continue;  // every member would fall back to shape 0
            for (int i : kv.second)
                member_set_shape(b->runs[i], sh);
            rc = rebuild_tables(b);
            if (rc)
                break;
            auto launch = [&]() -> int {
                for (auto &c : b->sweep)
                    if (c.precision == prec && c.comp == comp)
                        BHIPCHK(b, launch_sweep_group(c.t.g, c.t.total, c.precision, c.comp, c.shape, b->stream));
                const int pi = prec == 32 ? 0 : 1;
                BHIPCHK(b, launch_mur_group(b->mur[pi].g, b->mur[pi].total, b->mur_edge[pi].g, b->mur_edge[pi].total,
                                            prec, b->stream));
                return MITHRA_OK;
            };
            rc = launch();  // warm
            BHIPCHK(b, hipEventRecord(e0, b->stream));
            for (int it = 0; it < iters && !rc; ++it)
                rc = launch();
            BHIPCHK(b, hipEventRecord(e1, b->stream));
            BHIPCHK(b, hipEventSynchronize(e1));
            float t = 0.f;
            BHIPCHK(b, hipEventElapsedTime(&t, e0, e1));
            if (!rc && t < best_t) {
                best_t = t;
                best = sh;
            }
        }
        if (rc)
            break;
        for (int i : kv.second)
            member_set_shape(b->runs[i], best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto h : b->runs)
        BHIPCHK(b, hipMemcpy(&h->R.ctl->target, &h->steps, sizeof(int64_t), hipMemcpyHostToDevice));
    if (!rc)
        rc = rebuild_tables(b);
    if (!rc) {
        for (hipGraphExec_t *gx : {&b->graph, &b->graph_nosort})
            if (*gx) {
                (void)hipGraphExecDestroy(*gx);
                *gx = nullptr;
            }
        rc = build_batch_graph(b);
    }
    if (rc)
        return rc;
    if (shapes_out)
        for (int i = 0; i < n; ++i)
            shapes_out[i] = b->runs[i]->sweep_shape;
    return MITHRA_OK;
}

extern "C" int mithra_batch_run(mithra_batch b, const int64_t *n_steps)
{
    if (!b || !n_steps)
        return MITHRA_EINVAL;
    const size_t n = b->runs.size();
    int64_t most = 0;
    for (size_t i = 0; i < n; ++i) {
        if (n_steps[i] < 0)
            return bfail(b, MITHRA_EINVAL, "negative step count for member %zu", i);
        most = std::max(most, n_steps[i]);
    }
    // the previous call's replays read the old targets until they finish
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->host_targets.resize(n);
    for (size_t i = 0; i < n; ++i) {
        mithra_handle h = b->runs[i];
        b->host_targets[i] = h->steps + n_steps[i];
        BHIPCHK(b, hipMemcpy(&h->R.ctl->target, &b->host_targets[i], sizeof(int64_t), hipMemcpyHostToDevice));
    }
    // When every member that steps in this call sorts after the same pushes
    // (one sort interval, one step phase), the steps after which none sorts
    // replay the graph without the sort passes; otherwise every step carries
    // them and a member whose step does not sort skips them on the device.
    int se = 0;
    int64_t phase = -1;
    bool uniform = true;
    for (size_t i = 0; i < n; ++i) {
        if (n_steps[i] == 0)
            continue;
        const int e = b->runs[i]->R.sort_every > 1 ? b->runs[i]->R.sort_every : 1;
        const int64_t p = b->runs[i]->steps % e;
        if (phase < 0) {
            se = e;
            phase = p;
        } else if (e != se || p != phase) {
            uniform = false;
        }
    }
    uniform = uniform && se > 1;
    if (uniform && !b->graph_nosort) {
        const int rc = build_batch_graph(b, false);
        if (rc)
            return rc;
    }
    for (int64_t k = 0; k < most; ++k) {
        const bool sorts = !uniform || (phase + k + 1) % se == 0;
        BHIPCHK(b, hipGraphLaunch(sorts ? b->graph : b->graph_nosort, b->stream));
    }
    for (size_t i = 0; i < n; ++i)
        b->runs[i]->steps += n_steps[i];
    return MITHRA_OK;
}

extern "C" int mithra_batch_sync(mithra_batch b)
{
    if (!b)
        return MITHRA_EINVAL;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    return MITHRA_OK;
}

extern "C" const char *mithra_batch_last_error(mithra_batch b)
{
    return b ? b->err.c_str() : "null batch";
}

extern "C" int mithra_batch_destroy(mithra_batch b)
{
    if (!b)
        return MITHRA_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    for (auto h : b->runs) {
        h->batched = false;
        h->ext_stream = nullptr;
    }
    if (b->graph)
        (void)hipGraphExecDestroy(b->graph);
    if (b->graph_nosort)
        (void)hipGraphExecDestroy(b->graph_nosort);
    batch_free_streams(b);
    delete b;
    return MITHRA_OK;
}
