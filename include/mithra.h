/*
 * mithra.h -- C ABI of the MI355X boosted-frame FEL particle-in-cell step.
 *
 * The operation is the time step of the MITHRA 2.0 manual (arXiv
 * 2009.13645), ch. 3 "Methodology", in the bunch rest frame:
 *   - NSFD finite-difference update of the vector potential A and the
 *     scalar potential phi (sec. "FDTD for Wave Equation", eqs. NSFDtrick,
 *     NSFDCoefficient, updateEquation; sec. "FDTD for Scalar Potential");
 *   - Mur absorbing boundaries of first or second order (sec. "Boundary
 *     Truncation");
 *   - E and B at the vertices and trilinear gather (sec. "Field
 *     Evaluation", eq. fieldInterpolation);
 *   - Boris push in the total field, the static undulator field being
 *     evaluated in the lab frame and Lorentz-boosted (sec. "Update
 *     Algorithm", eq. BorisScheme; sec. "Static Undulator Field", eqs.
 *     undulatorField, fringingField, LorentzTransformR2L,
 *     LorentzTransformElectric, LorentzTransformMagnetic);
 *   - charge-conserving zigzag current deposition and cloud-in-cell charge
 *     (sec. "Current Deposition").
 *
 * Memory: the caller owns all device memory.  `mithra_footprint_bytes`
 * gives the exact arena size; `mithra_init_grid` borrows an arena of at
 * least that size (any device allocation aligned to 256 bytes, e.g. a
 * torch uint8 tensor) for the handle's lifetime, and enqueues all work on
 * the caller's HIP stream.  Host arrays passed in are copied; host arrays
 * passed out are written synchronously.
 *
 * Errors: every call returns MITHRA_OK (0) or a negative code; the
 * handle keeps a message readable with `mithra_last_error`.  One thread
 * per handle; handles are independent.
 *
 * Units: SI.  The mesh is given in the boosted frame: node (i,j,k) sits at
 * (x0 + i dx, y0 + j dy, z0 + k dz); arrays are [nz][ny][nx], x fastest.
 */
#ifndef MITHRA_H_
#define MITHRA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MITHRA_OK 0
#define MITHRA_EINVAL (-1)   /* descriptor or argument out of range */
#define MITHRA_ENOMEM (-2)   /* arena smaller than the footprint */
#define MITHRA_EDEVICE (-3)  /* a HIP call failed */
#define MITHRA_ESTATE (-4)   /* call not allowed in the handle's state */
#define MITHRA_ENUMERIC (-5) /* non-finite value detected in the run */

/* Field ids of the manual's field sampling (sec. "FIELD", field list):
 * Ex Ey Ez Bx By Bz Ax Ay Az Jx Jy Jz F(phi) Q(rho). */
enum mithra_field_id {
    MITHRA_FIELD_EX = 0, MITHRA_FIELD_EY, MITHRA_FIELD_EZ,
    MITHRA_FIELD_BX, MITHRA_FIELD_BY, MITHRA_FIELD_BZ,
    MITHRA_FIELD_AX, MITHRA_FIELD_AY, MITHRA_FIELD_AZ,
    MITHRA_FIELD_JX, MITHRA_FIELD_JY, MITHRA_FIELD_JZ,
    MITHRA_FIELD_PHI, MITHRA_FIELD_RHO
};

enum mithra_dtype { MITHRA_DTYPE_F32 = 0, MITHRA_DTYPE_F64 = 1 };

/* Run descriptor.  Parameter names follow the manual's MESH group (ch. 4
 * "MESH": mesh resolution, mesh-truncation-order, space-charge, solver,
 * bunch-time-step), UNDULATOR group (ch. 4 "UNDULATOR": undulator-parameter,
 * period, length, polarization-angle) and the radiation-power group of
 * FEL-OUTPUT (ch. 4: plane-position, normalized frequencies), with the
 * mesh already in the boosted frame. */
typedef struct mithra_grid_desc {
    int32_t nx, ny, nz;          /* nodes per axis, 6..2^20 each */
    int32_t truncation_order;    /* Mur order: 1 or 2 */
    int32_t space_charge;        /* 1: solve for phi; 0: phi = 0 */
    int32_t solver;              /* 0: NSFD (dt = dz/c); 1: standard FD (dt = 0.99 of the stable step of eq. CFLcondition) */
    int32_t n_sub;               /* bunch sub-steps per field step, dt_b = dt / n_sub, >= 1 */
    int32_t field_precision;     /* 32 or 64: storage of potentials, sources, E, B */
    int32_t compensated;         /* 1 (with 32): two-sum compensated current/charge sums */
    int32_t und_type;            /* 0 planar, 1 helical, 2 optical plane wave, 3 optical Gaussian beam
                                    (optical: strength a0 = K, wavelength 2 lambda_u, see mithra_set_undulator) */
    int32_t n_periods;           /* undulator length in periods, >= 1 */
    int32_t k_plane;             /* node plane of the radiated-power diagnostic, 1..nz-2 */
    int32_t tile[3];             /* sort tile, cells per axis, each 1..64 */
    int32_t record_power;        /* 1: radiated power through k_plane every step */
    int64_t max_particles;       /* capacity reserved in the arena */
    double dx, dy, dz;           /* boosted-frame spacings (m); NSFD needs (dz/dx)^2+(dz/dy)^2 < 1 */
    double x0, y0, z0;           /* position of node (0,0,0) (m) */
    double gamma;                /* beam Lorentz factor in the lab, > 1 */
    double K;                    /* undulator parameter, > 0 */
    double lambda_u;             /* undulator period, lab frame (m) */
    double pol_angle_deg;        /* field direction (sin, cos, 0) of this angle: 0 = along y, > 0 toward +x */
    double z_entrance;           /* boosted-frame z of the undulator entrance at t = 0 (m) */
    int32_t n_freq;              /* spectral power: number of normalised frequencies (0: none, <= 64) */
    int32_t sort_every;          /* sort by cell after every sort_every-th push (0 or 1: every push,
                                    <= 1024); in between the particles keep their order */
    double nu_min, nu_max;       /* normalised frequencies nu_min..nu_max (equally spaced; one: nu_min) */
} mithra_grid_desc;

/* Undulator extensions (ch. 3 "Static Undulator Array Field", "Optical
 * Undulator Field"; ch. 4 UNDULATOR static-undulator-array and
 * optical-undulator).  Static undulators: n_modules modules of n_periods
 * periods separated by `gap` (lab, m), K of module m = K + m dK
 * (tapering-parameter); the fringes inside a gap are damped by the
 * window of eq. fringingFieldGap.  Optical undulators (und_type 2, 3): a
 * wave propagating along -z with strength a0 = K and wavelength
 * 2 lambda_u, magnetic field along the polarisation direction of
 * pol_angle_deg; signal type of eq. signalTypes (0 modulated Neumann,
 * 1 modulated Gaussian, 2 modulated hyperbolic secant, 3 sinusoidal pulse),
 * pulse length c tau, offset c t0 and CEP as in the manual; Gaussian beam:
 * waists along and across the polarisation and the focus (lab z' from the
 * undulator reference). */
typedef struct mithra_undulator_desc {
    int32_t n_modules;           /* >= 1 */
    int32_t signal;              /* 0..3 */
    double gap;                  /* lab gap between modules (m), >= 0; > 0 when n_modules > 1 */
    double dK;                   /* tapering step of K */
    double ctau, ct0, cep_deg;   /* optical pulse length, offset (m, lab) and CEP (deg) */
    double w0_par, w0_perp;      /* Gaussian-beam waists (m) */
    double z_focus;              /* Gaussian-beam focus (lab z' from the undulator reference, m) */
} mithra_undulator_desc;

/* Seed field injected by total-field / scattered-field boundaries on the
 * node planes k = 1 (scattered) and k = 2 (total) next to z_min (ch. 3
 * "Seed Field"; ch. 4 FIELD seed).  Incident transverse vector potential
 * A = A0 p s(t - (z - z_2)/c) propagating along +z, A0 = a0 m c / e,
 * p = (cos psi, sin psi, 0); the lab wavelength, pulse length and offset
 * are Doppler-scaled by gamma0 (1 + beta0) to the boosted frame.  Gaussian
 * beam: amplitude (w0/w(l)) exp(-r^2/w^2), phase -k r^2 / (2 R(l)) +
 * atan(l / z_R), l = z - z_focus (boosted). */
typedef struct mithra_seed_desc {
    int32_t type;                /* 0 plane wave, 1 Gaussian beam */
    int32_t signal;              /* 0..3, as for the optical undulator */
    double a0;                   /* normalised amplitude */
    double wavelength;           /* lab wavelength (m) */
    double ctau, ct0, cep_deg;   /* pulse length, offset (lab, m), CEP (deg) */
    double pol_deg;              /* direction of A from x toward y (deg) */
    double w0;                   /* Gaussian waist (m) */
    double z_focus;              /* Gaussian focus, boosted z (m) */
} mithra_seed_desc;

/* Bunch generated on the device by Halton quasi-random filling (ch. 3
 * "Electron Bunch Generation"; ch. 4 BUNCH bunch-initialization).
 * Element j of sequence i is 1 minus the radical inverse of j in the base
 * of the i-th prime.  Coordinates: x, y from sequences 0, 1 (uniform: eq.
 * uniform1D over full widths; Gaussian: eq. gaussian2D); z from sequence
 * 2 (flat-top, eq. uniform1D) or 2 and 3 (Gaussian, eq. gaussian1D); lab
 * energy gamma (1 + spread g), g from sequences 4, 5; transverse momentum
 * from 6, 7.  Flat-top tapers against coherent scattering emission: a
 * Gaussian of the same density, rms one lab radiation wavelength, split
 * behind the tail and ahead of the head.  Lab lengths along z map to the
 * boosted frame by 1 / (gamma0 (1 - beta beta0)); u_z = gamma0 (u'_z -
 * beta0 gamma').  Bunching factor (eq. bunchingFactor) and shot noise
 * (slices one load wavelength long, b_s = sqrt(-2 ln x_s)/sqrt(N_s), x_s
 * and phase / 2 pi from sequences 8 and 9) displace z by
 * -(2 b / k) sin(k z + phase), k the load wavenumber that the undulator
 * entrance compresses to the bunching wavenumber k_b = gamma0 k_u
 * (1 + beta0) (see mithra_bunching). */
typedef struct mithra_bunch_desc {
    int32_t long_profile;        /* 0 flat-top, 1 Gaussian */
    int32_t trans_profile;       /* 0 uniform, 1 Gaussian */
    int32_t shot_noise;          /* 0 / 1 */
    int32_t tapers;              /* flat-top tapers: 0 / 1 */
    double center[3];            /* bunch centre, boosted frame (m) */
    double size[3];              /* lab: transverse full widths or sigmas; flat-top length or sigma_z (m) */
    double gamma;                /* mean lab Lorentz factor */
    double sigma_gamma_rel;      /* relative energy spread */
    double sigma_u_perp;         /* transverse spread of gamma beta */
    double bunching, bunching_phase; /* b_f and its phase (rad) */
    double n_electrons;          /* electrons represented (shot noise) */
} mithra_bunch_desc;

typedef struct mithra_engine *mithra_handle;

/* Exact device bytes of the run's arena: potentials (3 time levels),
 * sources (2 sets, plus compensation terms), vertex fields, particle
 * state (2 buffers), sort scratch and diagnostics (power history,
 * spectral accumulators).  Returns 0 for an invalid descriptor.  Pure
 * function; no device call. */
size_t mithra_footprint_bytes(const mithra_grid_desc *d, int64_t n_particles);

/* Mesh auto-adjustment of the MESH group (ch. 4 "MESH", the conditions
 * checked before a run): for NSFD, if sqrt((dz/dx)^2 + (dz/dy)^2) >= 1,
 * dx and dy are scaled up by one common factor to the closest values
 * meeting it (the sum of squares becomes 0.98); the field step is then
 * dz/c (NSFD) or the FD step, and n_sub becomes the integer closest to
 * dt / bunch_time_step (at least 1), so that the bunch step divides the
 * field step.  bunch_time_step <= 0 keeps n_sub.  The adapted values are
 * written back to *d; *changed (nullable) receives a bit mask (1: dx, dy;
 * 2: n_sub).  Pure host function.  Errors: EINVAL (null or non-positive
 * spacings). */
int mithra_adapt_mesh(mithra_grid_desc *d, double bunch_time_step, int32_t *changed);

/* Validate `d`, derive the boost (gamma0 from the first undulator as in
 * ch. 3 "Lorentz Transformation"; dt = dz/c for NSFD, eq. CFLcondition for
 * FD; dt_b = dt/n_sub), the update coefficients (eqs. NSFDCoefficient and
 * updateEquation) and the Mur coefficients (sec. "Boundary Truncation"),
 * carve `dev_arena` and zero the fields.  `hip_stream` is a hipStream_t (NULL = default
 * stream).  On success *out is a new handle.  On an error *out is a
 * handle that holds only the message (read it with `mithra_last_error`,
 * then pass it to `mithra_destroy`), or NULL when `out` itself is
 * NULL.  Errors: EINVAL (bad
 * descriptor: sizes, NSFD condition, precision, tiles, key range),
 * ENOMEM (arena_bytes < footprint or misaligned), EDEVICE. */
int mithra_init_grid(const mithra_grid_desc *d, void *dev_arena, size_t arena_bytes,
                     void *hip_stream, mithra_handle *out);

/* Load n macro-electrons (ids 0..n-1 in input order) in the manual's
 * six-column particle format (ch. 4 BUNCH, bunch-initialization type
 * file: x, y, z, gamma beta_x, gamma beta_y, gamma beta_z), here in the
 * boosted frame.  Host arrays n x 3 row-major, copied: xyz = positions at
 * t = dt/2 (m), u = gamma*beta at t = 0.  q_macro = charge per macro-particle (C,
 * negative for electrons).  Deposits the first current from the backward
 * drift r - c dt u/gamma -> r and the charge at r, and sorts.  Errors:
 * EINVAL (n <= 0, n > max_particles, non-finite input), ESTATE (after a
 * step), EDEVICE. */
int mithra_load_bunch(mithra_handle h, int64_t n, const double *xyz, const double *u,
                      double q_macro);

/* Enqueue n_steps PIC steps (ch. 3 "Methodology": field update, Mur
 * boundaries, vertex fields, gather and Boris push in the total field,
 * charge-conserving deposit; plus bin and sort) on the stream and return
 * without waiting.
 * A non-finite value seen by the diagnostics is reported as ENUMERIC by
 * the next read.  Errors: ESTATE (no bunch loaded), EDEVICE. */
int mithra_step(mithra_handle h, int64_t n_steps);

/* Copy one field to host memory after synchronising the stream.  After n
 * completed steps: A and J at t_n, phi and rho at t_{n+1/2}, E and B at
 * t_{n-1/2} (the fields of the last push; evaluated at all nodes whose
 * neighbours are inside the box, zero on the boundary).  J_l(i,j,k) is
 * the edge current between nodes (i,j,k) and (i,j,k)+e_l.  Layout
 * [nz][ny][nx]; dtype converts on request; bytes must equal
 * nx*ny*nz*sizeof(dtype).  Errors: EINVAL, ENUMERIC, EDEVICE. */
int mithra_read_fields(mithra_handle h, int field_id, int dtype, void *host_out, size_t bytes);

/* Copy the particles in id order, in the six-column format of the
 * manual's bunch output (ch. 4 BUNCH), after synchronising the stream:
 * xyz (n x 3, m) at t_{n+1/2}, u (n x 3) at t_n.  Optional (nullable):
 * cell[id] = linear node index of the cell corner (-1 outside the active
 * region 1 <= cell <= n-3 on every axis) and sort_perm[rank] = id of the
 * current sort order (ascending tile-major key, ties in the previous
 * order: a stable sort; before the first sort, by id).  Any pointer
 * may be NULL.  Errors: ESTATE, ENUMERIC, EDEVICE. */
int mithra_read_particles(mithra_handle h, double *xyz, double *u, int32_t *cell,
                          int32_t *sort_perm);

/* Lab-frame radiated power (W) through node plane k_plane at the latest
 * step: the boosted-frame E and B of the last push are transformed to
 * the lab and the Poynting flux is summed over the plane's interior
 * nodes (the manual's radiation-power output; its formula is not
 * printed).  Synchronises.  Errors: EINVAL (plane), ESTATE, EDEVICE. */
int mithra_radiated_power(mithra_handle h, int32_t k_plane, double *p_lab_W);

/* Per-step history of the power through the descriptor's k_plane
 * (record_power = 1): copies min(n, steps done) values, oldest first,
 * and returns the count (or a negative code). */
int64_t mithra_power_history(mithra_handle h, double *out, int64_t n);

/* |<exp(i k_b z)>| over particles in active cells, k_b = 2 pi gamma0
 * (1 + beta0) / lambda_u (ch. 3 "Bunching factor"): the wavenumber of the
 * ponderomotive wave of the forward radiation and the backward undulator,
 * i.e. the lab resonant wavenumber over gamma0 (microbunches are at rest in
 * this frame, half a boosted radiation wavelength apart).  Instantaneous:
 * in a planar undulator the figure-eight motion adds a modulation of order
 * J1(K^2 / (4 + 2 K^2)).  Synchronises. */
int mithra_bunching(mithra_handle h, double *b);

/* mithra_bunching for callers that cannot allocate device memory (code
 * that must not call hipMalloc: graph-capturing or allocation-free serving
 * loops).  Same result as mithra_bunching; its kernel's partial sums (3
 * doubles for each of 256 blocks, whatever the particle count, so no input
 * exceeds them) go to a library-held device array of 6 KiB, one per
 * device, kept until the process ends, instead of the run's arena.  The
 * run's device must be the current device (EINVAL otherwise).  Every call
 * on a device shares that device's array: calls that overlap on one
 * device (other threads or streams) race.  Synchronises.  Errors: EINVAL,
 * ESTATE, EDEVICE. */
int mithra_bunching_noalloc(mithra_handle h, double *b);

/* Spectral radiated energy through the power plane (ch. 4 FEL-OUTPUT,
 * radiation-power at normalized frequencies): running Fourier transforms
 * over boosted time t_{n+1/2} of the lab-frame E'_x E'_y B'_x B'_y at the
 * plane's interior nodes, F(omega) = sum_n F(t_n) exp(-i omega t_n) dt,
 * omega = nu * 2 pi c / lambda*, give dW/domega = (1/pi) (dx dy / mu0)
 * sum Re(E'_x B'_y* - E'_y B'_x*) (J s), whose integral over omega >= 0 is
 * the time integral of the plane power.  Writes min(n, n_freq) values
 * and returns that count (or a negative code).  Synchronises. */
int64_t mithra_spectral_power(mithra_handle h, double *dW_domega, int64_t n);

/* Undulator arrays, tapering and optical-undulator parameters (see
 * mithra_undulator_desc); allowed before the first step.  Errors: EINVAL,
 * ESTATE (after a step). */
int mithra_set_undulator(mithra_handle h, const mithra_undulator_desc *u);

/* TF/SF seed (see mithra_seed_desc); allowed before the first step.  A
 * seeded run updates the x faces in the boundary kernel (after the
 * injection), not inside the sweep.  Errors: EINVAL, ESTATE. */
int mithra_set_seed(mithra_handle h, const mithra_seed_desc *s);

/* Generate n macro-electrons on the device (see mithra_bunch_desc) and
 * load them as mithra_load_bunch would (first current, charge, sort).
 * q_macro as for mithra_load_bunch.  Errors: EINVAL (n outside
 * 1..max_particles, bad description, shot-noise slices beyond the sort
 * scratch), ESTATE (already loaded), EDEVICE. */
int mithra_generate_bunch(mithra_handle h, const mithra_bunch_desc *b, int64_t n, double q_macro);

/* Derived constants: out[0..7] = gamma0, beta0, dt, dt_b, NSFD A,
 * q_macro, steps done, particles. */
int mithra_constants(mithra_handle h, double *out8);

/* Tuning calls.  The field sweep (NSFD update of A and phi) has several
 * workgroup tile shapes (x columns, y rows, z planes per workgroup);
 * `mithra_sweep_shape_count` gives their number, `mithra_set_sweep_shape`
 * selects one for the handle (EINVAL out of range), and
 * `mithra_time_sweep` times `iters` launches of the sweep for the current
 * step with HIP events on the handle's stream (shape -1: the current one),
 * writing the mean milliseconds to *ms.  Repeating the sweep leaves the
 * run's state unchanged.  Errors: EINVAL, ESTATE, EDEVICE. */
int mithra_sweep_shape_count(void);
int mithra_set_sweep_shape(mithra_handle h, int shape);
int mithra_time_sweep(mithra_handle h, int shape, int iters, double *ms);

/* Measurement call: run n_steps exactly as mithra_step would, by direct
 * launches with HIP events on the handle's stream around every sweep
 * launch and around every whole step; synchronises, then adds the summed
 * milliseconds to *sweep_ms and *step_ms.  Errors: EINVAL, ESTATE,
 * EDEVICE. */
int mithra_step_timed(mithra_handle h, int64_t n_steps, double *sweep_ms, double *step_ms);

/* Measurement call: run n_steps exactly as mithra_step would, by direct
 * launches with HIP events on the handle's stream between the stages of
 * every step; synchronises, then adds the summed milliseconds per stage to
 * stage_ms[0..5] (0 field sweep, 1 Mur boundaries, 2 vertex E and B with
 * the plane-power partial sums, 3 gather + push + deposit, 4 box
 * reductions + bin and sort, 5 step tail) and of the whole steps to
 * stage_ms[6] (seven doubles, caller-owned).  Errors: EINVAL, ESTATE,
 * EDEVICE. */
int mithra_step_profile(mithra_handle h, int64_t n_steps, double *stage_ms);

/* Sweep-shape autotuner: times every distinct sweep tile shape on this
 * run's grid, each with the boundary kernel it implies, over `iters`
 * launches, selects the fastest for the handle and writes it to
 * *best_shape (nullable).  Results are cached per (precision,
 * compensation, space charge, grid size) for the process.  The run's state
 * is unchanged.  Errors: EINVAL, ESTATE (no bunch loaded), EDEVICE. */
int mithra_autotune_sweep(mithra_handle h, int iters, int *best_shape);

/* ---- Batches: many independent runs stepped together -------------------
 *
 * Runs of different grid sizes, particle counts, precisions and sweep
 * shapes, each created and loaded as usual, are stepped by grouped
 * launches: every stage of the PIC step is one launch per kernel variant
 * for all member runs that use it, the members' workgroups laid end to
 * end.  One batched step is captured into a HIP graph at creation and
 * replayed.  Each member stops at its own step count.  Results are those
 * of the same runs stepped alone (the step arithmetic of a run does not
 * depend on the other members; only the order of floating-point atomic
 * additions in the deposit may differ, as between two solo runs).
 *
 * While a handle belongs to a batch, mithra_step and mithra_step_timed on
 * it fail with ESTATE; the read calls synchronise the batch stream as well
 * as the handle's own.  Destroy the batch before destroying its members. */
typedef struct mithra_batch_s *mithra_batch;

/* Device workspace needed by a batch of n runs (group tables), or 0 for
 * n <= 0.  Pure function. */
size_t mithra_batch_workspace_bytes(int32_t n_runs);

/* Create a batch of n distinct loaded handles (not in another batch) on
 * `hip_stream`, borrowing
 * `dev_workspace` (256-byte aligned, at least the size above) for the
 * batch's lifetime.  Synchronises the members' streams.  Errors: EINVAL,
 * ENOMEM (workspace), ESTATE (a member not loaded or already batched),
 * EDEVICE. */
int mithra_batch_create(const mithra_handle *runs, int32_t n_runs, void *dev_workspace, size_t workspace_bytes,
                        void *hip_stream, mithra_batch *out);

/* Advance member i by n_steps[i] >= 0 steps (array of n_runs).  Waits for
 * the batch's previous work, then enqueues max_i n_steps[i] replays of the
 * batched step and returns without waiting.  Errors: EINVAL, EDEVICE. */
int mithra_batch_run(mithra_batch b, const int64_t *n_steps);

/* Choose the sweep tile shape of the batch's members with the whole batch
 * on the device: per member class (precision, compensation), every shape is
 * timed as the class's grouped sweep and Mur launches (`iters` >= 1 timed
 * repetitions after one warm-up), the fastest is kept for all members of
 * the class, and the batched step is captured again.  A small grid timed
 * alone (mithra_autotune_sweep) leaves most of the GPU idle, so the two
 * choices differ.  The runs' state is unchanged (sweep and Mur only
 * rewrite the next time level and re-clear the next source set).  Waits
 * for the batch's previous work.  If `shapes_out` is not NULL it receives
 * each member's shape (n_runs entries).  Errors: EINVAL, ENOMEM, EDEVICE;
 * after an error, destroy the batch. */
int mithra_batch_autotune_sweep(mithra_batch b, int iters, int32_t *shapes_out);

/* Wait for the batch's enqueued work. */
int mithra_batch_sync(mithra_batch b);

/* Message of the last error on the batch (never NULL). */
const char *mithra_batch_last_error(mithra_batch b);

/* Wait for the batch's work and release it; the members become ordinary
 * handles again (their step counts include the batched steps). */
int mithra_batch_destroy(mithra_batch b);

/* Message of the last error on this handle (never NULL). */
const char *mithra_last_error(mithra_handle h);

/* Release the host-side state.  The arena stays the caller's. */
int mithra_destroy(mithra_handle h);

#ifdef __cplusplus
}
#endif

#endif /* MITHRA_H_ */
