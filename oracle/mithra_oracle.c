/*
 * mithra_oracle.c -- plain FP64 CPU reference of the boosted-frame FDTD/PIC
 * time step of the MITHRA 2.0 manual (arXiv 2009.13645).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU path is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg may load it; no product code path calls it.  It shares no
 * code, header, constant table or helper with the GPU library.
 *
 * Written for obviousness, not speed: one loop nest per equation, FP64
 * throughout, compiled with -O2 -ffp-contract=off.  OpenMP only on the
 * per-node sweep loops and the per-particle push loop, whose results do
 * not depend on thread count.  The deposit runs serially in sorted order.
 *
 * Where the manual is silent, ambiguous or garbled, the reading taken is
 * stated at the function that implements it.
 *
 * Units: SI.  Boosted-frame mesh spacings dx, dy, dz; node (i,j,k) sits at
 * (x0 + i dx, y0 + j dy, z0 + k dz); arrays are [nz][ny][nx], x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 */
static const double c_light = 299792458.0;
static const double q_e = 1.602176634e-19;
static const double m_e = 9.1093837015e-31;
static const double eps_0 = 8.8541878128e-12;
#define MU_0 (1.0 / (eps_0 * c_light * c_light))
#define PI_ 3.14159265358979323846

/* Run description.  Mirrors the physical inputs of the manual's MESH and
 * UNDULATOR groups, with the mesh already in the boosted frame. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t truncation_order; /* 1 or 2 (Mur order) */
    int32_t space_charge;     /* 0: phi == 0; 1: solve for phi */
    int32_t solver;           /* 0: NSFD, 1: standard FD */
    int32_t n_sub;            /* bunch sub-steps per field step, N = dt/dt_b */
    int32_t und_type;         /* 0 planar, 1 helical */
    int32_t n_periods;        /* undulator length in periods */
    int32_t k_plane;          /* radiated-power plane (node index along z) */
    int32_t tile[3];          /* sort tile dimensions (cells) */
    int32_t sort_every;       /* sort after every sort_every-th push (0, 1: every push) */
    double dx, dy, dz;
    double x0, y0, z0;
    double gamma;             /* beam Lorentz factor (lab) */
    double K, lambda_u, pol_angle_deg;
    double z_entrance;        /* boosted-frame z of the entrance at t = 0 */
} ora_desc;

enum { F_EX = 0, F_EY, F_EZ, F_BX, F_BY, F_BZ, F_AX, F_AY, F_AZ, F_JX, F_JY, F_JZ, F_PHI, F_RHO };

typedef struct {
    ora_desc d;
    int64_t nn;
    int ncomp;                          /* 3 or 4 potentials */
    double gamma0, beta0, dt, dtb;
    double nsfd_A;                      /* NSFD averaging coefficient */
    double a1, a2, a3, a4, a5, a6, a7, a8;
    double *pot[3][4];                  /* [0]=n-1, [1]=n, [2]=n+1 */
    double *J[3];                       /* edge currents J_l(node + 1/2 e_l) */
    double *rho;
    double *E[3], *B[3];
    int64_t np;
    double *r[3], *u[3];                /* indexed by particle id */
    double *r_old[3];
    double q;                           /* macro-particle charge (C) */
    uint32_t *key;                      /* per id */
    int32_t *perm;                      /* perm[rank] = id */
    int32_t *prev_rank;                 /* prev_rank[id]: rank in the last order */
    int32_t *cell;                      /* per id: linear node index of the cell corner, -1 inactive */
    int64_t step;
    int loaded;
    int generic_faces;                  /* test hook: first-order faces via the residual solve */
    /* undulator extensions (ora_set_undulator) */
    int n_modules;                      /* static array: modules, K_m = K + m dK */
    double gap, dK;                     /* lab gap between modules (m), tapering step of K */
    int opt_signal;                     /* optical: signal type (0 Neumann, 1 Gaussian, 2 sech, 3 sinusoidal) */
    double opt_a0, opt_lambda, opt_ctau, opt_ct0, opt_cep; /* strength, wavelength, pulse length, offset, CEP (deg) */
    double opt_w0[2], opt_zf;           /* Gaussian beam: waists along / across the polarisation, focus (lab z') */
    /* TF/SF seed (ora_set_seed) */
    int seed_on, seed_type, seed_signal;
    double seed_a0, seed_lambda, seed_ctau, seed_ct0, seed_cep, seed_pol_deg, seed_w0, seed_zf;
    /* spectral power through the diagnostic plane (ora_set_spectrum) */
    int nf;
    double *omega;                      /* boosted angular frequencies */
    double *spec;                       /* [nf][8][nx*ny]: re/im of Ex' Ey' Bx' By' (lab) */
} ora_state;

static inline int64_t IDX(const ora_state *S, int i, int j, int k)
{
    return ((int64_t)k * S->d.ny + j) * S->d.nx + i;
}

/* ------------------------------------------------------------------ */
/* Set-up: Lorentz boost of the mesh and time step (sec. "Lorentz       */
/* Transformation"), NSFD coefficients (eq. NSFDCoefficient and the     */
/* update-equation coefficients).                                       */
/* ------------------------------------------------------------------ */

void *ora_create(const ora_desc *d)
{
    ora_state *S = (ora_state *)calloc(1, sizeof(ora_state));
    S->d = *d;
    S->nn = (int64_t)d->nx * d->ny * d->nz;
    S->ncomp = d->space_charge ? 4 : 3;
    /* gamma0 from the first undulator: planar gamma/sqrt(1+K^2/2); helical
     * (not in the manual; textbook resonance) gamma/sqrt(1+K^2). */
    if (d->und_type == 1)
        S->gamma0 = d->gamma / sqrt(1.0 + d->K * d->K);
    else
        S->gamma0 = d->gamma / sqrt(1.0 + 0.5 * d->K * d->K);
    S->beta0 = sqrt(1.0 - 1.0 / (S->gamma0 * S->gamma0));
    /* NSFD: dispersion-free along z with dt = dz / c.  Standard FD cannot
     * take that step (it violates the stability condition, eq.
     * CFLcondition); reading: it takes 0.99 of the largest stable step
     * 1 / (c sqrt(1/dx^2 + 1/dy^2 + 1/dz^2)).  Bunch step dt_b = dt / N. */
    if (d->solver == 1)
        S->dt = 0.99 / (c_light * sqrt(1.0 / (d->dx * d->dx) + 1.0 / (d->dy * d->dy) + 1.0 / (d->dz * d->dz)));
    else
        S->dt = d->dz / c_light;
    S->dtb = S->dt / (double)(d->n_sub > 0 ? d->n_sub : 1);

    double cdt = c_light * S->dt;
    double rx2 = (cdt / d->dx) * (cdt / d->dx);
    double ry2 = (cdt / d->dy) * (cdt / d->dy);
    double rz2 = (cdt / d->dz) * (cdt / d->dz);
    if (d->solver == 0) {
        double qx = (d->dz / d->dx) * (d->dz / d->dx) + (d->dz / d->dy) * (d->dz / d->dy);
        S->nsfd_A = 0.25 * (1.0 + 0.02 / qx);
        double A = S->nsfd_A;
        S->a1 = 2.0 * (1.0 - (1.0 - 2.0 * A) * rx2 - (1.0 - 2.0 * A) * ry2 - rz2);
        S->a2 = S->a3 = rx2;
        S->a4 = S->a5 = ry2;
        /* The manual prints the x ratio twice in alpha'_6; the averaging of
         * the y second difference makes the second term the y ratio. */
        S->a6 = S->a7 = rz2 - 2.0 * A * rx2 - 2.0 * A * ry2;
    } else {
        S->nsfd_A = 0.0;
        S->a1 = 2.0 * (1.0 - rx2 - ry2 - rz2);
        S->a2 = S->a3 = rx2;
        S->a4 = S->a5 = ry2;
        S->a6 = S->a7 = rz2;
    }
    S->a8 = cdt * cdt;

    for (int l = 0; l < 3; ++l)
        for (int c = 0; c < 4; ++c)
            S->pot[l][c] = (double *)calloc((size_t)S->nn, sizeof(double));
    for (int c = 0; c < 3; ++c) {
        S->J[c] = (double *)calloc((size_t)S->nn, sizeof(double));
        S->E[c] = (double *)calloc((size_t)S->nn, sizeof(double));
        S->B[c] = (double *)calloc((size_t)S->nn, sizeof(double));
    }
    S->rho = (double *)calloc((size_t)S->nn, sizeof(double));
    S->n_modules = 1;
    return S;
}

void ora_destroy(void *h)
{
    ora_state *S = (ora_state *)h;
    if (!S)
        return;
    for (int l = 0; l < 3; ++l)
        for (int c = 0; c < 4; ++c)
            free(S->pot[l][c]);
    for (int c = 0; c < 3; ++c) {
        free(S->J[c]);
        free(S->E[c]);
        free(S->B[c]);
        free(S->r[c]);
        free(S->u[c]);
        free(S->r_old[c]);
    }
    free(S->rho);
    free(S->omega);
    free(S->spec);
    free(S->key);
    free(S->perm);
    free(S->prev_rank);
    free(S->cell);
    free(S);
}

/* out[0..15]: gamma0 beta0 dt dtb A a1 a2 a3 a4 a5 a6 a7 a8 q np step */
void ora_consts(void *h, double *out)
{
    ora_state *S = (ora_state *)h;
    out[0] = S->gamma0;
    out[1] = S->beta0;
    out[2] = S->dt;
    out[3] = S->dtb;
    out[4] = S->nsfd_A;
    out[5] = S->a1;
    out[6] = S->a2;
    out[7] = S->a3;
    out[8] = S->a4;
    out[9] = S->a5;
    out[10] = S->a6;
    out[11] = S->a7;
    out[12] = S->a8;
    out[13] = S->q;
    out[14] = (double)S->np;
    out[15] = (double)S->step;
}

/* ------------------------------------------------------------------ */
/* FDTD: NSFD update of one potential component at interior nodes      */
/* (eqs. NSFDtrick and updateEquation; scalar potential with the same   */
/* scheme, sec. "FDTD for Scalar Potential").                          */
/*                                                                     */
/* Source reading: discretising  lap(psi) - psi_tt / c^2 = zeta  gives  */
/* the source term -(c dt)^2 zeta.  With zeta = -mu0 J for A and       */
/* zeta = -rho/eps0 for phi this is +(c dt)^2 mu0 J and +(c dt)^2      */
/* rho/eps0, which makes a positive charge raise phi.                  */
/*                                                                     */
/* Current reading: the zigzag current lives on cell edges; the nodal  */
/* A_l update takes the mean of the two edges adjacent along l.        */
/* ------------------------------------------------------------------ */

static double source_at(const ora_state *S, int comp, int i, int j, int k)
{
    int64_t c = IDX(S, i, j, k);
    switch (comp) {
    case 0:
        return MU_0 * 0.5 * (S->J[0][IDX(S, i - 1, j, k)] + S->J[0][c]);
    case 1:
        return MU_0 * 0.5 * (S->J[1][IDX(S, i, j - 1, k)] + S->J[1][c]);
    case 2:
        return MU_0 * 0.5 * (S->J[2][IDX(S, i, j, k - 1)] + S->J[2][c]);
    default:
        return S->rho[c] / eps_0;
    }
}

static void sweep_component(ora_state *S, int comp)
{
    const double *pm = S->pot[0][comp];
    const double *p0 = S->pot[1][comp];
    double *pp = S->pot[2][comp];
    const int nx = S->d.nx, ny = S->d.ny, nz = S->d.nz;
    const double A = S->nsfd_A;
#pragma omp parallel for schedule(static)
    for (int k = 1; k < nz - 1; ++k)
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                /* z-averaged neighbour value psi-bar at (ii, jj, k) */
#define BAR(ii, jj) (A * p0[IDX(S, ii, jj, k - 1)] + (1.0 - 2.0 * A) * p0[IDX(S, ii, jj, k)] + A * p0[IDX(S, ii, jj, k + 1)])
                int64_t c = IDX(S, i, j, k);
                double v = -pm[c] + S->a1 * p0[c]
                           + S->a2 * BAR(i + 1, j) + S->a3 * BAR(i - 1, j)
                           + S->a4 * BAR(i, j + 1) + S->a5 * BAR(i, j - 1)
                           + S->a6 * p0[IDX(S, i, j, k + 1)] + S->a7 * p0[IDX(S, i, j, k - 1)]
                           + S->a8 * source_at(S, comp, i, j, k);
#undef BAR
                pp[c] = v;
            }
}

/* ------------------------------------------------------------------ */
/* Mur absorbing boundaries (sec. "Boundary Truncation").               */
/* Faces: first-order beta or second-order gamma update, written for   */
/* the z faces in the manual; the x and y faces permute the axes.       */
/* The manual's second-order PDE prints the transverse terms with a     */
/* minus sign; its gamma coefficients correspond to the plus sign, and  */
/* the coefficients are taken as authoritative.                         */
/* Edges and corners: the manual asks to discretise the conditions at   */
/* the centre of the square (edge) or cube (corner) and add them.  The  */
/* second-order conditions would reach outside the box there, so the    */
/* first-order condition of each adjacent face is used; the sum is      */
/* solved for the edge (corner) node.  Order: faces, edges, corners.    */
/* ------------------------------------------------------------------ */

static int n_of(const ora_state *S, int ax) { return ax == 0 ? S->d.nx : (ax == 1 ? S->d.ny : S->d.nz); }
static double h_of(const ora_state *S, int ax) { return ax == 0 ? S->d.dx : (ax == 1 ? S->d.dy : S->d.dz); }

static int64_t IDXv(const ora_state *S, const int p[3]) { return IDX(S, p[0], p[1], p[2]); }

/* boundary status of one coordinate: -1 low face, +1 high face, 0 inside */
static int bside(const ora_state *S, int ax, int v)
{
    if (v == 0)
        return -1;
    if (v == n_of(S, ax) - 1)
        return 1;
    return 0;
}

static double mur_face_value(const ora_state *S, int comp, const int p[3], int ax, int side)
{
    const double *xm = S->pot[0][comp], *x0 = S->pot[1][comp], *xp = S->pot[2][comp];
    int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
    double cdt = c_light * S->dt;
    double hn = h_of(S, ax);
    double r1 = cdt / h_of(S, t1), r2 = cdt / h_of(S, t2);
    int q[3] = {p[0], p[1], p[2]};
    q[ax] = p[ax] - side; /* first node inside along the normal */
    int64_t b = IDXv(S, p), in = IDXv(S, q);
    if (S->d.truncation_order == 1) {
        double be0 = (cdt - hn) / (cdt + hn), be1 = 2.0 * hn / (cdt + hn), be2 = -1.0;
        double be3 = be1, be4 = be0;
        return be0 * xm[b] + be1 * x0[b] + be2 * xm[in] + be3 * x0[in] + be4 * xp[in];
    }
    double g0 = (cdt - hn) / (cdt + hn);
    double g1 = hn * (2.0 - r1 * r1 - r2 * r2) / (cdt + hn);
    double g2 = -1.0, g3 = g1, g4 = g0;
    double g5 = r1 * r1 * hn / (2.0 * (cdt + hn)), g6 = g5, g9 = g5, g10 = g5;
    double g7 = r2 * r2 * hn / (2.0 * (cdt + hn)), g8 = g7, g11 = g7, g12 = g7;
    /* transverse neighbours at time n on the boundary plane (p) and on the
     * first inner plane (q) */
    int qa[3], qb[3], qc[3], qd[3], pa[3], pb[3], pc[3], pd[3];
    for (int a = 0; a < 3; ++a) {
        qa[a] = qb[a] = qc[a] = qd[a] = q[a];
        pa[a] = pb[a] = pc[a] = pd[a] = p[a];
    }
    qa[t1] += 1; qb[t1] -= 1; qc[t2] += 1; qd[t2] -= 1;
    pa[t1] += 1; pb[t1] -= 1; pc[t2] += 1; pd[t2] -= 1;
    double v = g0 * xm[b] + g1 * x0[b] + g2 * xm[in] + g3 * x0[in] + g4 * xp[in]
               + g5 * x0[IDXv(S, qa)] + g6 * x0[IDXv(S, qb)]
               + g7 * x0[IDXv(S, qc)] + g8 * x0[IDXv(S, qd)]
               + g9 * x0[IDXv(S, pa)] + g10 * x0[IDXv(S, pb)]
               + g11 * x0[IDXv(S, pc)] + g12 * x0[IDXv(S, pd)];
    return v;
}

/* Residual of the sum of the first-order one-way conditions of the
 * boundary axes of node p, each discretised at the centre of the 2^m node
 * stencil spanned by those axes, with the node's own n+1 value set to u. */
static double edge_residual(const ora_state *S, int comp, const int p[3], const int axes[3], int m, double u)
{
    const double *xm = S->pot[0][comp], *x0 = S->pot[1][comp], *xp = S->pot[2][comp];
    int64_t self = IDXv(S, p);
    int nstencil = 1 << m;
    double res = 0.0;
    for (int ia = 0; ia < m; ++ia) {
        int a = axes[ia];
        int side = bside(S, a, p[a]);
        double ha = h_of(S, a);
        /* outward normal derivative, time-centred mixed derivative:
         * (1/(2 dt ha)) * mean over pairs of [(X_b - X_i)^{n+1} - (X_b - X_i)^{n-1}] */
        double mix = 0.0;
        int npairs = 0;
        for (int s = 0; s < nstencil; ++s) {
            int bit_a = (s >> ia) & 1;
            if (bit_a)
                continue; /* enumerate pairs by their boundary-side member */
            int pb[3] = {p[0], p[1], p[2]};
            for (int ib = 0; ib < m; ++ib)
                if ((s >> ib) & 1)
                    pb[axes[ib]] -= bside(S, axes[ib], p[axes[ib]]);
            int pi_[3] = {pb[0], pb[1], pb[2]};
            pi_[a] -= side;
            int64_t ib_ = IDXv(S, pb), ii_ = IDXv(S, pi_);
            double xb_p = (ib_ == self) ? u : xp[ib_];
            double xi_p = (ii_ == self) ? u : xp[ii_];
            mix += (xb_p - xi_p) - (xm[ib_] - xm[ii_]);
            ++npairs;
        }
        mix /= (2.0 * S->dt * ha * (double)npairs);
        /* (1/c) second time derivative at the centre: mean over the stencil */
        double tt = 0.0;
        for (int s = 0; s < nstencil; ++s) {
            int pn[3] = {p[0], p[1], p[2]};
            for (int ib = 0; ib < m; ++ib)
                if ((s >> ib) & 1)
                    pn[axes[ib]] -= bside(S, axes[ib], p[axes[ib]]);
            int64_t id = IDXv(S, pn);
            double xn1 = (id == self) ? u : xp[id];
            tt += xn1 - 2.0 * x0[id] + xm[id];
        }
        tt /= ((double)nstencil * c_light * S->dt * S->dt);
        res += mix + tt;
    }
    return res;
}

static void mur_component(ora_state *S, int comp)
{
    double *xp = S->pot[2][comp];
    const int nx = S->d.nx, ny = S->d.ny, nz = S->d.nz;
    for (int pass = 1; pass <= 3; ++pass) /* faces, edges, corners */
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int p[3] = {i, j, k};
                    int axes[3], m = 0;
                    for (int a = 0; a < 3; ++a)
                        if (bside(S, a, p[a]) != 0)
                            axes[m++] = a;
                    if (m != pass)
                        continue;
                    if (m == 1 && !(S->generic_faces && S->d.truncation_order == 1)) {
                        xp[IDXv(S, p)] = mur_face_value(S, comp, p, axes[0], bside(S, axes[0], p[axes[0]]));
                    } else {
                        double r0 = edge_residual(S, comp, p, axes, m, 0.0);
                        double r1 = edge_residual(S, comp, p, axes, m, 1.0);
                        xp[IDXv(S, p)] = -r0 / (r1 - r0);
                    }
                }
}

/* ------------------------------------------------------------------ */
/* Fields at the vertices (sec. "Field Evaluation"): E and B at         */
/* t_{n+1/2} from A^n, A^{n+1} and phi (which is stored half a step     */
/* ahead).  The printed B_z at n+1 has A_x(i-1) where the curl needs    */
/* A_y(i-1); A_y is used.  Evaluated at nodes whose six neighbours are  */
/* inside the box.                                                      */
/* ------------------------------------------------------------------ */

static void fields_at_vertices(ora_state *S)
{
    const int nx = S->d.nx, ny = S->d.ny, nz = S->d.nz;
    const double dx = S->d.dx, dy = S->d.dy, dz = S->d.dz, dt = S->dt;
    const double *Axn = S->pot[1][0], *Ayn = S->pot[1][1], *Azn = S->pot[1][2];
    const double *Axp = S->pot[2][0], *Ayp = S->pot[2][1], *Azp = S->pot[2][2];
    const double *ph = S->pot[1][3];
    const int sc = S->d.space_charge;
#pragma omp parallel for schedule(static)
    for (int k = 1; k < nz - 1; ++k)
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                int64_t c = IDX(S, i, j, k);
                int64_t xp_ = IDX(S, i + 1, j, k), xm_ = IDX(S, i - 1, j, k);
                int64_t yp_ = IDX(S, i, j + 1, k), ym_ = IDX(S, i, j - 1, k);
                int64_t zp_ = IDX(S, i, j, k + 1), zm_ = IDX(S, i, j, k - 1);
                S->B[0][c] = 0.5 * ((Azn[yp_] - Azn[ym_]) / (2 * dy) - (Ayn[zp_] - Ayn[zm_]) / (2 * dz)
                                    + (Azp[yp_] - Azp[ym_]) / (2 * dy) - (Ayp[zp_] - Ayp[zm_]) / (2 * dz));
                S->B[1][c] = 0.5 * ((Axn[zp_] - Axn[zm_]) / (2 * dz) - (Azn[xp_] - Azn[xm_]) / (2 * dx)
                                    + (Axp[zp_] - Axp[zm_]) / (2 * dz) - (Azp[xp_] - Azp[xm_]) / (2 * dx));
                S->B[2][c] = 0.5 * ((Ayn[xp_] - Ayn[xm_]) / (2 * dx) - (Axn[yp_] - Axn[ym_]) / (2 * dy)
                                    + (Ayp[xp_] - Ayp[xm_]) / (2 * dx) - (Axp[yp_] - Axp[ym_]) / (2 * dy));
                double gx = 0.0, gy = 0.0, gz = 0.0;
                if (sc) {
                    gx = (ph[xp_] - ph[xm_]) / (2 * dx);
                    gy = (ph[yp_] - ph[ym_]) / (2 * dy);
                    gz = (ph[zp_] - ph[zm_]) / (2 * dz);
                }
                S->E[0][c] = -(Axp[c] - Axn[c]) / dt - gx;
                S->E[1][c] = -(Ayp[c] - Ayn[c]) / dt - gy;
                S->E[2][c] = -(Azp[c] - Azn[c]) / dt - gz;
            }
}

/* ------------------------------------------------------------------ */
/* Particles: grid coordinates and the active region                    */
/* ------------------------------------------------------------------ */

static void grid_coords(const ora_state *S, const double r[3], double g[3])
{
    g[0] = (r[0] - S->d.x0) / S->d.dx;
    g[1] = (r[1] - S->d.y0) / S->d.dy;
    g[2] = (r[2] - S->d.z0) / S->d.dz;
}

/* A cell (i,j,k) is active when 1 <= i <= nx-3 (same in y, z): all eight
 * corners are interior nodes, where fields are evaluated and sources are
 * consumed.  Returns the corner's linear node index or -1. */
static int64_t active_cell(const ora_state *S, const double g[3], int c[3])
{
    for (int a = 0; a < 3; ++a) {
        double f = floor(g[a]);
        if (!(f >= 1.0 && f <= (double)(n_of(S, a) - 3)))
            return -1;
        c[a] = (int)f;
    }
    return IDX(S, c[0], c[1], c[2]);
}

/* Trilinear (cloud-in-cell) gather (eq. fieldInterpolation).  The printed
 * weights carry an absolute value that would give node i full weight at
 * delta = dx; the linear weights 1 - delta and delta are used. */
static void gather(const ora_state *S, const double r[3], double E[3], double B[3])
{
    double g[3];
    int c[3];
    grid_coords(S, r, g);
    for (int a = 0; a < 3; ++a)
        E[a] = B[a] = 0.0;
    if (active_cell(S, g, c) < 0)
        return;
    double w[3][2];
    for (int a = 0; a < 3; ++a) {
        double del = g[a] - (double)c[a];
        w[a][0] = 1.0 - del;
        w[a][1] = del;
    }
    for (int K = 0; K < 2; ++K)
        for (int J = 0; J < 2; ++J)
            for (int I = 0; I < 2; ++I) {
                double wt = w[0][I] * w[1][J] * w[2][K];
                int64_t n = IDX(S, c[0] + I, c[1] + J, c[2] + K);
                for (int a = 0; a < 3; ++a) {
                    E[a] += wt * S->E[a][n];
                    B[a] += wt * S->B[a][n];
                }
            }
}

/* ------------------------------------------------------------------ */
/* External undulator field (sec. "Static Undulator Field").            */
/* Lab-frame field of a planar undulator whose field direction makes    */
/* angle theta with y (theta = 0: field along y, as in eq.              */
/* undulatorField), entrance fringe (eq. fringingField) for z' < 0 and  */
/* the same fringe mirrored at the exit (reading: the exit is silent).  */
/* Position mapped by eq. LorentzTransformR2L with the entrance at      */
/* z_entrance at t = 0; fields boosted by eqs.                          */
/* LorentzTransformElectric/Magnetic with E' = 0.  Helical (reading):   */
/* the theta = 0 pattern plus the theta = 90 deg pattern shifted        */
/* upstream by a quarter period.                                        */
/* ------------------------------------------------------------------ */

/* Window of the fringe fields inside the gap of an undulator array (eq.
 * fringingFieldGap and the window function after it): 1 at the module
 * edge (dz = 0), about 6e-5 at the far end of the gap (dz = g). */
static double gap_window(double dz, double g)
{
    double t = PI_ * dz / g;
    return 0.35875 + 0.48829 * cos(t) + 0.14128 * cos(2.0 * t) + 0.01168 * cos(3.0 * t);
}

/* Longitudinal profile of the planar pattern at lab position zl (entrance
 * of the first module at 0): *gB multiplies cosh(k_u eta) for the
 * transverse field, *hB multiplies sinh(k_u eta) for B'_z; both include
 * the module's field amplitude B0_m = 2 pi m c K_m / (e lambda_u),
 * K_m = K + m dK (tapering).  Modules of N_u periods are separated by
 * gaps g.  Inside a module: sin and cos of k_u (zl - entrance).  Before the
 * first entrance and after the last exit: the fringe of eq. fringingField
 * (reading: the exit mirrors the entrance).  Inside a gap: the exit fringe
 * of the module before and the entrance fringe of the module after, each
 * times the gap window of its distance to its own edge. */
static void array_profile(const ora_state *S, double zl, double *gB, double *hB)
{
    const double ku = 2.0 * PI_ / S->d.lambda_u;
    const double Lu = S->d.n_periods * S->d.lambda_u;
    const int M = S->n_modules > 0 ? S->n_modules : 1;
    const double pitch = Lu + S->gap;
    double B0[2];
    int m = (int)floor(zl / pitch);
    if (m < 0)
        m = 0;
    if (m > M - 1)
        m = M - 1;
    const double ent = m * pitch, ext = ent + Lu;
    B0[0] = 2.0 * PI_ * m_e * c_light * (S->d.K + m * S->dK) / (q_e * S->d.lambda_u);
    if (zl >= ent && zl <= ext) {
        *gB = B0[0] * sin(ku * (zl - ent));
        *hB = B0[0] * cos(ku * (zl - ent));
        return;
    }
    if (zl < ent) { /* before the first module (m == 0) */
        double a = ku * (zl - ent), e = exp(-0.5 * a * a);
        *gB = B0[0] * (a * e);
        *hB = B0[0] * e;
        return;
    }
    /* after module m's exit */
    double a1 = ku * (zl - ext), e1 = exp(-0.5 * a1 * a1);
    if (m == M - 1) {
        *gB = B0[0] * (a1 * e1);
        *hB = B0[0] * e1;
        return;
    }
    const double ent2 = (m + 1) * pitch;
    B0[1] = 2.0 * PI_ * m_e * c_light * (S->d.K + (m + 1) * S->dK) / (q_e * S->d.lambda_u);
    double a2 = ku * (zl - ent2), e2 = exp(-0.5 * a2 * a2);
    double f1 = gap_window(zl - ext, S->gap), f2 = gap_window(ent2 - zl, S->gap);
    *gB = B0[0] * (a1 * e1) * f1 + B0[1] * (a2 * e2) * f2;
    *hB = B0[0] * e1 * f1 + B0[1] * e2 * f2;
}

static void lab_planar(const ora_state *S, double x, double y, double zl, double theta, double Bl[3])
{
    double ku = 2.0 * PI_ / S->d.lambda_u;
    double eta = x * sin(theta) + y * cos(theta);
    double gB, hB;
    array_profile(S, zl, &gB, &hB);
    double Bperp = gB * cosh(ku * eta);
    Bl[0] = Bperp * sin(theta);
    Bl[1] = Bperp * cos(theta);
    Bl[2] = hB * sinh(ku * eta);
}

/* Time signature of an optical pulse (eq. signalTypes) with unit
 * amplitude: tau is the retarded time, f the carrier frequency, tp the
 * pulse duration (FWHM of the intensity), t0 the offset, ph the phase.
 * The modulated Neumann form is scaled by tp so that it is dimensionless
 * (reading: the printed form carries a 1/time factor). */
static double signal_value(int type, double tau, double f, double tp, double t0, double ph)
{
    double d = tau - t0;
    double car = cos(2.0 * PI_ * f * d + ph);
    double ln2 = log(2.0);
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

/* Lab-frame fields of the optical undulator (sec. "Optical Undulator
 * Field"), a wave propagating along -z with strength a0 = K and
 * wavelength lambda_l = 2 lambda_u (the static undulator it matches).
 * Its magnetic field points along (sin theta, cos theta, 0) like the static
 * field, its electric field along p = (-cos theta, sin theta, 0).
 * Field amplitude E0 = a0 m c omega / e.  Plane wave (und_type 2): eq.
 * opticalUndulatorPW.  Gaussian beam (und_type 3): eq. opticalUndulatorGB
 * with w(l) = w0 sqrt(1 + (l/z_R)^2) and R(l) = l (1 + (z_R/l)^2)
 * (reading of the printed r/z_R), l = z_f - z' the distance along the
 * propagation from the focus, E_perp = B_par = 0. */
static void lab_optical(const ora_state *S, double x, double y, double zl, double tl, double El[3], double Bl[3])
{
    const double th = S->d.pol_angle_deg * PI_ / 180.0;
    const double lam = 2.0 * S->d.lambda_u;
    const double om = 2.0 * PI_ * c_light / lam;
    const double E0 = S->d.K * m_e * c_light * om / q_e;
    const double f = c_light / lam, tp = S->opt_ctau / c_light, t0 = S->opt_ct0 / c_light;
    const double cep = S->opt_cep * PI_ / 180.0;
    const double p[3] = {-cos(th), sin(th), 0.0}; /* E direction */
    const double q[3] = {sin(th), cos(th), 0.0};  /* B direction, (-z) x p */
    if (S->d.und_type == 2) {
        double sv = signal_value(S->opt_signal, tl + zl / c_light, f, tp, t0, cep);
        for (int a = 0; a < 3; ++a) {
            El[a] = E0 * sv * p[a];
            Bl[a] = (E0 / c_light) * sv * q[a];
        }
        return;
    }
    const double k0 = 2.0 * PI_ / lam;
    const double l = S->opt_zf - zl;
    const double rp = x * p[0] + y * p[1], rq = x * q[0] + y * q[1]; /* along / across the polarisation */
    const double w0p = S->opt_w0[0], w0q = S->opt_w0[1];
    const double zRp = PI_ * w0p * w0p / lam, zRq = PI_ * w0q * w0q / lam;
    const double wp = w0p * sqrt(1.0 + (l / zRp) * (l / zRp)), wq = w0q * sqrt(1.0 + (l / zRq) * (l / zRq));
    const double iRp = l / (l * l + zRp * zRp), iRq = l / (l * l + zRq * zRq);
    const double amp = sqrt((w0p * w0q) / (wp * wq)) * exp(-rq * rq / (wq * wq) - rp * rp / (wp * wp));
    const double curv = -0.5 * k0 * rp * rp * iRp - 0.5 * k0 * rq * rq * iRq;
    const double Gp = atan(l / zRp), Gq = atan(l / zRq);
    const double tau = tl - l / c_light; /* retarded time along the propagation */
    const double Epar = E0 * amp * signal_value(S->opt_signal, tau, f, tp, t0, cep + curv - 0.5 * PI_ + 0.5 * (Gp + Gq));
    const double Elon = E0 * (rp * w0p / (zRp * wp)) * amp *
                        signal_value(S->opt_signal, tau, f, tp, t0, cep + curv + 0.5 * (3.0 * Gp + Gq));
    const double Blon = (E0 / c_light) * (rq * w0q / (zRq * wq)) * amp *
                        signal_value(S->opt_signal, tau, f, tp, t0, cep + curv + 0.5 * (Gp + 3.0 * Gq));
    /* propagation direction -z: E = E_par p + E_l (-z), B = (E_par / c) q + B_l (-z);
     * with l along the propagation, r_par along p and r_perp along q the
     * printed longitudinal components make both fields divergence-free to
     * paraxial order */
    for (int a = 0; a < 2; ++a) {
        El[a] = Epar * p[a];
        Bl[a] = (Epar / c_light) * q[a];
    }
    El[2] = -Elon;
    Bl[2] = -Blon;
}

void ora_external_field(void *h, const double r[3], double t, double E[3], double B[3])
{
    ora_state *S = (ora_state *)h;
    double g0 = S->gamma0, b0 = S->beta0;
    double zl = g0 * (r[2] - S->d.z_entrance + b0 * c_light * t);
    double Bl[3] = {0, 0, 0}, El[3] = {0, 0, 0}, tmp[3];
    double th = S->d.pol_angle_deg * PI_ / 180.0;
    if (S->d.und_type >= 2) {
        /* lab time of the event: t' = gamma0 (t + beta0 (z - z_entrance) / c) */
        double tl = g0 * (t + b0 * (r[2] - S->d.z_entrance) / c_light);
        lab_optical(S, r[0], r[1], zl, tl, El, Bl);
    } else if (S->d.und_type == 1) {
        lab_planar(S, r[0], r[1], zl, 0.0, tmp);
        for (int a = 0; a < 3; ++a)
            Bl[a] += tmp[a];
        lab_planar(S, r[0], r[1], zl + 0.25 * S->d.lambda_u, 0.5 * PI_, tmp);
        for (int a = 0; a < 3; ++a)
            Bl[a] += tmp[a];
    } else {
        lab_planar(S, r[0], r[1], zl, th, Bl);
    }
    /* eqs. LorentzTransformElectric/Magnetic with beta0 along z:
     * E = g0 (E' + c beta0 z x B') - (g0-1) E'_z z ; B = g0 (B' - beta0 z x E' / c) - (g0-1) B'_z z */
    E[0] = g0 * (El[0] + c_light * b0 * (-Bl[1]));
    E[1] = g0 * (El[1] + c_light * b0 * (Bl[0]));
    E[2] = g0 * El[2] - (g0 - 1.0) * El[2];
    B[0] = g0 * (Bl[0] - b0 * (-El[1]) / c_light);
    B[1] = g0 * (Bl[1] - b0 * (El[0]) / c_light);
    B[2] = g0 * Bl[2] - (g0 - 1.0) * Bl[2];
}

/* Undulator extensions: p[0] modules, p[1] gap (lab, m), p[2] tapering
 * step dK, p[3] optical signal type, p[4] pulse length c tau (lab, m),
 * p[5] offset c t0 (lab, m), p[6] CEP (deg), p[7] Gaussian-beam waist along
 * the polarisation, p[8] waist across it (m), p[9] focus (lab z' relative to
 * the undulator reference, m). */
void ora_set_undulator(void *h, const double *p)
{
    ora_state *S = (ora_state *)h;
    S->n_modules = (int)p[0];
    S->gap = p[1];
    S->dK = p[2];
    S->opt_signal = (int)p[3];
    S->opt_ctau = p[4];
    S->opt_ct0 = p[5];
    S->opt_cep = p[6];
    S->opt_w0[0] = p[7];
    S->opt_w0[1] = p[8];
    S->opt_zf = p[9];
}

/* ------------------------------------------------------------------ */
/* Boris push (eq. BorisScheme); the printed r^l is r^m.                */
/* ------------------------------------------------------------------ */

void ora_boris(const double u_in[3], const double E[3], const double B[3], double dtb, double u_out[3])
{
    double ek = q_e * dtb / (2.0 * m_e * c_light);
    double t1[3], t2[3], t3[3];
    for (int a = 0; a < 3; ++a)
        t1[a] = u_in[a] - ek * E[a];
    double alpha = -q_e * dtb / (2.0 * m_e * sqrt(1.0 + t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]));
    double cr[3];
    cr[0] = t1[1] * B[2] - t1[2] * B[1];
    cr[1] = t1[2] * B[0] - t1[0] * B[2];
    cr[2] = t1[0] * B[1] - t1[1] * B[0];
    for (int a = 0; a < 3; ++a)
        t2[a] = t1[a] + alpha * cr[a];
    double bb = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    double f = 2.0 * alpha / (1.0 + alpha * alpha * bb);
    double s[3] = {f * B[0], f * B[1], f * B[2]};
    cr[0] = t2[1] * s[2] - t2[2] * s[1];
    cr[1] = t2[2] * s[0] - t2[0] * s[2];
    cr[2] = t2[0] * s[1] - t2[1] * s[0];
    for (int a = 0; a < 3; ++a)
        t3[a] = t1[a] + cr[a];
    for (int a = 0; a < 3; ++a)
        u_out[a] = t3[a] - ek * E[a];
}

/* One field step of particle motion: N sub-steps with the grid field
 * held at t_{n+1/2} and the undulator field re-evaluated at each
 * sub-step's position and time. */
static void push_particles(ora_state *S)
{
    double t_half = ((double)S->step + 0.5) * S->dt;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < S->np; ++p) {
        double r[3] = {S->r[0][p], S->r[1][p], S->r[2][p]};
        double u[3] = {S->u[0][p], S->u[1][p], S->u[2][p]};
        for (int a = 0; a < 3; ++a)
            S->r_old[a][p] = r[a];
        double Eg[3], Bg[3];
        gather(S, r, Eg, Bg);
        for (int s = 0; s < S->d.n_sub; ++s) {
            double Ee[3], Be[3], Et[3], Bt[3], un[3];
            ora_external_field(S, r, t_half + (double)s * S->dtb, Ee, Be);
            for (int a = 0; a < 3; ++a) {
                Et[a] = Eg[a] + Ee[a];
                Bt[a] = Bg[a] + Be[a];
            }
            ora_boris(u, Et, Bt, S->dtb, un);
            double ig = 1.0 / sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
            for (int a = 0; a < 3; ++a) {
                u[a] = un[a];
                r[a] = r[a] + c_light * S->dtb * un[a] * ig;
            }
        }
        for (int a = 0; a < 3; ++a) {
            S->r[a][p] = r[a];
            S->u[a][p] = u[a];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Cell index and sort order.  key = tile-major cell index for an       */
/* active cell, 0xFFFFFFFF otherwise; the order is ascending key, ties  */
/* in the previous order (the last sort's ranks; before the first sort, */
/* the particle ids): a stable sort of the previous order by key.       */
/* ------------------------------------------------------------------ */

static uint32_t cell_key(const ora_state *S, const double r[3], int32_t *cell_lin)
{
    double g[3];
    int c[3];
    grid_coords(S, r, g);
    if (active_cell(S, g, c) < 0) {
        *cell_lin = -1;
        return 0xFFFFFFFFu;
    }
    *cell_lin = (int32_t)IDX(S, c[0], c[1], c[2]);
    int Tx = S->d.tile[0], Ty = S->d.tile[1], Tz = S->d.tile[2];
    int ntx = (S->d.nx - 1 + Tx - 1) / Tx, nty = (S->d.ny - 1 + Ty - 1) / Ty;
    uint64_t tile_lin = ((uint64_t)(c[2] / Tz) * nty + (uint64_t)(c[1] / Ty)) * ntx + (uint64_t)(c[0] / Tx);
    uint64_t local = ((uint64_t)(c[2] % Tz) * Ty + (uint64_t)(c[1] % Ty)) * Tx + (uint64_t)(c[0] % Tx);
    return (uint32_t)(tile_lin * (uint64_t)(Tx * Ty * Tz) + local);
}

static const uint32_t *g_sort_keys;
static const int32_t *g_prev_rank;
static int cmp_key_rank(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    uint32_t ka = g_sort_keys[ia], kb = g_sort_keys[ib];
    if (ka != kb)
        return ka < kb ? -1 : 1;
    int32_t ra = g_prev_rank[ia], rb = g_prev_rank[ib];
    return ra < rb ? -1 : (ra > rb ? 1 : 0);
}

/* Cells and keys of the current positions, the order unchanged (a step
 * without a sort). */
static void update_cells(ora_state *S)
{
    for (int64_t p = 0; p < S->np; ++p) {
        double r[3] = {S->r[0][p], S->r[1][p], S->r[2][p]};
        S->key[p] = cell_key(S, r, &S->cell[p]);
    }
}

static void sort_particles(ora_state *S)
{
    for (int64_t rank = 0; rank < S->np; ++rank)
        S->prev_rank[S->perm[rank]] = (int32_t)rank;
    for (int64_t p = 0; p < S->np; ++p) {
        double r[3] = {S->r[0][p], S->r[1][p], S->r[2][p]};
        S->key[p] = cell_key(S, r, &S->cell[p]);
    }
    g_sort_keys = S->key;
    g_prev_rank = S->prev_rank;
    qsort(S->perm, (size_t)S->np, sizeof(int32_t), cmp_key_rank);
}

/* ------------------------------------------------------------------ */
/* Charge-conserving deposit (sec. "Current Deposition").               */
/* Zigzag path of Umeda et al.: the move r1 -> r2 is split at the relay */
/* point (printed relay formula), so that each segment stays in one     */
/* cell.  The current of a straight segment inside one cell is the      */
/* exact one for linear weights: the flux of the trilinear weight       */
/* through each edge, i.e. F_x [(1-Wy)(1-Wz) + dy dz / 12] at (i+1/2,   */
/* j, k) and the matching terms at j+1, k+1 (W = segment midpoint in    */
/* the cell, d = segment displacement, grid units).  Without the dy dz  */
/* term, the midpoint product leaves a continuity residual of           */
/* dx dy dz / 4 per segment in 3-D.  Charge: cloud-in-cell at nodes.    */
/* ------------------------------------------------------------------ */

static void deposit_segment(ora_state *S, const double a[3], const double b[3], const int c[3])
{
    const double V = S->d.dx * S->d.dy * S->d.dz;
    const double h[3] = {S->d.dx, S->d.dy, S->d.dz};
    double d[3], W[3];
    for (int l = 0; l < 3; ++l) {
        d[l] = b[l] - a[l];
        W[l] = 0.5 * (a[l] + b[l]) - (double)c[l];
    }
    for (int l = 0; l < 3; ++l) {
        int m1 = (l + 1) % 3, m2 = (l + 2) % 3;
        double F = S->q * d[l] * h[l] / (S->dt * V);
        double cross = d[m1] * d[m2] / 12.0;
        double w00 = (1.0 - W[m1]) * (1.0 - W[m2]) + cross;
        double w10 = W[m1] * (1.0 - W[m2]) - cross;
        double w01 = (1.0 - W[m1]) * W[m2] - cross;
        double w11 = W[m1] * W[m2] + cross;
        int p[3] = {c[0], c[1], c[2]};
        S->J[l][IDXv(S, p)] += F * w00;
        p[m1] += 1;
        S->J[l][IDXv(S, p)] += F * w10;
        p[m2] += 1;
        S->J[l][IDXv(S, p)] += F * w11;
        p[m1] -= 1;
        S->J[l][IDXv(S, p)] += F * w01;
    }
}

static void deposit_move(ora_state *S, const double r1[3], const double r2[3])
{
    double g1[3], g2[3], gr[3];
    int c1[3], c2[3];
    grid_coords(S, r1, g1);
    grid_coords(S, r2, g2);
    if (active_cell(S, g1, c1) < 0 || active_cell(S, g2, c2) < 0)
        return;
    for (int l = 0; l < 3; ++l) {
        double lo = (double)(c1[l] < c2[l] ? c1[l] : c2[l]) + 1.0;
        double hi = (double)(c1[l] > c2[l] ? c1[l] : c2[l]);
        double mid = 0.5 * (g1[l] + g2[l]);
        gr[l] = fmin(lo, fmax(hi, mid));
    }
    deposit_segment(S, g1, gr, c1);
    deposit_segment(S, gr, g2, c2);
}

static void deposit_charge(ora_state *S, const double r[3])
{
    double g[3];
    int c[3];
    grid_coords(S, r, g);
    if (active_cell(S, g, c) < 0)
        return;
    const double V = S->d.dx * S->d.dy * S->d.dz;
    double w[3][2];
    for (int a = 0; a < 3; ++a) {
        double del = g[a] - (double)c[a];
        w[a][0] = 1.0 - del;
        w[a][1] = del;
    }
    for (int K = 0; K < 2; ++K)
        for (int J = 0; J < 2; ++J)
            for (int I = 0; I < 2; ++I)
                S->rho[IDX(S, c[0] + I, c[1] + J, c[2] + K)] += (S->q / V) * w[0][I] * w[1][J] * w[2][K];
}

/* J from the moves r_old -> r (both cells active), rho from r (cell
 * active), accumulated in sorted order. */
static void deposit_all(ora_state *S)
{
    for (int c = 0; c < 3; ++c)
        memset(S->J[c], 0, sizeof(double) * (size_t)S->nn);
    memset(S->rho, 0, sizeof(double) * (size_t)S->nn);
    for (int64_t rank = 0; rank < S->np; ++rank) {
        int32_t p = S->perm[rank];
        double r1[3] = {S->r_old[0][p], S->r_old[1][p], S->r_old[2][p]};
        double r2[3] = {S->r[0][p], S->r[1][p], S->r[2][p]};
        deposit_move(S, r1, r2);
        deposit_charge(S, r2);
    }
}

/* ------------------------------------------------------------------ */
/* Bunch loading.  Inputs: positions at t = dt/2, momenta u = gamma     */
/* beta at t = 0.  The previous half-step position is the straight      */
/* backward drift r - c dt u / gamma (reading; the manual is silent).   */
/* ------------------------------------------------------------------ */

int ora_load_bunch(void *h, int64_t n, const double *xyz, const double *u, double q)
{
    ora_state *S = (ora_state *)h;
    if (n <= 0)
        return -1;
    S->np = n;
    S->q = q;
    for (int a = 0; a < 3; ++a) {
        free(S->r[a]);
        free(S->u[a]);
        free(S->r_old[a]);
        S->r[a] = (double *)malloc(sizeof(double) * (size_t)n);
        S->u[a] = (double *)malloc(sizeof(double) * (size_t)n);
        S->r_old[a] = (double *)malloc(sizeof(double) * (size_t)n);
    }
    free(S->key);
    free(S->perm);
    free(S->prev_rank);
    free(S->cell);
    S->key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    S->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S->prev_rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S->cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t p = 0; p < n; ++p) /* the order before the first sort: by id */
        S->perm[p] = (int32_t)p;
    for (int64_t p = 0; p < n; ++p)
        for (int a = 0; a < 3; ++a) {
            S->r[a][p] = xyz[3 * p + a];
            S->u[a][p] = u[3 * p + a];
        }
    for (int64_t p = 0; p < n; ++p) {
        double uu[3] = {S->u[0][p], S->u[1][p], S->u[2][p]};
        double ig = 1.0 / sqrt(1.0 + uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]);
        for (int a = 0; a < 3; ++a)
            S->r_old[a][p] = S->r[a][p] - c_light * S->dt * uu[a] * ig;
    }
    sort_particles(S);
    deposit_all(S);
    S->step = 0;
    S->loaded = 1;
    return 0;
}

/* Swap time levels after a completed step: n-1 <- n, n <- n+1. */
static void rotate_levels(ora_state *S)
{
    for (int c = 0; c < 4; ++c) {
        double *t = S->pot[0][c];
        S->pot[0][c] = S->pot[1][c];
        S->pot[1][c] = S->pot[2][c];
        S->pot[2][c] = t;
    }
}

/* ------------------------------------------------------------------ */
/* Seed field by total-field / scattered-field injection (sec. "Seed   */
/* Field").  Nodes k = 1 (scattered-field boundary) and k = 2 (total-    */
/* field boundary) next to the z_min face: after the update of A, the   */
/* terms through which each used the other region's values are          */
/* corrected by the incident wave f at time level n.  Reading of the    */
/* signs: the printed corrections add the incident wave at the SF node  */
/* and subtract it at the TF node, which injects -f into the total      */
/* field; the corrections are taken with the opposite signs so that the */
/* total-field region (k >= 2) holds +f, the wave the seed describes.   */
/*                                                                      */
/* Incident wave (boosted frame, propagating along +z): transverse      */
/* vector potential A = A0 p s(t - (z - z_2)/c), p = (cos psi, sin psi,  */
/* 0), A0 = a0 m c / e, z_2 the TF plane.  The lab signal (wavelength,  */
/* duration, offset) is Doppler-scaled by D = gamma0 (1 + beta0), since */
/* t' - z'/c = (t - z/c) / D.  Gaussian seed: transverse amplitude      */
/* (w0/w(l)) exp(-r^2/w^2), phase -k r^2 / (2 R(l)) + atan(l / z_R),    */
/* l = z - z_f, with the boosted wavelength lambda D and z_R = pi w0^2  */
/* / (lambda D).                                                        */
/* ------------------------------------------------------------------ */

static double seed_incident(const ora_state *S, int comp, double x, double y, double z, double t)
{
    const double psi = S->seed_pol_deg * PI_ / 180.0;
    const double pc = comp == 0 ? cos(psi) : sin(psi);
    const double D = S->gamma0 * (1.0 + S->beta0);
    const double lam = S->seed_lambda * D;
    const double f = c_light / lam, tp = S->seed_ctau / c_light * D, t0 = S->seed_ct0 / c_light * D;
    const double A0 = S->seed_a0 * m_e * c_light / q_e;
    const double z2 = S->d.z0 + 2.0 * S->d.dz;
    const double tau = t - (z - z2) / c_light;
    double amp = 1.0, ph = S->seed_cep * PI_ / 180.0;
    if (S->seed_type == 1) {
        const double zR = PI_ * S->seed_w0 * S->seed_w0 / lam;
        const double l = z - S->seed_zf;
        const double w = S->seed_w0 * sqrt(1.0 + (l / zR) * (l / zR));
        const double r2 = x * x + y * y;
        amp = (S->seed_w0 / w) * exp(-r2 / (w * w));
        ph += -0.5 * (2.0 * PI_ / lam) * r2 * l / (l * l + zR * zR) + atan(l / zR);
    }
    return pc * A0 * amp * signal_value(S->seed_signal, tau, f, tp, t0, ph);
}

static void seed_inject(ora_state *S)
{
    if (!S->seed_on)
        return;
    const int nx = S->d.nx, ny = S->d.ny;
    const double t = (double)S->step * S->dt; /* time level n of the update */
    const double A = S->nsfd_A;
    for (int comp = 0; comp < 2; ++comp) {
        double *pp = S->pot[2][comp];
#define FI(ii, jj, kk) seed_incident(S, comp, S->d.x0 + (ii) * S->d.dx, S->d.y0 + (jj) * S->d.dy, S->d.z0 + (kk) * S->d.dz, t)
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                /* SF node (k = 1) used total-field values at k = 2 */
                double c1 = A * (S->a2 * FI(i + 1, j, 2) + S->a3 * FI(i - 1, j, 2) + S->a4 * FI(i, j + 1, 2) +
                                 S->a5 * FI(i, j - 1, 2)) + S->a6 * FI(i, j, 2);
                /* TF node (k = 2) used scattered-field values at k = 1 */
                double c2 = A * (S->a2 * FI(i + 1, j, 1) + S->a3 * FI(i - 1, j, 1) + S->a4 * FI(i, j + 1, 1) +
                                 S->a5 * FI(i, j - 1, 1)) + S->a7 * FI(i, j, 1);
                pp[IDX(S, i, j, 1)] -= c1;
                pp[IDX(S, i, j, 2)] += c2;
            }
#undef FI
    }
}

/* Seed: p[0] type (0 plane wave, 1 Gaussian beam), p[1] signal type, p[2]
 * a0, p[3] wavelength (lab, m), p[4] pulse length c tau (lab, m), p[5]
 * offset c t0 (lab, m), p[6] CEP (deg), p[7] polarisation angle psi of A
 * from x toward y (deg), p[8] waist (m), p[9] focus (boosted z, m). */
void ora_set_seed(void *h, const double *p)
{
    ora_state *S = (ora_state *)h;
    S->seed_on = 1;
    S->seed_type = (int)p[0];
    S->seed_signal = (int)p[1];
    S->seed_a0 = p[2];
    S->seed_lambda = p[3];
    S->seed_ctau = p[4];
    S->seed_ct0 = p[5];
    S->seed_cep = p[6];
    S->seed_pol_deg = p[7];
    S->seed_w0 = p[8];
    S->seed_zf = p[9];
}

/* Incident seed potential at a point (for tests). */
double ora_seed_incident(void *h, int comp, const double r[3], double t)
{
    return seed_incident((ora_state *)h, comp, r[0], r[1], r[2], t);
}

/* ------------------------------------------------------------------ */
/* Spectral radiated power (ch. 4 FEL-OUTPUT, radiation power at a       */
/* normalised frequency).  Reading: running Fourier transforms, over     */
/* the boosted time t_{n+1/2} of the vertex fields, of the lab-frame     */
/* fields E'_x E'_y B'_x B'_y at every interior node of the diagnostic   */
/* plane, F(omega) = sum_n F(t_n) exp(-i omega t_n) dt, at omega =        */
/* nu omega_r (omega_r = 2 pi c / lambda*, the boosted resonant          */
/* frequency).  The spectral energy through the plane per unit angular   */
/* frequency is dW/domega = (1/pi) (dx dy / mu0) sum Re(E'_x B'_y* -     */
/* E'_y B'_x*), so that its integral over omega >= 0 is the time         */
/* integral of the instantaneous power (Parseval).                       */
/* ------------------------------------------------------------------ */

void ora_set_spectrum(void *h, int nf, double nu_min, double nu_max)
{
    ora_state *S = (ora_state *)h;
    free(S->omega);
    free(S->spec);
    S->omega = NULL;
    S->spec = NULL;
    S->nf = nf > 0 ? nf : 0;
    if (!S->nf)
        return;
    const double om_r = 2.0 * PI_ * c_light * S->gamma0 * S->beta0 / S->d.lambda_u;
    S->omega = (double *)malloc(sizeof(double) * (size_t)nf);
    for (int f = 0; f < nf; ++f) {
        double nu = nf == 1 ? nu_min : nu_min + (nu_max - nu_min) * f / (double)(nf - 1);
        S->omega[f] = nu * om_r;
    }
    S->spec = (double *)calloc((size_t)nf * 8 * (size_t)S->d.nx * S->d.ny, sizeof(double));
}

static void spectrum_accumulate(ora_state *S)
{
    if (!S->nf)
        return;
    const int nx = S->d.nx, ny = S->d.ny, k = S->d.k_plane;
    const double g0 = S->gamma0, b0 = S->beta0;
    const double t = ((double)S->step + 0.5) * S->dt;
    const size_t plane = (size_t)nx * ny;
    for (int f = 0; f < S->nf; ++f) {
        const double c = cos(S->omega[f] * t) * S->dt, sn = -sin(S->omega[f] * t) * S->dt;
        double *acc = S->spec + (size_t)f * 8 * plane;
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                int64_t n = IDX(S, i, j, k);
                double Ex = S->E[0][n], Ey = S->E[1][n], Bx = S->B[0][n], By = S->B[1][n];
                double F[4];
                F[0] = g0 * (Ex + b0 * c_light * By);
                F[1] = g0 * (Ey - b0 * c_light * Bx);
                F[2] = g0 * (Bx - b0 * Ey / c_light);
                F[3] = g0 * (By + b0 * Ex / c_light);
                size_t p = (size_t)j * nx + i;
                for (int q = 0; q < 4; ++q) {
                    acc[(size_t)(2 * q) * plane + p] += F[q] * c;
                    acc[(size_t)(2 * q + 1) * plane + p] += F[q] * sn;
                }
            }
    }
}

/* dW/domega (J s) at each frequency, accumulated over the steps so far. */
void ora_spectral_power(void *h, double *out)
{
    ora_state *S = (ora_state *)h;
    const int nx = S->d.nx, ny = S->d.ny;
    const size_t plane = (size_t)nx * ny;
    for (int f = 0; f < S->nf; ++f) {
        const double *acc = S->spec + (size_t)f * 8 * plane;
        double sum = 0.0;
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                size_t p = (size_t)j * nx + i;
                double exr = acc[0 * plane + p], exi = acc[1 * plane + p];
                double eyr = acc[2 * plane + p], eyi = acc[3 * plane + p];
                double bxr = acc[4 * plane + p], bxi = acc[5 * plane + p];
                double byr = acc[6 * plane + p], byi = acc[7 * plane + p];
                /* Re(Ex By* - Ey Bx*) */
                sum += (exr * byr + exi * byi) - (eyr * bxr + eyi * bxi);
            }
        out[f] = sum * S->d.dx * S->d.dy / (MU_0 * PI_);
    }
}

/* One full PIC step in the order: potentials, Mur, vertex fields, push,
 * sort, deposit. */
void ora_step(void *h, int64_t nsteps)
{
    ora_state *S = (ora_state *)h;
    for (int64_t it = 0; it < nsteps; ++it) {
        for (int c = 0; c < S->ncomp; ++c)
            sweep_component(S, c);
        seed_inject(S);
        for (int c = 0; c < S->ncomp; ++c)
            mur_component(S, c);
        fields_at_vertices(S);
        spectrum_accumulate(S);
        if (S->np > 0) {
            push_particles(S);
            /* the order is refreshed after every sort_every-th push (the
             * push of step n is the (n+1)-th); in between the particles keep
             * their order, which the deposit follows */
            const int se = S->d.sort_every > 1 ? S->d.sort_every : 1;
            if ((S->step + 1) % se == 0)
                sort_particles(S);
            else
                update_cells(S);
            deposit_all(S);
        }
        rotate_levels(S);
        S->step += 1;
    }
}

/* Field-only step (no particles touched): potentials and Mur. */
void ora_field_step(void *h, int64_t nsteps)
{
    ora_state *S = (ora_state *)h;
    for (int64_t it = 0; it < nsteps; ++it) {
        for (int c = 0; c < S->ncomp; ++c)
            sweep_component(S, c);
        seed_inject(S);
        for (int c = 0; c < S->ncomp; ++c)
            mur_component(S, c);
        fields_at_vertices(S);
        spectrum_accumulate(S);
        rotate_levels(S);
        S->step += 1;
    }
}

/* ------------------------------------------------------------------ */
/* Bunch generation (sec. "Electron Bunch Generation").                 */
/* Quasi-random filling by Halton sequences: the value of element j of  */
/* sequence i is 1 minus the radical inverse of j in the base of the    */
/* i-th prime (the digits of j in that base mirrored behind the point). */
/* Uniform coordinates by eq. uniform1D, Gaussian ones by eqs.          */
/* gaussian1D and gaussian2D (Box-Muller on two sequences).             */
/* ------------------------------------------------------------------ */

double ora_halton(int i, uint64_t j)
{
    static const int prime[20] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71};
    const uint64_t b = (uint64_t)prime[i];
    double scale = 1.0, x = 0.0;
    for (uint64_t k = j; k > 0; k /= b) {
        scale /= (double)b;
        x += (double)(k % b) * scale;
    }
    return 1.0 - x;
}

/* Box-Muller pair from Halton sequences ia, ib at element j */
static void halton_normal(int ia, int ib, uint64_t j, double *c, double *s)
{
    double r = sqrt(-2.0 * log(ora_halton(ia, j)));
    double a = 2.0 * PI_ * ora_halton(ib, j);
    *c = r * cos(a);
    *s = r * sin(a);
}

/* Generate n macro-electrons in the boosted frame at the first half step.
 * p[0] longitudinal profile (0 flat-top, 1 Gaussian), p[1] transverse
 * profile (0 uniform, 1 Gaussian), p[2..4] bunch centre (boosted, m),
 * p[5], p[6] transverse sizes (lab: full widths if uniform, sigma if
 * Gaussian), p[7] longitudinal size (lab: flat-top length or sigma),
 * p[8] gamma, p[9] relative energy spread, p[10] transverse spread of u,
 * p[11] bunching factor b_f, p[12] its phase (rad), p[13] shot noise
 * (0/1), p[14] electrons represented, p[15] flat-top tapers (0/1).
 *
 * Sequences: x, y: 0, 1; z: 2 (and 3 for a Gaussian or a taper); energy:
 * 4, 5; transverse momentum: 6, 7; shot-noise slices: 8, 9 (by slice).
 * Flat-top with tapers (reading of the CSE remedy): a Gaussian of the
 * same density with rms width one lab radiation wavelength lambda* /
 * (gamma0 (1 + beta0)) is split, its lower half put behind the tail and
 * its upper half ahead of the head; the first round(n L / (L + sqrt(2
 * pi) sigma_t)) particles fill the flat part.
 * Lab lengths along z map to the boosted frame at fixed boosted time by
 * 1 / (gamma0 (1 - beta beta0)) (beta of the beam energy).  Momenta: lab
 * gamma' and u'_perp, u'_z = sqrt(gamma'^2 - 1 - u'_perp^2), boosted
 * u_z = gamma0 (u'_z - beta0 gamma') (4-velocity boost).
 * Bunching (eq. bunchingFactor; reading of the garbled form): the
 * modulation that becomes resonant after the undulator entrance has, at
 * load, the wavenumber k = k_b gamma0^2 (1 - beta beta0) beta0 / beta, with
 * k_b = gamma0 k_u (1 + beta0) the ponderomotive wavenumber (the lab
 * resonant wavenumber over gamma0: microbunches at rest in this frame,
 * half the boosted radiation wavelength apart), the entrance compressing
 * the bunch by that factor; dz = -(2 b_f / k) sin(k z + phase) gives
 * <exp(i k z)> = b_f exp(-i phase) to first order.  Shot noise: slices
 * 2 pi / k long; slice s has b_s = sqrt(-2 ln x_s) / sqrt(N_s), x_s from
 * sequence 8, phase 2 pi y_s from sequence 9 (reading: the printed [0, pi]
 * range is taken as [0, 2 pi)), N_s the electrons of the slice, and the
 * same displacement form. */
void ora_generate_bunch(void *h, const double *p, int64_t n, double *xyz, double *u)
{
    ora_state *S = (ora_state *)h;
    const double g0 = S->gamma0, b0 = S->beta0;
    const double gam = p[8];
    const double beta = sqrt(1.0 - 1.0 / (gam * gam));
    const double lz = 1.0 / (g0 * (1.0 - beta * b0));
    const double kr = 2.0 * PI_ * g0 * b0 / S->d.lambda_u; /* boosted radiation */
    const double kb = 2.0 * PI_ * g0 * (1.0 + b0) / S->d.lambda_u;
    const double k = kb * g0 * g0 * (1.0 - beta * b0) * b0 / beta;
    const double lam_lab = (2.0 * PI_ / kr) / (g0 * (1.0 + b0));
    const double L = p[7];
    const double sig_t = lam_lab;
    int64_t n_flat = n;
    if ((int)p[0] == 0 && (int)p[15] == 1)
        n_flat = (int64_t)llround((double)n * L / (L + sqrt(2.0 * PI_) * sig_t));
    for (int64_t q = 0; q < n; ++q) {
        const uint64_t j = (uint64_t)q;
        double x, y, zl, c, sn;
        if ((int)p[1] == 0) {
            x = p[5] * (ora_halton(0, j) - 0.5);
            y = p[6] * (ora_halton(1, j) - 0.5);
        } else {
            halton_normal(0, 1, j, &c, &sn);
            x = p[5] * c;
            y = p[6] * sn;
        }
        if ((int)p[0] == 1) {
            halton_normal(2, 3, j, &c, &sn);
            zl = L * c;
        } else if (q < n_flat) {
            zl = L * (ora_halton(2, j) - 0.5);
        } else {
            halton_normal(2, 3, j, &c, &sn);
            zl = (q & 1) ? 0.5 * L + sig_t * fabs(c) : -0.5 * L - sig_t * fabs(c);
        }
        double ge, ux, uy;
        halton_normal(4, 5, j, &c, &sn);
        ge = gam * (1.0 + p[9] * c);
        halton_normal(6, 7, j, &c, &sn);
        ux = p[10] * c;
        uy = p[10] * sn;
        double uzl = sqrt(ge * ge - 1.0 - ux * ux - uy * uy);
        xyz[3 * q + 0] = p[2] + x;
        xyz[3 * q + 1] = p[3] + y;
        xyz[3 * q + 2] = p[4] + zl * lz;
        u[3 * q + 0] = ux;
        u[3 * q + 1] = uy;
        u[3 * q + 2] = g0 * (uzl - b0 * ge);
    }
    /* bunching factor and shot noise act on the boosted z at load */
    if (p[11] != 0.0)
        for (int64_t q = 0; q < n; ++q) {
            double z = xyz[3 * q + 2];
            xyz[3 * q + 2] = z - (2.0 * p[11] / k) * sin(k * z + p[12]);
        }
    if ((int)p[13] == 1 && n > 0) {
        double zmin = xyz[2];
        for (int64_t q = 1; q < n; ++q)
            if (xyz[3 * q + 2] < zmin)
                zmin = xyz[3 * q + 2];
        const double sl = 2.0 * PI_ / k;
        int64_t ns = 0;
        for (int64_t q = 0; q < n; ++q) {
            int64_t s_ = (int64_t)floor((xyz[3 * q + 2] - zmin) / sl);
            if (s_ + 1 > ns)
                ns = s_ + 1;
        }
        int64_t *cnt = (int64_t *)calloc((size_t)ns, sizeof(int64_t));
        for (int64_t q = 0; q < n; ++q)
            cnt[(int64_t)floor((xyz[3 * q + 2] - zmin) / sl)] += 1;
        double *dz = (double *)malloc(sizeof(double) * (size_t)n);
        for (int64_t q = 0; q < n; ++q) {
            double z = xyz[3 * q + 2];
            int64_t s_ = (int64_t)floor((z - zmin) / sl);
            double ne = fmax((double)cnt[s_] * p[14] / (double)n, 1.0);
            double bs = sqrt(-2.0 * log(ora_halton(8, (uint64_t)s_ + 1))) / sqrt(ne);
            double ph = 2.0 * PI_ * ora_halton(9, (uint64_t)s_ + 1);
            dz[q] = -(2.0 * bs / k) * sin(k * z + ph);
        }
        for (int64_t q = 0; q < n; ++q)
            xyz[3 * q + 2] += dz[q];
        free(dz);
        free(cnt);
    }
}

/* ------------------------------------------------------------------ */
/* Access                                                               */
/* ------------------------------------------------------------------ */

/* level: 0 = previous (n-1), 1 = current (n), 2 = next (n+1) */
void ora_set_potential(void *h, int comp, int level, const double *in)
{
    ora_state *S = (ora_state *)h;
    memcpy(S->pot[level][comp], in, sizeof(double) * (size_t)S->nn);
}

void ora_get_potential(void *h, int comp, int level, double *out)
{
    ora_state *S = (ora_state *)h;
    memcpy(out, S->pot[level][comp], sizeof(double) * (size_t)S->nn);
}

int ora_get_field(void *h, int id, double *out)
{
    ora_state *S = (ora_state *)h;
    const double *src = NULL;
    switch (id) {
    case F_EX: src = S->E[0]; break;
    case F_EY: src = S->E[1]; break;
    case F_EZ: src = S->E[2]; break;
    case F_BX: src = S->B[0]; break;
    case F_BY: src = S->B[1]; break;
    case F_BZ: src = S->B[2]; break;
    case F_AX: src = S->pot[1][0]; break;
    case F_AY: src = S->pot[1][1]; break;
    case F_AZ: src = S->pot[1][2]; break;
    case F_JX: src = S->J[0]; break;
    case F_JY: src = S->J[1]; break;
    case F_JZ: src = S->J[2]; break;
    case F_PHI: src = S->pot[1][3]; break;
    case F_RHO: src = S->rho; break;
    default: return -1;
    }
    memcpy(out, src, sizeof(double) * (size_t)S->nn);
    return 0;
}

/* Particles in id order; cell (linear corner node index or -1) and the
 * current sort permutation are optional. */
void ora_get_particles(void *h, double *xyz, double *u, int32_t *cell, int32_t *perm)
{
    ora_state *S = (ora_state *)h;
    for (int64_t p = 0; p < S->np; ++p)
        for (int a = 0; a < 3; ++a) {
            if (xyz)
                xyz[3 * p + a] = S->r[a][p];
            if (u)
                u[3 * p + a] = S->u[a][p];
        }
    if (cell)
        memcpy(cell, S->cell, sizeof(int32_t) * (size_t)S->np);
    if (perm)
        memcpy(perm, S->perm, sizeof(int32_t) * (size_t)S->np);
}

void ora_get_keys(void *h, uint32_t *keys)
{
    ora_state *S = (ora_state *)h;
    memcpy(keys, S->key, sizeof(uint32_t) * (size_t)S->np);
}

/* Vertex fields from the stored levels n (1) and n+1 (2), without a step. */
void ora_compute_fields(void *h)
{
    fields_at_vertices((ora_state *)h);
}

/* Field gather at an arbitrary point from the current vertex fields. */
void ora_gather(void *h, const double r[3], double E[3], double B[3])
{
    gather((ora_state *)h, r, E, B);
}

/* ------------------------------------------------------------------ */
/* Diagnostics                                                          */
/* ------------------------------------------------------------------ */

/* Lab-frame power through node plane k (reading: instantaneous Poynting
 * flux; the manual gives no formula).  Fields are inverted to the lab,
 * which moves at -beta0 relative to the simulation frame. */
double ora_radiated_power(void *h, int k)
{
    ora_state *S = (ora_state *)h;
    double g0 = S->gamma0, b0 = S->beta0, P = 0.0;
    if (k < 1 || k > S->d.nz - 2)
        return 0.0;
    for (int j = 1; j < S->d.ny - 1; ++j)
        for (int i = 1; i < S->d.nx - 1; ++i) {
            int64_t c = IDX(S, i, j, k);
            double Ex = S->E[0][c], Ey = S->E[1][c], Bx = S->B[0][c], By = S->B[1][c];
            double Exl = g0 * (Ex + b0 * c_light * By);
            double Eyl = g0 * (Ey - b0 * c_light * Bx);
            double Bxl = g0 * (Bx - b0 * Ey / c_light);
            double Byl = g0 * (By + b0 * Ex / c_light);
            P += (Exl * Byl - Eyl * Bxl);
        }
    return P * S->d.dx * S->d.dy / MU_0;
}

/* |<exp(i k_b z)>| over particles in active cells (sec. "Bunching
 * factor"; reading of the printed k_u): k_b = gamma0 k_u (1 + beta0), the
 * wavenumber of the ponderomotive wave that the forward radiation
 * (gamma0 beta0 k_u) and the backward undulator (gamma0 k_u) beat into,
 * i.e. the lab resonant wavenumber k_u beta0 / (1 - beta0) over gamma0. */
double ora_bunching(void *h)
{
    ora_state *S = (ora_state *)h;
    double kr = 2.0 * PI_ * S->gamma0 * (1.0 + S->beta0) / S->d.lambda_u;
    double re = 0.0, im = 0.0;
    int64_t n = 0;
    for (int64_t p = 0; p < S->np; ++p) {
        if (S->cell[p] < 0)
            continue;
        re += cos(kr * S->r[2][p]);
        im += sin(kr * S->r[2][p]);
        ++n;
    }
    if (n == 0)
        return 0.0;
    return sqrt(re * re + im * im) / (double)n;
}

/* Test hook: with first-order truncation, solve the faces with the same
 * summed-residual code as edges and corners (m = 1), so that the printed
 * beta update pins that code. */
void ora_set_generic_faces(void *h, int on)
{
    ((ora_state *)h)->generic_faces = on;
}

int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops (sweep and push) for later calls. */
void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
