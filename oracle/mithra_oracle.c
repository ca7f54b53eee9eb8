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
    int32_t pad_;
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
    int32_t *cell;                      /* per id: linear node index of the cell corner, -1 inactive */
    int64_t step;
    int loaded;
    int generic_faces;                  /* test hook: first-order faces via the residual solve */
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
    /* dispersion-free along z: dt = dz / c; bunch step dt_b = dt / N */
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
    free(S->key);
    free(S->perm);
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

static void lab_planar(const ora_state *S, double x, double y, double zl, double theta, double Bl[3])
{
    double ku = 2.0 * PI_ / S->d.lambda_u;
    double B0 = 2.0 * PI_ * m_e * c_light * S->d.K / (q_e * S->d.lambda_u);
    double Lu = S->d.n_periods * S->d.lambda_u;
    double eta = x * sin(theta) + y * cos(theta);
    double gfun, hfun;
    if (zl < 0.0) {
        double s = ku * zl;
        gfun = s * exp(-0.5 * s * s);
        hfun = exp(-0.5 * s * s);
    } else if (zl > Lu) {
        double s = ku * (zl - Lu);
        gfun = s * exp(-0.5 * s * s);
        hfun = exp(-0.5 * s * s);
    } else {
        gfun = sin(ku * zl);
        hfun = cos(ku * zl);
    }
    double Bperp = B0 * cosh(ku * eta) * gfun;
    Bl[0] = Bperp * sin(theta);
    Bl[1] = Bperp * cos(theta);
    Bl[2] = B0 * sinh(ku * eta) * hfun;
}

void ora_external_field(void *h, const double r[3], double t, double E[3], double B[3])
{
    ora_state *S = (ora_state *)h;
    double g0 = S->gamma0, b0 = S->beta0;
    double zl = g0 * (r[2] - S->d.z_entrance + b0 * c_light * t);
    double Bl[3] = {0, 0, 0}, tmp[3];
    double th = S->d.pol_angle_deg * PI_ / 180.0;
    if (S->d.und_type == 1) {
        lab_planar(S, r[0], r[1], zl, 0.0, tmp);
        for (int a = 0; a < 3; ++a)
            Bl[a] += tmp[a];
        lab_planar(S, r[0], r[1], zl + 0.25 * S->d.lambda_u, 0.5 * PI_, tmp);
        for (int a = 0; a < 3; ++a)
            Bl[a] += tmp[a];
    } else {
        lab_planar(S, r[0], r[1], zl, th, Bl);
    }
    /* E = g0 (E' + c beta0 z x B') - (g0-1) E'_z z ; B = g0 B' - (g0-1) B'_z z */
    E[0] = g0 * (c_light * b0 * (-Bl[1]));
    E[1] = g0 * (c_light * b0 * (Bl[0]));
    E[2] = 0.0;
    B[0] = g0 * Bl[0];
    B[1] = g0 * Bl[1];
    B[2] = g0 * Bl[2] - (g0 - 1.0) * Bl[2];
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
/* by particle id.                                                      */
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
static int cmp_key_id(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    uint32_t ka = g_sort_keys[ia], kb = g_sort_keys[ib];
    if (ka != kb)
        return ka < kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

static void sort_particles(ora_state *S)
{
    for (int64_t p = 0; p < S->np; ++p) {
        double r[3] = {S->r[0][p], S->r[1][p], S->r[2][p]};
        S->key[p] = cell_key(S, r, &S->cell[p]);
        S->perm[p] = (int32_t)p;
    }
    g_sort_keys = S->key;
    qsort(S->perm, (size_t)S->np, sizeof(int32_t), cmp_key_id);
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
    free(S->cell);
    S->key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    S->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S->cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
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

/* One full PIC step in the order: potentials, Mur, vertex fields, push,
 * sort, deposit. */
void ora_step(void *h, int64_t nsteps)
{
    ora_state *S = (ora_state *)h;
    for (int64_t it = 0; it < nsteps; ++it) {
        for (int c = 0; c < S->ncomp; ++c)
            sweep_component(S, c);
        for (int c = 0; c < S->ncomp; ++c)
            mur_component(S, c);
        fields_at_vertices(S);
        if (S->np > 0) {
            push_particles(S);
            sort_particles(S);
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
        for (int c = 0; c < S->ncomp; ++c)
            mur_component(S, c);
        fields_at_vertices(S);
        rotate_levels(S);
        S->step += 1;
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

/* |<exp(i k_r z)>| over particles in active cells, k_r = 2 pi / lambda*,
 * lambda* = lambda_u / (gamma0 beta0). */
double ora_bunching(void *h)
{
    ora_state *S = (ora_state *)h;
    double kr = 2.0 * PI_ * S->gamma0 * S->beta0 / S->d.lambda_u;
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
