/*
 * dss_oracle.c -- plain, slow, FP64 CPU reference for one time step of the
 * dense-suspension method of Monti, Rathee, Shen & Rosti, "A fast and efficient
 * tool to study the rheology of dense suspensions" (arXiv 2108.01013).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file: only tests/, the smoke check and the CPU-baseline leg of the benchmark
 * do.  It shares no code, header, table or constant with the HIP library.
 *
 * Everything is written from the paper's definitions, in the paper's notation,
 * without blocking, fusion or reordering:
 *   - ambient simple shear, Sec. 2 (opening paragraph);
 *   - minimum image + Lees-Edwards offset, eq. (le);
 *   - pair set = all pairs closer than the cutoff, by brute force, Sec. 2.1
 *     (the O(N^2) check the cell list replaces);
 *   - lubrication, eq. (hydro) with the matrices of Appendix A, eqs. (rst), (rlu),
 *     (rlu1) and the g^X, g^Y table, assembled as the printed 12x12 block matrices;
 *   - contact, eqs. (contact0) and (csi);
 *   - repulsion eq. (rep) and attraction eq. (att);
 *   - stresslets and bulk stress, eqs. (stress), (stresslet);
 *   - modified velocity-Verlet, Sec. 2.1 (numerical algorithm).
 *
 * Readings taken where the text is silent, garbled or inconsistent (each is
 * listed in the design notes and pinned by a CPU test):
 *   R1  prefactor of every X/Y coefficient is 6*pi*eta0;
 *   R2  the Y^C blocks act through the tangential projector T (printed "N x");
 *   R3  R'(E) rows: force rows multiply n, torque rows multiply n_perp;
 *   R4  n_perp = 2 n x (E n) (the printed (A + A^T) carries a factor 1/2);
 *   R5  g^{Y^H_ji}(a) = g^{Y^H_ij}(1/a) (printed with G, a typo);
 *   R6  "g(1/alpha)" substitutes alpha -> 1/alpha holding a_i and a_i + a_j fixed;
 *   R7  d* is clamped at >= 0 inside the lubrication coefficients;
 *   R8  each unordered pair enters the stress once;
 *   R9  Sigma_ab = (1/V) sum r_a F_b with r = x_j - x_i and F the force on i;
 *   R10 Lees-Edwards: crossing y >= L_y shifts x by -delta and u_x by -gdot L_y
 *       (opposite for y < 0), delta = fmod(gdot L_y t, L_x);
 *   R11 xi* = T(xi_old + u_t dt), capped when |xi*| >= mu |F_nor| / k_t, with
 *       |F_nor| including the dashpot; xi_old = 0 at first contact;
 *   R12 every listed pair (|r| < c (a_i + a_j)) gets lubrication; repulsion and
 *       attraction are truncated at the same list.
 *   R20 wavy shear, eq. (uinf): U_inf = (gdot y + W sin(k y), 0, 0), k = 2 pi n / L_y,
 *       so Omega_inf(y) = (0, 0, -(gdot + W k cos(k y)) / 2) and E_inf_xy(y) = E_inf_yx(y) =
 *       (gdot + W k cos(k y)) / 2 at each particle's own wrapped y; Faxen terms of eq. (rst)
 *       (F = -6 pi eta0 a [u - U_inf - a^2/6 lap U_inf]) and of the stresslet S^S
 *       ((1 + a^2/10 lap) E_inf_i); R'(E) takes E_i and E_j at the two particles; the
 *       2 eta0 E_inf of eq. (stress) is the box average (gdot/2: the wave averages out); the
 *       sine part is periodic in y, so the Lees-Edwards shift stays gdot L_y.
 *   R19 rolling resistance (Appendix roll), with k_r > 0: a second spring per
 *       contact, xi^r* = T(xi^r_old + u_r dt) with u_r = a_ij (n x w_i - n x w_j),
 *       a_ij = 2 a_i a_j / (a_i + a_j), capped when |xi^r*| >= mu_r |F_nor| / k_r
 *       (the Coulomb limitation, with its own coefficient mu_r); torques
 *       T_i = a_ij n x k_r xi^r*, T_j = -T_i; no force and no stress (the
 *       pseudo-force only drives the torque); xi^r_old = 0 at first contact.
 *   R18 with ec_ranges = 1 the electro-chemical forces keep the ranges of
 *       Fig. elch instead: repulsion while the surface distance d_ij < 20 lambda_D,
 *       attraction while d_ij < 4 a0; lubrication stays on |r| < c (a_i + a_j);
 *       the pair set is every pair inside any of these ranges.
 *
 * Beyond the invariants, three parts are pinned against hand-evaluated values of
 * the Appendix A table and closed forms: the magnitude of the log-singular Y
 * coefficients (tangential lubrication over sizes and gaps; the equal-sphere value
 * a/6 of Jeffrey and Onishi), the lubrication stresslet S^L (squeeze and sliding
 * pairs, and the stress power of a sheared pair), and which particle's strain
 * enters each column of R'(E).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no FMA contraction, so
 * the pair test r^2 < r_c^2 is evaluated as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    double L[3];          /* box lengths L_x, L_y, L_z */
    double shear_rate;    /* gdot */
    double eta0;          /* carrier-fluid viscosity */
    double rho;           /* particle density */
    double kn, kt;        /* normal / tangential spring constants */
    double gamma_n;       /* normal damping constant */
    double mu;            /* Coulomb friction coefficient mu_C */
    double F_ER;          /* repulsion strength */
    double lambda_D;      /* Debye length */
    double a0;            /* reference radius */
    double hamaker;       /* Hamaker constant A */
    double eps_vdw;       /* attraction regularisation, as a fraction of abar */
    double eps_lub;       /* lubrication regularisation epsilon */
    double cutoff_factor; /* pair listed iff |r| < cutoff_factor * (a_i + a_j) */
    double dt;            /* time step */
    double ec_ranges;     /* 1: electro-chemical forces over their own ranges (R18) */
    double kr;            /* rolling spring stiffness k_r (0: no rolling resistance, R19) */
    double mu_r;          /* rolling Coulomb coefficient (R19) */
    double wave_amp;      /* amplitude W of the wavy shear, eq. (uinf) (0: simple shear, R20) */
    double wave_n;        /* spatial periods n of the wave in L_y */
} orc_params;

/* ------------------------------------------------------------------------- */
/* Ambient flow: shear along x, gradient along y (Sec. 2), with the wave of   */
/* eq. (uinf) (R20):                                                          */
/*   U_inf(x) = (gdot y + W sin(k y), 0, 0),  k = 2 pi n / L_y,               */
/*   dU/dy = gdot + W k cos(k y),  Omega_inf = (0, 0, -dU/dy / 2),            */
/*   E_inf_12 = E_inf_21 = dU/dy / 2;  W = 0 is the simple shear.             */
/* ------------------------------------------------------------------------- */
static double wave_k(const orc_params *p) { return 2.0 * M_PI * p->wave_n / p->L[1]; }

static double shear_at(const orc_params *p, double y) /* dU/dy */
{
    if (p->wave_amp == 0.0) return p->shear_rate;
    double k = wave_k(p);
    return p->shear_rate + p->wave_amp * k * cos(k * y);
}

static void ambient_U(const orc_params *p, const double *x, double *U)
{
    U[0] = p->shear_rate * x[1];
    if (p->wave_amp != 0.0) U[0] += p->wave_amp * sin(wave_k(p) * x[1]);
    U[1] = 0.0;
    U[2] = 0.0;
}

static void ambient_Omega(const orc_params *p, double y, double *W)
{
    W[0] = 0.0;
    W[1] = 0.0;
    W[2] = -0.5 * shear_at(p, y);
}

static void ambient_E(const orc_params *p, double y, double E[3][3])
{
    memset(E, 0, 9 * sizeof(double));
    E[0][1] = 0.5 * shear_at(p, y);
    E[1][0] = 0.5 * shear_at(p, y);
}

/* Faxen Laplacians: lap U_inf = (-W k^2 sin(k y), 0, 0); lap E_inf_xy = -W k^3 cos(k y) / 2 */
static double lap_Ux(const orc_params *p, double y)
{
    if (p->wave_amp == 0.0) return 0.0;
    double k = wave_k(p);
    return -p->wave_amp * k * k * sin(k * y);
}

static double lap_Exy(const orc_params *p, double y)
{
    if (p->wave_amp == 0.0) return 0.0;
    double k = wave_k(p);
    return -0.5 * p->wave_amp * k * k * k * cos(k * y);
}

/* small vector helpers */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static void matvec3(const double M[3][3], const double *v, double *out)
{
    for (int a = 0; a < 3; ++a)
        out[a] = M[a][0] * v[0] + M[a][1] * v[1] + M[a][2] * v[2];
}

double orc_particle_mass(const orc_params *p, double a) { return p->rho * (4.0 / 3.0) * M_PI * a * a * a; }
double orc_particle_inertia(const orc_params *p, double a) { return 0.4 * orc_particle_mass(p, a) * a * a; }

/* History capacity M (Sec. 2.1, memory paragraph): volume of the shell of
 * thickness 2 a_min around a particle of radius a, in units of the smallest
 * particle's volume, rounded up. */
int orc_history_capacity(double a, double a_min)
{
    double shell = (a + 2.0 * a_min) * (a + 2.0 * a_min) * (a + 2.0 * a_min) - a * a * a;
    return (int)ceil(shell / (a_min * a_min * a_min));
}

/* ------------------------------------------------------------------------- */
/* Lees-Edwards boundary conditions, eq. (le).                                */
/* ------------------------------------------------------------------------- */
double orc_le_offset(const orc_params *p, int64_t step)
{
    double t = (double)step * p->dt;
    double s = p->shear_rate * p->L[1] * t;
    return fmod(s, p->L[0]);
}

/* Nearest periodic image of b seen from a: rows above / below are displaced by
 * +delta / -delta along x. */
void orc_min_image(const orc_params *p, double delta, const double *xa, const double *xb, double *r)
{
    double dx = xb[0] - xa[0];
    double dy = xb[1] - xa[1];
    double dz = xb[2] - xa[2];
    if (dy > 0.5 * p->L[1]) {
        dy -= p->L[1];
        dx -= delta;
    } else if (dy < -0.5 * p->L[1]) {
        dy += p->L[1];
        dx += delta;
    }
    dx -= p->L[0] * nearbyint(dx / p->L[0]);
    dz -= p->L[2] * nearbyint(dz / p->L[2]);
    r[0] = dx;
    r[1] = dy;
    r[2] = dz;
}

/* Ranges of the electro-chemical forces in surface distance (Fig. elch):     */
/* repulsion below 20 lambda_D, attraction below 4 a0; 0 for a force that is  */
/* off.  Only with ec_ranges (R18).                                           */
static double repulsion_range(const orc_params *p)
{
    return (p->F_ER != 0.0 && p->lambda_D > 0.0) ? 20.0 * p->lambda_D : 0.0;
}

static double attraction_range(const orc_params *p) { return p->hamaker != 0.0 ? 4.0 * p->a0 : 0.0; }

/* Listed pair test on squares: |r| < cutoff_factor (a_a + a_b), or with      */
/* ec_ranges |r| < max(cutoff_factor (a_a + a_b), a_a + a_b + longest range).  */
static double pair_cutoff(const orc_params *p, double aa, double ab)
{
    double rc = p->cutoff_factor * (aa + ab);
    if (p->ec_ranges != 0.0) {
        double rr = repulsion_range(p), ra = attraction_range(p);
        double ext = (aa + ab) + (rr > ra ? rr : ra);
        if (ext > rc) rc = ext;
    }
    return rc;
}

static int pair_listed(const orc_params *p, const double *r, double aa, double ab)
{
    double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    double rc = pair_cutoff(p, aa, ab);
    return r2 < rc * rc;
}

/* Wrap one particle into the primary box after the drift, eq. (le).  The
 * velocities given (any number of them, stride 3) receive the matching shift. */
static void le_wrap(const orc_params *p, double delta, double *x, double *u1, double *u2)
{
    const double Lx = p->L[0], Ly = p->L[1], Lz = p->L[2];
    if (x[1] >= Ly) {
        x[1] -= Ly;
        x[0] -= delta;
        if (u1) u1[0] -= p->shear_rate * Ly;
        if (u2) u2[0] -= p->shear_rate * Ly;
    } else if (x[1] < 0.0) {
        x[1] += Ly;
        x[0] += delta;
        if (u1) u1[0] += p->shear_rate * Ly;
        if (u2) u2[0] += p->shear_rate * Ly;
    }
    x[0] -= Lx * floor(x[0] / Lx);
    x[2] -= Lz * floor(x[2] / Lz);
}

/* ------------------------------------------------------------------------- */
/* Pair set by brute force: every pair checked once (the O(N^2) search that   */
/* the cell list of Sec. 2.1 replaces).  Output (a, b), a < b, sorted.        */
/* ------------------------------------------------------------------------- */
int64_t orc_pairs_brute(const orc_params *p, int64_t N, const double *x, const double *rad, double delta,
                        int64_t cap, int32_t *out)
{
    int64_t count = 0;
    double r[3];
    for (int64_t a = 0; a < N; ++a)
        for (int64_t b = a + 1; b < N; ++b) {
            orc_min_image(p, delta, x + 3 * a, x + 3 * b, r);
            if (pair_listed(p, r, rad[a], rad[b])) {
                if (count < cap) {
                    out[2 * count] = (int32_t)a;
                    out[2 * count + 1] = (int32_t)b;
                }
                ++count;
            }
        }
    return count;
}

/* ------------------------------------------------------------------------- */
/* Cell lattice and counting sort (Sec. 2.1, after Hoetzlein).               */
/* Lattice spacing: the largest cutoff 2 c a_max, with a 1e-9 margin so that */
/* a listed pair never spans more than one cell boundary.                    */
/* ------------------------------------------------------------------------- */
void orc_cell_dims(const orc_params *p, double a_max, int32_t *n)
{
    double rc = pair_cutoff(p, a_max, a_max) * (1.0 + 1e-9);
    for (int d = 0; d < 3; ++d) {
        n[d] = (int32_t)floor(p->L[d] / rc);
        if (n[d] < 1) n[d] = 1;
    }
}

static int32_t cell_coord(double xd, double L, int32_t n)
{
    double dc = L / (double)n;
    int32_t c = (int32_t)(xd / dc);
    if (c < 0) c = 0;
    if (c > n - 1) c = n - 1;
    return c;
}

int32_t orc_cell_of(const orc_params *p, const int32_t *n, const double *x)
{
    int32_t cx = cell_coord(x[0], p->L[0], n[0]);
    int32_t cy = cell_coord(x[1], p->L[1], n[1]);
    int32_t cz = cell_coord(x[2], p->L[2], n[2]);
    return (cz * n[1] + cy) * n[0] + cx;
}

/* Counting sort: count per cell, exclusive scan, place ids in ascending id
 * order within each cell.  cell_start has n_cells + 1 entries. */
void orc_cell_sort(const orc_params *p, int64_t N, const double *x, const int32_t *n, int32_t *cell_start,
                   int32_t *order)
{
    int64_t ncell = (int64_t)n[0] * n[1] * n[2];
    int32_t *count = (int32_t *)calloc((size_t)ncell, sizeof(int32_t));
    int32_t *cell = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    for (int64_t i = 0; i < N; ++i) {
        cell[i] = orc_cell_of(p, n, x + 3 * i);
        count[cell[i]]++;
    }
    cell_start[0] = 0;
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] = cell_start[c] + count[c];
    for (int64_t c = 0; c < ncell; ++c) count[c] = 0;
    for (int64_t i = 0; i < N; ++i) {
        int32_t c = cell[i];
        order[cell_start[c] + count[c]] = (int32_t)i;
        count[c]++;
    }
    free(count);
    free(cell);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Pair set through the cell list: each particle scans the 27 surrounding
 * cells (the whole x row for rows reached across a y face, where the
 * Lees-Edwards offset moves the images) and keeps partners of larger id.
 * Same output as orc_pairs_brute.  Falls back to brute force on lattices with
 * fewer than 3 cells along a direction. */
int64_t orc_pairs_cells(const orc_params *p, int64_t N, const double *x, const double *rad, double delta,
                        int64_t cap, int32_t *out)
{
    double a_max = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (rad[i] > a_max) a_max = rad[i];
    int32_t n[3];
    orc_cell_dims(p, a_max, n);
    if (n[0] < 3 || n[1] < 3 || n[2] < 3) return orc_pairs_brute(p, N, x, rad, delta, cap, out);
    int64_t ncell = (int64_t)n[0] * n[1] * n[2];
    int32_t *cell_start = (int32_t *)malloc((size_t)(ncell + 1) * sizeof(int32_t));
    int32_t *order = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    orc_cell_sort(p, N, x, n, cell_start, order);

    /* first pass: count partners per particle; second pass: fill */
    int64_t *cnt = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int32_t *buf = NULL;
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t a = 0; a < N; ++a) {
            double r[3];
            int32_t c = orc_cell_of(p, n, x + 3 * a);
            int32_t cx = c % n[0], cy = (c / n[0]) % n[1], cz = c / (n[0] * n[1]);
            int64_t k = 0;
            int64_t base = pass ? cnt[a] : 0;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy) {
                    int32_t zz = (cz + dz + n[2]) % n[2];
                    int32_t yraw = cy + dy;
                    int crossing = (yraw < 0 || yraw >= n[1]);
                    int32_t yy = (yraw + n[1]) % n[1];
                    int32_t xlo = crossing ? 0 : cx - 1;
                    int32_t xhi = crossing ? n[0] - 1 : cx + 1;
                    for (int32_t xr = xlo; xr <= xhi; ++xr) {
                        int32_t xc = (xr + n[0]) % n[0];
                        int32_t cc = (zz * n[1] + yy) * n[0] + xc;
                        for (int32_t s = cell_start[cc]; s < cell_start[cc + 1]; ++s) {
                            int32_t b = order[s];
                            if (b <= a) continue;
                            orc_min_image(p, delta, x + 3 * a, x + 3 * b, r);
                            if (pair_listed(p, r, rad[a], rad[b])) {
                                if (pass) buf[base + k] = b;
                                ++k;
                            }
                        }
                    }
                }
            if (!pass) cnt[a] = k;
            else qsort(buf + base, (size_t)k, sizeof(int32_t), cmp_i32);
        }
        if (!pass) {
            int64_t run = 0;
            for (int64_t a = 0; a < N; ++a) {
                int64_t k = cnt[a];
                cnt[a] = run;
                run += k;
            }
            cnt[N] = run;
            buf = (int32_t *)malloc((size_t)(run > 0 ? run : 1) * sizeof(int32_t));
        }
    }
    int64_t total = cnt[N];
    for (int64_t a = 0; a < N; ++a)
        for (int64_t k = cnt[a]; k < cnt[a + 1]; ++k)
            if (k < cap) {
                out[2 * k] = (int32_t)a;
                out[2 * k + 1] = buf[k];
            }
    free(buf);
    free(cnt);
    free(order);
    free(cell_start);
    return total;
}

/* ------------------------------------------------------------------------- */
/* Lubrication resistance functions, Appendix A (g^X and g^Y table).          */
/* al = alpha = a_j / a_i; ai = a_i; s = a_i + a_j.  The "jj" and "ji"        */
/* entries are the printed transformations of the "ii" / "ij" entries,        */
/* evaluated at 1/alpha with a_i and a_i + a_j held fixed (reading R6).       */
/* ------------------------------------------------------------------------- */
static double gXA_ii(double al, double ai, double s) { (void)s; return 2.0 * ai * al * al / pow(1.0 + al, 3); }
static double gXA_jj(double al, double ai, double s) { return al * gXA_ii(1.0 / al, ai, s); }
static double gXA_ij(double al, double ai, double s) { (void)ai; return -2.0 * s * al * al / pow(1.0 + al, 4); }
static double gXA_ji(double al, double ai, double s) { return gXA_ij(1.0 / al, ai, s); }

static double gYA_ii(double al, double ai, double s)
{
    (void)s;
    return 4.0 * ai / 15.0 * al * (2.0 + al + 2.0 * al * al) / pow(1.0 + al, 3);
}
static double gYA_jj(double al, double ai, double s) { return al * gYA_ii(1.0 / al, ai, s); }
static double gYA_ij(double al, double ai, double s)
{
    (void)ai;
    return -4.0 * s / 15.0 * al * (2.0 + al + 2.0 * al * al) / pow(1.0 + al, 4);
}
static double gYA_ji(double al, double ai, double s) { return gYA_ij(1.0 / al, ai, s); }

static double gYB_ii(double al, double ai, double s)
{
    (void)s;
    return -2.0 * ai * ai / 15.0 * al * (4.0 + al) / pow(1.0 + al, 2);
}
static double gYB_jj(double al, double ai, double s) { return -al * al * gYB_ii(1.0 / al, ai, s); }
static double gYB_ij(double al, double ai, double s)
{
    (void)ai;
    return 2.0 * s * s / 15.0 * al * (4.0 + al) / pow(1.0 + al, 4);
}
static double gYB_ji(double al, double ai, double s) { return -gYB_ij(1.0 / al, ai, s); }

static double gYC_ii(double al, double ai, double s) { (void)s; return 8.0 * ai * ai * ai / 15.0 * al / (1.0 + al); }
static double gYC_jj(double al, double ai, double s) { return al * al * al * gYC_ii(1.0 / al, ai, s); }
static double gYC_ij(double al, double ai, double s)
{
    (void)ai;
    return 2.0 * s * s * s / 15.0 * al * al / pow(1.0 + al, 4);
}

static double gXG_ii(double al, double ai, double s) { (void)s; return 2.0 * ai * ai * al * al / pow(1.0 + al, 3); }
static double gXG_jj(double al, double ai, double s) { return -al * al * gXG_ii(1.0 / al, ai, s); }
static double gXG_ij(double al, double ai, double s) { (void)ai; return -2.0 * s * s * al * al / pow(1.0 + al, 5); }
static double gXG_ji(double al, double ai, double s) { return -gXG_ij(1.0 / al, ai, s); }

static double gYG_ii(double al, double ai, double s)
{
    (void)s;
    return ai * ai / 15.0 * al * (4.0 - al + 7.0 * al * al) / pow(1.0 + al, 3);
}
static double gYG_jj(double al, double ai, double s) { return -al * al * gYG_ii(1.0 / al, ai, s); }
static double gYG_ij(double al, double ai, double s)
{
    (void)ai;
    return -s * s / 15.0 * al * (4.0 - al + 7.0 * al * al) / pow(1.0 + al, 5);
}
static double gYG_ji(double al, double ai, double s) { return -gYG_ij(1.0 / al, ai, s); }

static double gYH_ii(double al, double ai, double s)
{
    (void)s;
    return 2.0 * ai * ai * ai / 15.0 * al * (2.0 - al) / pow(1.0 + al, 2);
}
static double gYH_jj(double al, double ai, double s) { return al * al * al * gYH_ii(1.0 / al, ai, s); }
static double gYH_ij(double al, double ai, double s)
{
    (void)ai;
    return s * s * s / 15.0 * al * al * (1.0 + 7.0 * al) / pow(1.0 + al, 5);
}
/* reading R5: the printed g^{Y^G_ij} here is a typo for g^{Y^H_ij} */
static double gYH_ji(double al, double ai, double s) { return gYH_ij(1.0 / al, ai, s); }

/* The scalar coefficients X = g^X / (d* + eps), Y = g^Y log(1 / (d* + eps)),
 * each multiplied by the prefactor 6 pi eta0 (reading R1). */
typedef struct {
    double XA_ii, XA_ij, XA_ji, XA_jj;
    double YA_ii, YA_ij, YA_ji, YA_jj;
    double YB_ii, YB_ij, YB_ji, YB_jj;
    double YC_ii, YC_ij, YC_jj;
    double XG_ii, XG_ij, XG_ji, XG_jj;
    double YG_ii, YG_ij, YG_ji, YG_jj;
    double YH_ii, YH_ij, YH_ji, YH_jj;
} lub_coeffs;

static void lubrication_coefficients(const orc_params *p, double ai, double aj, double h, lub_coeffs *c)
{
    double al = aj / ai;
    double s = ai + aj;
    double dstar = 2.0 * h / s;
    if (dstar < 0.0) dstar = 0.0; /* reading R7 */
    double inv = 1.0 / (dstar + p->eps_lub);
    double lg = log(1.0 / (dstar + p->eps_lub));
    double K = 6.0 * M_PI * p->eta0;
    c->XA_ii = K * gXA_ii(al, ai, s) * inv;
    c->XA_ij = K * gXA_ij(al, ai, s) * inv;
    c->XA_ji = K * gXA_ji(al, ai, s) * inv;
    c->XA_jj = K * gXA_jj(al, ai, s) * inv;
    c->YA_ii = K * gYA_ii(al, ai, s) * lg;
    c->YA_ij = K * gYA_ij(al, ai, s) * lg;
    c->YA_ji = K * gYA_ji(al, ai, s) * lg;
    c->YA_jj = K * gYA_jj(al, ai, s) * lg;
    c->YB_ii = K * gYB_ii(al, ai, s) * lg;
    c->YB_ij = K * gYB_ij(al, ai, s) * lg;
    c->YB_ji = K * gYB_ji(al, ai, s) * lg;
    c->YB_jj = K * gYB_jj(al, ai, s) * lg;
    c->YC_ii = K * gYC_ii(al, ai, s) * lg;
    c->YC_ij = K * gYC_ij(al, ai, s) * lg;
    c->YC_jj = K * gYC_jj(al, ai, s) * lg;
    c->XG_ii = K * gXG_ii(al, ai, s) * inv;
    c->XG_ij = K * gXG_ij(al, ai, s) * inv;
    c->XG_ji = K * gXG_ji(al, ai, s) * inv;
    c->XG_jj = K * gXG_jj(al, ai, s) * inv;
    c->YG_ii = K * gYG_ii(al, ai, s) * lg;
    c->YG_ij = K * gYG_ij(al, ai, s) * lg;
    c->YG_ji = K * gYG_ji(al, ai, s) * lg;
    c->YG_jj = K * gYG_jj(al, ai, s) * lg;
    c->YH_ii = K * gYH_ii(al, ai, s) * lg;
    c->YH_ij = K * gYH_ij(al, ai, s) * lg;
    c->YH_ji = K * gYH_ji(al, ai, s) * lg;
    c->YH_jj = K * gYH_jj(al, ai, s) * lg;
}

/* 3x3 building blocks of eq. (rlu): N = n n, T = I - N, Nx = (n x). */
static void set_block(double R[12][12], int bi, int bj, const double B[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) R[3 * bi + a][3 * bj + b] = B[a][b];
}

static void block_XN_YT(const double *n, double X, double Y, double B[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double N = n[a] * n[b];
            double T = (a == b ? 1.0 : 0.0) - N;
            B[a][b] = X * N + Y * T;
        }
}

static void block_Ncross(const double *n, double Y, double B[3][3])
{
    /* (n x v)_a = sum_b B_ab v_b */
    B[0][0] = 0.0;       B[0][1] = -Y * n[2]; B[0][2] = Y * n[1];
    B[1][0] = Y * n[2];  B[1][1] = 0.0;       B[1][2] = -Y * n[0];
    B[2][0] = -Y * n[1]; B[2][1] = Y * n[0];  B[2][2] = 0.0;
}

/* eq. (rlu): the 12x12 symmetric lubrication resistance, upper triangle as
 * printed, lower triangle by symmetry; the Y^C blocks act through T (R2). */
void orc_lub_matrix(const orc_params *p, double ai, double aj, double h, const double *n, double *Rflat)
{
    double (*R)[12] = (double (*)[12])Rflat;
    lub_coeffs c;
    lubrication_coefficients(p, ai, aj, h, &c);
    double B[3][3];
    memset(R, 0, 144 * sizeof(double));
    block_XN_YT(n, c.XA_ii, c.YA_ii, B); set_block(R, 0, 0, B);
    block_XN_YT(n, c.XA_ij, c.YA_ij, B); set_block(R, 0, 1, B);
    block_Ncross(n, c.YB_ii, B);         set_block(R, 0, 2, B);
    block_Ncross(n, c.YB_ji, B);         set_block(R, 0, 3, B);
    block_XN_YT(n, c.XA_jj, c.YA_jj, B); set_block(R, 1, 1, B);
    block_Ncross(n, c.YB_ij, B);         set_block(R, 1, 2, B);
    block_Ncross(n, c.YB_jj, B);         set_block(R, 1, 3, B);
    block_XN_YT(n, 0.0, c.YC_ii, B);     set_block(R, 2, 2, B);
    block_XN_YT(n, 0.0, c.YC_ij, B);     set_block(R, 2, 3, B);
    block_XN_YT(n, 0.0, c.YC_jj, B);     set_block(R, 3, 3, B);
    for (int a = 0; a < 12; ++a)
        for (int b = 0; b < a; ++b) R[a][b] = R[b][a];
}

/* The strain quantities of eq. (rlu1) for the ambient strain at height y:
 * P = E : N - Tr E / 3, Q n = 2 E n - 2 (E : N) n, n_perp = 2 n x (E n) (R3, R4). */
static void strain_terms_at(const orc_params *p, double y, const double *n, double *P, double *Qn, double *nperp)
{
    double E[3][3];
    ambient_E(p, y, E);
    double EN = 0.0, trE = E[0][0] + E[1][1] + E[2][2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) EN += E[a][b] * n[a] * n[b];
    *P = EN - trE / 3.0;
    double En[3];
    matvec3((const double (*)[3])E, n, En);
    for (int a = 0; a < 3; ++a) Qn[a] = 2.0 * En[a] - 2.0 * EN * n[a];
    cross3(n, En, nperp);
    for (int a = 0; a < 3; ++a) nperp[a] *= 2.0;
}

/* eq. (rlu1) applied to (n, n, n_perp_i, n_perp_j) (readings R3, R4): returns
 * the 12-vector (F_i, F_j, T_i, T_j) of the ambient-strain terms; column i of
 * the matrix takes the strain E_i at particle i (height yi), column j E_j (R20;
 * E_i = E_j for the simple shear). */
void orc_lub_strain_terms(const orc_params *p, double ai, double aj, double h, const double *n, double yi,
                          double yj, double *out12)
{
    lub_coeffs c;
    lubrication_coefficients(p, ai, aj, h, &c);
    double Pi, Pj, Qi[3], Qj[3], npi[3], npj[3];
    strain_terms_at(p, yi, n, &Pi, Qi, npi);
    strain_terms_at(p, yj, n, &Pj, Qj, npj);
    for (int a = 0; a < 3; ++a) {
        out12[a] = (c.XG_ii * Pi * n[a] + c.YG_ii * Qi[a]) + (c.XG_ji * Pj * n[a] + c.YG_ji * Qj[a]);
        out12[3 + a] = (c.XG_ij * Pi * n[a] + c.YG_ij * Qi[a]) + (c.XG_jj * Pj * n[a] + c.YG_jj * Qj[a]);
        out12[6 + a] = c.YH_ii * npi[a] + c.YH_ji * npj[a];
        out12[9 + a] = c.YH_ij * npi[a] + c.YH_jj * npj[a];
    }
}

/* ------------------------------------------------------------------------- */
/* One listed pair (i, j): r = x_j - x_i (nearest image), fluctuation         */
/* velocities u' = u - U_inf(x) (own wrapped position), raw angular           */
/* velocities w.  xi_old, xr_old: stored tangential and rolling stretches of */
/* this pair (zeros if none).  Output layout (67 doubles):                    */
/*   [0:3] F^L_i  [3:6] F^L_j  [6:9] T^L_i  [9:12] T^L_j                       */
/*   [12:15] F^C_i [15:18] F^C_j [18:21] T^C_i [21:24] T^C_j                   */
/*   [24:27] F^E_i [27:30] F^E_j                                              */
/*   [30:39] S^L  [39:48] S^C  [48:57] S^E   (row-major 3x3)                  */
/*   [57:60] xi_new  [60] 1 if in contact (d_ij < 0) else 0                   */
/*   [61:64] xr_new  [64:67] rolling torque on i (included in T^C_i, T^C_j)   */
/*   [67] 1 if the Coulomb cap of eq. (csi) rescaled xi_new (slip), else 0    */
/*   [68] 1 if the rolling limit rescaled xr_new, else 0                      */
/* ------------------------------------------------------------------------- */
#define ORC_PAIR_OUT 69

void orc_pair_eval(const orc_params *p, double ai, double aj, const double *r, double yi, double yj,
                   const double *upi, const double *upj, const double *wi, const double *wj, const double *xi_old,
                   const double *xr_old, double *out)
{
    memset(out, 0, ORC_PAIR_OUT * sizeof(double));
    double dist = sqrt(dot3(r, r));
    double n[3] = {r[0] / dist, r[1] / dist, r[2] / dist};
    double h = dist - ai - aj; /* surface distance d_ij */

    /* --- lubrication, eq. (hydro): F = -R_Lub . (u'_i, u'_j, w'_i, w'_j) + R'(E) . (n, n, n_perp) */
    double Wi[3], Wj[3];
    ambient_Omega(p, yi, Wi);
    ambient_Omega(p, yj, Wj);
    double V[12];
    for (int a = 0; a < 3; ++a) {
        V[a] = upi[a];
        V[3 + a] = upj[a];
        V[6 + a] = wi[a] - Wi[a];
        V[9 + a] = wj[a] - Wj[a];
    }
    double R[12][12];
    orc_lub_matrix(p, ai, aj, h, n, &R[0][0]);
    double strain[12];
    orc_lub_strain_terms(p, ai, aj, h, n, yi, yj, strain);
    double FL[12];
    for (int a = 0; a < 12; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 12; ++b) acc += R[a][b] * V[b];
        FL[a] = -acc + strain[a];
    }
    /* R18: with the electro-chemical ranges the list is longer than the
     * lubrication range; lubrication acts only inside |r| < c (a_i + a_j) */
    if (p->ec_ranges != 0.0) {
        double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        double rl = p->cutoff_factor * (ai + aj);
        if (!(r2 < rl * rl))
            for (int a = 0; a < 12; ++a) FL[a] = 0.0;
    }
    for (int a = 0; a < 12; ++a) out[a] = FL[a];

    /* true relative velocity u_j - u_i of the image pair: the ambient flow
     * difference across r is gdot r_y along x for simple shear, plus the
     * difference of the wave at the two wrapped heights (R20) */
    double du[3] = {upj[0] - upi[0] + p->shear_rate * r[1], upj[1] - upi[1], upj[2] - upi[2]};
    if (p->wave_amp != 0.0) du[0] += p->wave_amp * (sin(wave_k(p) * yj) - sin(wave_k(p) * yi));

    /* --- contact, eqs. (contact0), (csi) */
    if (h < 0.0) {
        double un = dot3(n, du);
        double Fn[3];
        for (int a = 0; a < 3; ++a) Fn[a] = p->kn * h * n[a] + p->gamma_n * un * n[a];
        double wsum[3], wxn[3];
        for (int a = 0; a < 3; ++a) wsum[a] = ai * wi[a] + aj * wj[a];
        cross3(wsum, n, wxn);
        double vt[3];
        for (int a = 0; a < 3; ++a) vt[a] = du[a] - wxn[a];
        double vtn = dot3(vt, n);
        double ut[3];
        for (int a = 0; a < 3; ++a) ut[a] = vt[a] - vtn * n[a]; /* u_t = T (...) */
        double xi[3];
        for (int a = 0; a < 3; ++a) xi[a] = xi_old[a] + ut[a] * p->dt;
        double xin = dot3(xi, n);
        for (int a = 0; a < 3; ++a) xi[a] -= xin * n[a]; /* T (xi_old + u_t dt) */
        double Ft[3] = {0.0, 0.0, 0.0};
        if (p->kt > 0.0) {
            double fn_mag = sqrt(dot3(Fn, Fn));
            double cap = p->mu * fn_mag / p->kt;
            double xim = sqrt(dot3(xi, xi));
            if (xim >= cap && xim > 0.0) {
                for (int a = 0; a < 3; ++a) xi[a] *= cap / xim;
                out[67] = 1.0;
            }
            for (int a = 0; a < 3; ++a) Ft[a] = p->kt * xi[a];
        } else {
            for (int a = 0; a < 3; ++a) xi[a] = 0.0;
        }
        double Tci[3];
        cross3(n, Ft, Tci);
        for (int a = 0; a < 3; ++a) {
            out[12 + a] = Fn[a] + Ft[a];
            out[15 + a] = -(Fn[a] + Ft[a]);
            out[18 + a] = ai * Tci[a];
            out[21 + a] = (aj / ai) * (ai * Tci[a]);
            out[57 + a] = xi[a];
        }
        out[60] = 1.0;

        /* --- rolling resistance, Appendix roll (R19) */
        if (p->kr > 0.0) {
            double aij = 2.0 * ai * aj / (ai + aj);
            double nwi[3], nwj[3];
            cross3(n, wi, nwi);
            cross3(n, wj, nwj);
            double xr[3];
            for (int a = 0; a < 3; ++a) xr[a] = xr_old[a] + aij * (nwi[a] - nwj[a]) * p->dt;
            double xrn = dot3(xr, n);
            for (int a = 0; a < 3; ++a) xr[a] -= xrn * n[a]; /* T (xi^r_old + u_r dt) */
            double fn_mag = sqrt(dot3(Fn, Fn));
            double cap = p->mu_r * fn_mag / p->kr;
            double xm = sqrt(dot3(xr, xr));
            if (xm >= cap && xm > 0.0) {
                for (int a = 0; a < 3; ++a) xr[a] *= cap / xm;
                out[68] = 1.0;
            }
            double Fr[3], Tr[3];
            for (int a = 0; a < 3; ++a) Fr[a] = p->kr * xr[a]; /* pseudo-force */
            cross3(n, Fr, Tr);
            for (int a = 0; a < 3; ++a) {
                Tr[a] *= aij;
                out[18 + a] += Tr[a];
                out[21 + a] -= Tr[a];
                out[61 + a] = xr[a];
                out[64 + a] = Tr[a];
            }
        }
    }

    /* --- electro-chemical: repulsion eq. (rep) + attraction eq. (att) */
    double abar = 2.0 * ai * aj / (ai + aj);
    int rep_on = 1, att_on = 1;
    if (p->ec_ranges != 0.0) { /* R18: each force over its own range */
        rep_on = h < repulsion_range(p);
        att_on = h < attraction_range(p);
    }
    double FR = 0.0;
    if (p->F_ER != 0.0 && rep_on) {
        if (h >= 0.0)
            FR = -p->F_ER * (abar / p->a0) * (p->lambda_D > 0.0 ? exp(-h / p->lambda_D) : 0.0);
        else
            FR = -p->F_ER * (abar / p->a0);
    }
    double FA = 0.0;
    if (p->hamaker != 0.0 && att_on) {
        double eps = p->eps_vdw * abar;
        if (h >= 0.0)
            FA = p->hamaker * abar / (12.0 * (h * h + eps * eps));
        else
            FA = p->hamaker * abar / (12.0 * eps * eps);
    }
    for (int a = 0; a < 3; ++a) {
        out[24 + a] = (FR + FA) * n[a];
        out[27 + a] = -(FR + FA) * n[a];
    }

    /* --- stresslets, eq. (stresslet): r (x) F_i, the lubrication one symmetrised */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            out[30 + 3 * a + b] = 0.5 * (r[a] * FL[b] + r[b] * FL[a]);
            out[39 + 3 * a + b] = r[a] * out[12 + b];
            out[48 + 3 * a + b] = r[a] * out[24 + b];
        }
}

/* ------------------------------------------------------------------------- */
/* History lookup: the map {(a, b), a < b} -> xi, stored as arrays sorted by  */
/* (a, b); xi is oriented for the ordered pair (a, b).                        */
/* ------------------------------------------------------------------------- */
static int cmp_pair(const void *k, const void *e)
{
    const int32_t *x = (const int32_t *)k, *y = (const int32_t *)e;
    if (x[0] != y[0]) return (x[0] > y[0]) - (x[0] < y[0]);
    return (x[1] > y[1]) - (x[1] < y[1]);
}

/* Index of the entry (a, b) in the sorted history, or -1. */
static int64_t history_find(int64_t nh, const int32_t *hpair, int32_t a, int32_t b)
{
    if (nh <= 0) return -1;
    int32_t key[2] = {a, b};
    const int32_t *hit = (const int32_t *)bsearch(key, hpair, (size_t)nh, 2 * sizeof(int32_t), cmp_pair);
    if (!hit) return -1;
    return (int64_t)((hit - hpair) / 2);
}

/* ------------------------------------------------------------------------- */
/* Forces, torques and bulk stress at one state, eqs. (NErhs), (hydro),       */
/* (rst), (contact0), (csi), (rep), (att), (stress).  u, w: the velocities    */
/* the forces are evaluated with (the half-step ones in the integrator).      */
/* step: time index of the state (sets the Lees-Edwards offset).              */
/* Returns the number of listed pairs, or -1 if a capacity was too small.     */
/* ------------------------------------------------------------------------- */
/* hcap_new (nullable): per new history entry, bit 0 set when the Coulomb cap   */
/* rescaled its stretch at this evaluation, bit 1 when the rolling limit did  */
/* (the stick/slip state of the contact, part of the run's branch).           */
/* ------------------------------------------------------------------------- */
int64_t orc_forces_ex(const orc_params *p, int64_t N, const double *x, const double *u, const double *w,
                      const double *rad, int64_t step, int use_cells, int64_t nh_old, const int32_t *hpair_old,
                      const double *hxi_old, const double *hxr_old, int64_t hcap, int32_t *hpair_new,
                      double *hxi_new, double *hxr_new, int32_t *hcap_new, int64_t *nh_new, double *F, double *T,
                      double *Sigma)
{
    double delta = orc_le_offset(p, step);
    int64_t cap = 16 * N + 16;
    int32_t *pairs = NULL;
    int64_t np = 0;
    for (;;) {
        pairs = (int32_t *)malloc((size_t)(2 * cap) * sizeof(int32_t));
        np = use_cells ? orc_pairs_cells(p, N, x, rad, delta, cap, pairs)
                       : orc_pairs_brute(p, N, x, rad, delta, cap, pairs);
        if (np <= cap) break;
        free(pairs);
        cap = np;
    }
    double *res = (double *)malloc((size_t)(np > 0 ? np : 1) * ORC_PAIR_OUT * sizeof(double));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < np; ++k) {
        int32_t a = pairs[2 * k], b = pairs[2 * k + 1];
        double r[3], Ua[3], Ub[3], upa[3], upb[3];
        orc_min_image(p, delta, x + 3 * a, x + 3 * b, r);
        ambient_U(p, x + 3 * a, Ua);
        ambient_U(p, x + 3 * b, Ub);
        for (int c = 0; c < 3; ++c) {
            upa[c] = u[3 * a + c] - Ua[c];
            upb[c] = u[3 * b + c] - Ub[c];
        }
        int64_t e = history_find(nh_old, hpair_old, a, b);
        double zero[3] = {0.0, 0.0, 0.0};
        orc_pair_eval(p, rad[a], rad[b], r, x[3 * a + 1], x[3 * b + 1], upa, upb, w + 3 * a, w + 3 * b,
                      e >= 0 ? hxi_old + 3 * e : zero,
                      (e >= 0 && hxr_old) ? hxr_old + 3 * e : zero, res + (size_t)k * ORC_PAIR_OUT);
    }

    /* per-particle terms: Stokes drag and torque, eq. (rst), with the Faxen
     * Laplacian of the wave (zero for the simple shear, R20) */
    for (int64_t i = 0; i < N; ++i) {
        double U[3], W[3];
        ambient_U(p, x + 3 * i, U);
        ambient_Omega(p, x[3 * i + 1], W);
        double a = rad[i];
        if (p->wave_amp != 0.0) U[0] += a * a / 6.0 * lap_Ux(p, x[3 * i + 1]);
        for (int c = 0; c < 3; ++c) {
            F[3 * i + c] = -6.0 * M_PI * p->eta0 * a * (u[3 * i + c] - U[c]);
            T[3 * i + c] = -8.0 * M_PI * p->eta0 * a * a * a * (w[3 * i + c] - W[c]);
        }
    }
    /* pair sums, eq. (NErhs) */
    double S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int64_t nh = 0;
    int overflow = 0;
    for (int64_t k = 0; k < np; ++k) {
        int32_t a = pairs[2 * k], b = pairs[2 * k + 1];
        const double *o = res + (size_t)k * ORC_PAIR_OUT;
        for (int c = 0; c < 3; ++c) {
            F[3 * a + c] += o[0 + c] + o[12 + c] + o[24 + c];
            F[3 * b + c] += o[3 + c] + o[15 + c] + o[27 + c];
            T[3 * a + c] += o[6 + c] + o[18 + c];
            T[3 * b + c] += o[9 + c] + o[21 + c];
        }
        for (int c = 0; c < 9; ++c) S[c] += o[30 + c] + o[39 + c] + o[48 + c];
        if (o[60] != 0.0) {
            if (nh < hcap) {
                hpair_new[2 * nh] = a;
                hpair_new[2 * nh + 1] = b;
                for (int c = 0; c < 3; ++c) hxi_new[3 * nh + c] = o[57 + c];
                if (hxr_new)
                    for (int c = 0; c < 3; ++c) hxr_new[3 * nh + c] = o[61 + c];
                if (hcap_new) hcap_new[nh] = (o[67] != 0.0 ? 1 : 0) | (o[68] != 0.0 ? 2 : 0);
            } else {
                overflow = 1;
            }
            ++nh;
        }
    }
    *nh_new = nh;
    /* bulk stress, eq. (stress): 2 eta0 <E> + (1/V)(sum_i S^S_i + sum_pairs S);
     * <E> the box average of the ambient strain (gdot/2: the wave averages out) */
    double E[3][3];
    memset(E, 0, sizeof(E));
    E[0][1] = E[1][0] = 0.5 * p->shear_rate;
    double V = p->L[0] * p->L[1] * p->L[2];
    double SSxy = 0.0; /* sum_i 20/3 pi eta0 a^3 (1 + a^2/10 lap) E_i, xy component */
    double sum_a3 = 0.0;
    for (int64_t i = 0; i < N; ++i) sum_a3 += rad[i] * rad[i] * rad[i];
    if (p->wave_amp != 0.0)
        for (int64_t i = 0; i < N; ++i) {
            double a = rad[i], y = x[3 * i + 1];
            SSxy += 20.0 / 3.0 * M_PI * p->eta0 * a * a * a * (0.5 * shear_at(p, y) + a * a / 10.0 * lap_Exy(p, y));
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double SS = 20.0 / 3.0 * M_PI * p->eta0 * sum_a3 * E[a][b];
            if (p->wave_amp != 0.0) SS = ((a == 0 && b == 1) || (a == 1 && b == 0)) ? SSxy : 0.0;
            Sigma[3 * a + b] = 2.0 * p->eta0 * E[a][b] + (SS + S[3 * a + b]) / V;
        }
    free(res);
    free(pairs);
    return overflow ? -1 : np;
}

/* orc_forces_ex without the stick/slip record. */
int64_t orc_forces(const orc_params *p, int64_t N, const double *x, const double *u, const double *w,
                   const double *rad, int64_t step, int use_cells, int64_t nh_old, const int32_t *hpair_old,
                   const double *hxi_old, const double *hxr_old, int64_t hcap, int32_t *hpair_new,
                   double *hxi_new, double *hxr_new, int64_t *nh_new, double *F, double *T, double *Sigma)
{
    return orc_forces_ex(p, N, x, u, w, rad, step, use_cells, nh_old, hpair_old, hxi_old, hxr_old, hcap, hpair_new,
                         hxi_new, hxr_new, NULL, nh_new, F, T, Sigma);
}

/* ------------------------------------------------------------------------- */
/* Modified velocity-Verlet (Sec. 2.1, numerical algorithm), drift part:      */
/*   x^{n+1} = x^n + dt u^n + dt^2/2 alpha^n,  u^{n+1/2} = u^n + dt/2 alpha^n */
/* followed by the Lees-Edwards wrap at t_{n+1}; u^n receives the same shift. */
/* ------------------------------------------------------------------------- */
void orc_kick_drift(const orc_params *p, int64_t N, int64_t step_next, double *x, double *u, double *w,
                    const double *alpha, const double *alpha_w, double *uh, double *wh)
{
    double dt = p->dt;
    double delta = orc_le_offset(p, step_next);
    for (int64_t i = 0; i < N; ++i) {
        for (int c = 0; c < 3; ++c) {
            double xn = x[3 * i + c] + dt * u[3 * i + c] + 0.5 * dt * dt * alpha[3 * i + c];
            uh[3 * i + c] = u[3 * i + c] + 0.5 * dt * alpha[3 * i + c];
            wh[3 * i + c] = w[3 * i + c] + 0.5 * dt * alpha_w[3 * i + c];
            x[3 * i + c] = xn;
        }
        le_wrap(p, delta, x + 3 * i, u + 3 * i, uh + 3 * i);
    }
}

/* u^{n+1} = u^n + dt/2 (alpha^n + alpha^{n+1}); alpha = F/m, alpha_w = T/I. */
void orc_finish(const orc_params *p, int64_t N, const double *rad, const double *F, const double *T, double *u,
                double *w, double *alpha, double *alpha_w)
{
    double dt = p->dt;
    for (int64_t i = 0; i < N; ++i) {
        double m = orc_particle_mass(p, rad[i]);
        double I = orc_particle_inertia(p, rad[i]);
        for (int c = 0; c < 3; ++c) {
            double an = F[3 * i + c] / m;
            double awn = T[3 * i + c] / I;
            u[3 * i + c] = u[3 * i + c] + 0.5 * dt * (alpha[3 * i + c] + an);
            w[3 * i + c] = w[3 * i + c] + 0.5 * dt * (alpha_w[3 * i + c] + awn);
            alpha[3 * i + c] = an;
            alpha_w[3 * i + c] = awn;
        }
    }
}

/* alpha = F/m, alpha_w = T/I (initial accelerations). */
void orc_accelerations(const orc_params *p, int64_t N, const double *rad, const double *F, const double *T,
                       double *alpha, double *alpha_w)
{
    for (int64_t i = 0; i < N; ++i) {
        double m = orc_particle_mass(p, rad[i]);
        double I = orc_particle_inertia(p, rad[i]);
        for (int c = 0; c < 3; ++c) {
            alpha[3 * i + c] = F[3 * i + c] / m;
            alpha_w[3 * i + c] = T[3 * i + c] / I;
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
