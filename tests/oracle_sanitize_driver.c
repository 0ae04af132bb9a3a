/* Drives the oracle (oracle/dss_oracle.c) through pair searches at several Lees-Edwards offsets
 * and 30 full steps with contact history, for the simple shear, the electro-chemical ranges,
 * rolling resistance and the wavy shear, on random bidisperse centres (deep overlaps included).
 * Built with AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py;
 * any report aborts the run.  The declarations repeat the oracle's exported interface. */
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
typedef struct {
    double L[3]; double shear_rate, eta0, rho, kn, kt, gamma_n, mu, F_ER, lambda_D, a0, hamaker, eps_vdw, eps_lub,
        cutoff_factor, dt, ec_ranges, kr, mu_r, wave_amp, wave_n;
} orc_params;
int orc_history_capacity(double a, double a_min);
double orc_le_offset(const orc_params *p, int64_t step);
int64_t orc_pairs_brute(const orc_params *p, int64_t N, const double *x, const double *rad, double delta, int64_t cap, int32_t *out);
int64_t orc_pairs_cells(const orc_params *p, int64_t N, const double *x, const double *rad, double delta, int64_t cap, int32_t *out);
int64_t orc_forces(const orc_params *p, int64_t N, const double *x, const double *u, const double *w, const double *rad,
                   int64_t step, int use_cells, int64_t nh_old, const int32_t *hpair_old, const double *hxi_old,
                   const double *hxr_old, int64_t hcap, int32_t *hpair_new, double *hxi_new, double *hxr_new,
                   int64_t *nh_new, double *F, double *T, double *Sigma);
void orc_kick_drift(const orc_params *p, int64_t N, int64_t step_next, double *x, double *u, double *w,
                    const double *alpha, const double *alpha_w, double *uh, double *wh);
void orc_finish(const orc_params *p, int64_t N, const double *rad, const double *F, const double *T, double *u,
                double *w, double *alpha, double *alpha_w);
void orc_accelerations(const orc_params *p, int64_t N, const double *rad, const double *F, const double *T, double *a, double *aw);

static double urand(void) { return rand() / (RAND_MAX + 1.0); }

static int run(int variant, int N)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    double L = 20.0;
    p.L[0] = p.L[1] = p.L[2] = L;
    p.shear_rate = 1.0; p.eta0 = 1.0; p.rho = 0.1; p.kn = 4e5; p.kt = 4e5 * 2.0 / 7.0; p.gamma_n = 0.04;
    p.mu = 1.0; p.F_ER = 1.0; p.lambda_D = 0.05; p.a0 = 1.0; p.eps_vdw = 0.01; p.eps_lub = 0.02;
    p.cutoff_factor = 1.1; p.dt = 1e-4;
    if (variant == 1) { p.ec_ranges = 1.0; p.hamaker = 1e-3; }
    if (variant == 2) { p.kr = 0.05 * p.kn; p.mu_r = 0.1; }
    if (variant == 3) { p.wave_amp = 20.0; p.wave_n = 1.0; }
    double *x = malloc(sizeof(double) * 3 * N), *u = calloc(3 * N, sizeof(double)), *w = calloc(3 * N, sizeof(double));
    double *rad = malloc(sizeof(double) * N), *F = malloc(sizeof(double) * 3 * N), *T = malloc(sizeof(double) * 3 * N);
    double *a = malloc(sizeof(double) * 3 * N), *aw = malloc(sizeof(double) * 3 * N);
    double *uh = malloc(sizeof(double) * 3 * N), *wh = malloc(sizeof(double) * 3 * N);
    for (int i = 0; i < N; ++i) {
        rad[i] = (i % 3 == 0) ? 1.4 : 1.0;
        for (int d = 0; d < 3; ++d) x[3 * i + d] = urand() * L;
        u[3 * i] = p.shear_rate * x[3 * i + 1];
    }
    int M = orc_history_capacity(1.4, 1.0);
    int64_t hcap = (int64_t)N * M;
    int32_t *hp[2] = {malloc(sizeof(int32_t) * 2 * hcap), malloc(sizeof(int32_t) * 2 * hcap)};
    double *hx[2] = {malloc(sizeof(double) * 3 * hcap), malloc(sizeof(double) * 3 * hcap)};
    double *hr[2] = {malloc(sizeof(double) * 3 * hcap), malloc(sizeof(double) * 3 * hcap)};
    int64_t nh = 0, nh2 = 0;
    double S[9];
    int64_t cap = 64 * (int64_t)N;
    int32_t *pb = malloc(sizeof(int32_t) * 2 * cap), *pc = malloc(sizeof(int32_t) * 2 * cap);
    for (int k = 0; k < 5; ++k) {
        double delta = k * 0.37 * L / 5;
        int64_t nb = orc_pairs_brute(&p, N, x, rad, delta, cap, pb);
        int64_t nc = orc_pairs_cells(&p, N, x, rad, delta, cap, pc);
        if (nb > cap || nb != nc || memcmp(pb, pc, sizeof(int32_t) * 2 * nb)) { printf("pair mismatch v%d k%d\n", variant, k); return 1; }
    }
    orc_forces(&p, N, x, u, w, rad, 0, 1, 0, hp[0], hx[0], hr[0], hcap, hp[1], hx[1], hr[1], &nh2, F, T, S);
    orc_accelerations(&p, N, rad, F, T, a, aw);
    int c = 0;
    for (int n = 0; n < 30; ++n) {
        orc_kick_drift(&p, N, n + 1, x, u, w, a, aw, uh, wh);
        orc_forces(&p, N, x, uh, wh, rad, n + 1, n & 1, nh, hp[c], hx[c], hr[c], hcap, hp[1 - c], hx[1 - c], hr[1 - c], &nh2, F, T, S);
        orc_finish(&p, N, rad, F, T, u, w, a, aw);
        nh = nh2;
        c = 1 - c;
    }
    printf("variant %d: N=%d contacts %lld Sxy %.6g\n", variant, N, (long long)nh, S[1]);
    free(x); free(u); free(w); free(rad); free(F); free(T); free(a); free(aw); free(uh); free(wh);
    for (int k = 0; k < 2; ++k) { free(hp[k]); free(hx[k]); free(hr[k]); }
    free(pb); free(pc);
    return 0;
}

int main(void)
{
    srand(7);
    int rc = 0;
    for (int v = 0; v < 4; ++v) rc |= run(v, 600);
    return rc;
}
