// CPU harness for the pair VJP of the HIP library (built by test_pair_vjp_cpu.py with g++).
// in: gd, r[3], ai, aj, yi, yj, ui[3], uj[3], wi[3], wj[3], xo[3], mu, fer, xro[3]  (28 values)
// cst: k6, kn, kt, gn, a0, lamd, ham, eps_vdw, eps_lub, dt,
//      ec, cf, rep_rng, att_rng, roll, kr, mu_r                                    (17 values)
// bar: Fi, Ti, Tj, xi (12), S (9), xr (3)                                          (24 values)
// grad: r[3], yi, yj, ui[3], uj[3], wi[3], wj[3], xo[3], mu, fer, xro[3]           (25 values)
// val: Fi, Ti, Tj, xi, S, contact, capped, xr, rolling capped                     (27 values)
#include "pair_vjp.hpp"

extern "C" void pair_vjp_host(const double *in, const double *cst, const double *bar, double *grad, double *val)
{
    dss::PairConst C;
    C.k6 = cst[0]; C.kn = cst[1]; C.kt = cst[2]; C.gn = cst[3]; C.a0 = cst[4]; C.lamd = cst[5];
    C.ham = cst[6]; C.eps_vdw = cst[7]; C.eps_lub = cst[8]; C.dt = cst[9];
    C.ec = cst[10] != 0.0 ? 1 : 0; C.cf = cst[11]; C.rep_rng = cst[12]; C.att_rng = cst[13];
    C.roll = cst[14] != 0.0 ? 1 : 0; C.kr = cst[15]; C.mu_r = cst[16];
    C.mu = in[23];
    C.fer = in[24];
    dss::PairBar b;
    for (int k = 0; k < 3; ++k) {
        b.Fi[k] = bar[k];
        b.Ti[k] = bar[3 + k];
        b.Tj[k] = bar[6 + k];
        b.xi[k] = bar[9 + k];
    }
    for (int k = 0; k < 9; ++k) b.S[k] = bar[12 + k];
    for (int k = 0; k < 3; ++k) b.xr[k] = bar[21 + k];
    dss::PairGrad g = {};
    dss::PairVal v;
    dss::pair_vjp(C, in[0], in + 1, in[4], in[5], in[6], in[7], in + 8, in + 11, in + 14, in + 17, in + 20, b, g, &v, -1,
                  -1, in + 25);
    double *o = grad;
    for (int k = 0; k < 3; ++k) *o++ = g.r[k];
    *o++ = g.yi;
    *o++ = g.yj;
    for (int k = 0; k < 3; ++k) *o++ = g.ui[k];
    for (int k = 0; k < 3; ++k) *o++ = g.uj[k];
    for (int k = 0; k < 3; ++k) *o++ = g.wi[k];
    for (int k = 0; k < 3; ++k) *o++ = g.wj[k];
    for (int k = 0; k < 3; ++k) *o++ = g.xo[k];
    *o++ = g.mu;
    *o++ = g.fer;
    for (int k = 0; k < 3; ++k) *o++ = g.xro[k];
    o = val;
    for (int k = 0; k < 3; ++k) *o++ = v.Fi[k];
    for (int k = 0; k < 3; ++k) *o++ = v.Ti[k];
    for (int k = 0; k < 3; ++k) *o++ = v.Tj[k];
    for (int k = 0; k < 3; ++k) *o++ = v.xi[k];
    for (int k = 0; k < 9; ++k) *o++ = v.S[k];
    *o++ = v.contact ? 1.0 : 0.0;
    *o++ = v.capped ? 1.0 : 0.0;
    for (int k = 0; k < 3; ++k) *o++ = v.xr[k];
    *o++ = v.rcapped ? 1.0 : 0.0;
}
