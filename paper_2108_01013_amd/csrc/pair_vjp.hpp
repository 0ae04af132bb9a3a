// pair_vjp.hpp -- reverse-mode derivative of the FP64 pair physics of one listed pair.
//
// The pair function maps (r = x_j - x_i, y_i, y_j, u_i, u_j, w_i, w_j, xi_old; mu, F_ER) to
// (F_i, T_i, T_j, xi_new, S): lubrication in the reduced form of the resistance matrices of
// Appendix A, repulsion (eq. rep), attraction (eq. att), the spring-dashpot contact with its
// tangential stretch and Coulomb cap (eqs. contact0, csi), and the pair stresslet (eq.
// stresslet); F_j = -F_i.  pair_vjp recomputes the primal with the forward's formulas and
// branch decisions (listed pair, contact h < 0, Coulomb cap active, h >= 0 for the
// electro-chemical terms, d* > 0), then pulls a cotangent of the outputs back to every
// input: the vector-Jacobian product of the branch that the primal takes.  Plain C++ with
// a host/device qualifier, so the same code is differentiated numerically on the CPU.
#pragma once

#include <cmath>

#ifdef __HIPCC__
#define DSS_HD __host__ __device__
#else
#define DSS_HD
#endif

namespace dss {

// Constants the pair function reads (eta0 through k6 = 6 pi eta0).
struct PairConst {
    double k6, kn, kt, gn, mu, fer, a0, lamd, ham, eps_vdw, eps_lub, dt;
    // electro-chemical ranges (reading R18): lubrication only for |r| < cf (a_i + a_j),
    // repulsion for h < rep_rng, attraction for h < att_rng; ec = 0 keeps every term on
    int ec = 0;
    double cf = 0.0, rep_rng = 0.0, att_rng = 0.0;
    // rolling resistance (reading R19): a spring k_r on u_r = abar n x (w_i - w_j) with the
    // Coulomb limit mu_r |F_nor| / k_r, torques T_i = abar n x k_r xi^r = -T_j; roll = 0: none
    int roll = 0;
    double kr = 0.0, mu_r = 0.0;
};

// Cotangents of the outputs.  S: 9 weights of the pair's stresslet entries S_ab.
struct PairBar {
    double Fi[3], Ti[3], Tj[3], xi[3], S[9];
    double xr[3] = {0.0, 0.0, 0.0};   // of the new rolling stretch
};

// Gradients with respect to the inputs.
struct PairGrad {
    double r[3], yi, yj, ui[3], uj[3], wi[3], wj[3], xo[3], mu, fer;
    double xro[3];                    // of the stored rolling stretch
};

// Primal outputs (for checks against the forward).
struct PairVal {
    double Fi[3], Ti[3], Tj[3], xi[3], S[9];
    bool contact, capped;
    double xr[3];
    bool rcapped;                     // the rolling stretch was limited
};

DSS_HD inline double vdot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

DSS_HD inline void vcross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// out += s * a
DSS_HD inline void vaxpy(double s, const double a[3], double out[3])
{
    out[0] += s * a[0];
    out[1] += s * a[1];
    out[2] += s * a[2];
}

// g must be zero on entry; val may be null.  force_contact / force_capped / force_rcapped: the
// branch to differentiate (0 or 1, as decided by the forward run: contact, Coulomb cap, rolling
// limit), or -1 to decide it here.
DSS_HD inline void pair_vjp(const PairConst &C, double gd, const double r[3], double ai, double aj, double yi,
                            double yj, const double ui[3], const double uj[3], const double Wi[3], const double Wj[3],
                            const double xo[3], const PairBar &bar, PairGrad &g, PairVal *val,
                            int force_contact = -1, int force_capped = -1, const double *xro = nullptr,
                            int force_rcapped = -1)
{
    // ------------------------------------------------------------------ primal
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double dist = sqrt(r2);
    const double h = dist - ai - aj;
    const double s = ai + aj;
    const double dsr = 2.0 * h / s;
    const bool dpos = dsr > 0.0;
    const double gg = (dpos ? dsr : 0.0) + C.eps_lub;
    // the gates are piecewise constant: a term switched off has no value and no gradient
    const double rl = C.cf * s;
    const bool lub_on = !C.ec || r2 < rl * rl;
    const bool rep_on = !C.ec || h < C.rep_rng;
    const bool att_on = !C.ec || h < C.att_rng;
    const double invg = lub_on ? 1.0 / gg : 0.0;
    const double lg = lub_on ? -log(gg) : 0.0;
    const double dux = (uj[0] - gd * yj) - (ui[0] - gd * yi);
    const double duy = uj[1] - ui[1], duz = uj[2] - ui[2];
    const double inv_d = 1.0 / dist;
    const double n[3] = {r[0] * inv_d, r[1] * inv_d, r[2] * inv_d};
    const double wi[3] = {Wi[0], Wi[1], Wi[2] + 0.5 * gd};
    const double wj[3] = {Wj[0], Wj[1], Wj[2] + 0.5 * gd};
    const double K = C.k6;
    const double ai2 = ai * ai, aj2 = aj * aj;
    const double is = 1.0 / s, is2 = is * is, is3 = is2 * is;
    const double cXA = K * 2.0 * ai2 * aj2 * is3;
    const double cYA = K * (4.0 / 15.0) * ai * aj * (2.0 * ai2 + ai * aj + 2.0 * aj2) * is3;
    const double cYBi = -K * (2.0 / 15.0) * ai2 * aj * (4.0 * ai + aj) * is2;
    const double cYBj = K * (2.0 / 15.0) * ai * aj2 * (ai + 4.0 * aj) * is2;
    const double cYCii = K * (8.0 / 15.0) * ai2 * ai * aj * is;
    const double cYCij = K * (2.0 / 15.0) * ai2 * aj2 * is;
    const double cYCjj = K * (8.0 / 15.0) * ai * aj2 * aj * is;
    const double XA = cXA * invg, YA = cYA * lg, YBi = cYBi * lg, YBj = cYBj * lg;
    const double YCii = cYCii * lg, YCij = cYCij * lg, YCjj = cYCjj * lg;
    const double v[3] = {dux + s * 0.5 * gd * n[1], duy + s * 0.5 * gd * n[0], duz};
    const double vn = vdot(v, n);
    double ci[3], cj[3], nv[3];
    vcross(n, wi, ci);
    vcross(n, wj, cj);
    vcross(n, v, nv);
    double FL[3];
    for (int k = 0; k < 3; ++k) FL[k] = XA * vn * n[k] + YA * (v[k] - vn * n[k]) - YBi * ci[k] + YBj * cj[k];
    const double win = vdot(wi, n), wjn = vdot(wj, n);
    double ti[3], tj[3], Ti[3], Tj[3];
    for (int k = 0; k < 3; ++k) {
        ti[k] = wi[k] - win * n[k];
        tj[k] = wj[k] - wjn * n[k];
        Ti[k] = -YBi * nv[k] - YCii * ti[k] - YCij * tj[k];
        Tj[k] = YBj * nv[k] - YCij * ti[k] - YCjj * tj[k];
    }
    const double abar = 2.0 * ai * aj * is;
    const double E = h >= 0.0 ? (C.lamd > 0.0 ? exp(-h / C.lamd) : 0.0) : 1.0;
    double fe = 0.0;
    if (C.fer != 0.0 && rep_on) fe -= (C.fer / C.a0) * abar * E;
    const double ev = C.eps_vdw * abar;
    const double Q = (h >= 0.0 ? h * h : 0.0) + ev * ev;
    if (C.ham != 0.0 && att_on) fe += C.ham * abar / (12.0 * Q);
    const bool contact = force_contact >= 0 ? force_contact != 0 : h < 0.0;
    double FC[3] = {0.0, 0.0, 0.0}, Ft[3] = {0.0, 0.0, 0.0}, xpp[3] = {0.0, 0.0, 0.0};
    double D[3] = {0.0, 0.0, 0.0}, t[3] = {0.0, 0.0, 0.0}, sv[3] = {0.0, 0.0, 0.0}, xs[3] = {0.0, 0.0, 0.0};
    double xp[3] = {0.0, 0.0, 0.0};
    double fn = 0.0, tn = 0.0, xsn = 0.0, cap = 0.0, xm = 0.0, sc = 1.0;
    bool capped = false;
    // rolling spring: angular velocity difference, u_r / abar, unprojected and projected
    // stretch, capped stretch, its spring force and n x force
    double dwr[3] = {0.0, 0.0, 0.0}, urr[3] = {0.0, 0.0, 0.0}, qrr[3] = {0.0, 0.0, 0.0}, prr[3] = {0.0, 0.0, 0.0};
    double xrr[3] = {0.0, 0.0, 0.0}, frr[3] = {0.0, 0.0, 0.0}, qtr[3] = {0.0, 0.0, 0.0};
    double qrn = 0.0, capr = 0.0, prm = 0.0, rsc = 1.0;
    bool rcapped = false;
    if (contact) {
        D[0] = dux + gd * r[1];
        D[1] = duy;
        D[2] = duz;
        const double un = vdot(D, n);
        fn = C.kn * h + C.gn * un;
        for (int k = 0; k < 3; ++k) sv[k] = ai * Wi[k] + aj * Wj[k];
        double q[3];
        vcross(sv, n, q);
        for (int k = 0; k < 3; ++k) t[k] = D[k] - q[k];
        tn = vdot(t, n);
        for (int k = 0; k < 3; ++k) xs[k] = xo[k] + (t[k] - tn * n[k]) * C.dt;
        xsn = vdot(xs, n);
        for (int k = 0; k < 3; ++k) xp[k] = xs[k] - xsn * n[k];
        if (C.kt > 0.0) {
            cap = C.mu * fabs(fn) / C.kt;
            xm = sqrt(vdot(xp, xp));
            capped = (force_capped >= 0 ? force_capped != 0 : xm >= cap) && xm > 0.0;
            sc = capped ? cap / xm : 1.0;
            for (int k = 0; k < 3; ++k) {
                xpp[k] = xp[k] * sc;
                Ft[k] = C.kt * xpp[k];
            }
        }
        double m[3];
        vcross(n, Ft, m);
        for (int k = 0; k < 3; ++k) {
            FC[k] = fn * n[k] + Ft[k];
            Ti[k] += ai * m[k];
            Tj[k] += aj * m[k];
        }
        if (C.roll) {
            // xi^r' = P_n(xi^r_old + u_r dt), capped at mu_r |fn| / k_r; T_i += abar n x k_r xi^r'
            for (int k = 0; k < 3; ++k) dwr[k] = Wi[k] - Wj[k];
            vcross(n, dwr, urr);
            for (int k = 0; k < 3; ++k) qrr[k] = (xro ? xro[k] : 0.0) + abar * urr[k] * C.dt;
            qrn = vdot(qrr, n);
            for (int k = 0; k < 3; ++k) prr[k] = qrr[k] - qrn * n[k];
            capr = C.mu_r * fabs(fn) / C.kr;
            prm = sqrt(vdot(prr, prr));
            rcapped = (force_rcapped >= 0 ? force_rcapped != 0 : prm >= capr) && prm > 0.0;
            rsc = rcapped ? capr / prm : 1.0;
            for (int k = 0; k < 3; ++k) {
                xrr[k] = rsc * prr[k];
                frr[k] = C.kr * xrr[k];
            }
            vcross(n, frr, qtr);
            for (int k = 0; k < 3; ++k) {
                Ti[k] += abar * qtr[k];
                Tj[k] -= abar * qtr[k];
            }
        }
    }
    double FO[3];
    for (int k = 0; k < 3; ++k) FO[k] = FC[k] + fe * n[k];
    if (val) {
        for (int k = 0; k < 3; ++k) {
            val->Fi[k] = FL[k] + FO[k];
            val->Ti[k] = Ti[k];
            val->Tj[k] = Tj[k];
            val->xi[k] = xpp[k];
            val->xr[k] = xrr[k];
            val->rcapped = rcapped;
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) val->S[3 * a + b] = 0.5 * (r[a] * FL[b] + r[b] * FL[a]) + r[a] * FO[b];
        val->contact = contact;
        val->capped = capped;
    }

    // ------------------------------------------------------------------ reverse
    double rb[3] = {0.0, 0.0, 0.0}, nb[3] = {0.0, 0.0, 0.0};
    double hb = 0.0, duxb = 0.0, duyb = 0.0, duzb = 0.0;
    double wib[3] = {0.0, 0.0, 0.0}, wjb[3] = {0.0, 0.0, 0.0};
    // stresslet S_ab = (r_a FL_b + r_b FL_a) / 2 + r_a FO_b, F_i = FL + FO
    double FLb[3], FOb[3];
    for (int b = 0; b < 3; ++b) {
        FLb[b] = bar.Fi[b];
        FOb[b] = bar.Fi[b];
        for (int a = 0; a < 3; ++a) {
            FLb[b] += 0.5 * (bar.S[3 * a + b] + bar.S[3 * b + a]) * r[a];
            FOb[b] += bar.S[3 * a + b] * r[a];
        }
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) rb[a] += 0.5 * (bar.S[3 * a + b] + bar.S[3 * b + a]) * FL[b] + bar.S[3 * a + b] * FO[b];
    // FO = FC + fe n
    const double feb = vdot(FOb, n);
    vaxpy(fe, FOb, nb);
    if (C.fer != 0.0 && rep_on) {
        g.fer += -(abar / C.a0) * E * feb;
        if (h >= 0.0 && C.lamd > 0.0) hb += (C.fer / C.a0) * abar * E * feb / C.lamd;
    }
    if (C.ham != 0.0 && att_on && h >= 0.0) hb += -C.ham * abar * 2.0 * h / (12.0 * Q * Q) * feb;
    double Tib[3] = {bar.Ti[0], bar.Ti[1], bar.Ti[2]}, Tjb[3] = {bar.Tj[0], bar.Tj[1], bar.Tj[2]};
    if (contact) {
        // m = n x Ft feeds T_i += a_i m, T_j += a_j m
        double mb[3], tmp[3];
        for (int k = 0; k < 3; ++k) mb[k] = ai * Tib[k] + aj * Tjb[k];
        double Ftb[3];
        vcross(Ft, mb, tmp);
        vaxpy(1.0, tmp, nb);
        vcross(mb, n, Ftb);
        // FC = fn n + Ft
        for (int k = 0; k < 3; ++k) Ftb[k] += FOb[k];
        double fnb = vdot(FOb, n);
        vaxpy(fn, FOb, nb);
        if (C.roll) {
            // T_i += abar qt, T_j -= abar qt, qt = n x fr, fr = k_r xr
            double qtb[3], frb[3], xrb[3], prb[3], qb2[3], urb[3], dwb[3], t2[3];
            for (int k = 0; k < 3; ++k) qtb[k] = abar * (Tib[k] - Tjb[k]);
            vcross(frr, qtb, t2);
            vaxpy(1.0, t2, nb);
            vcross(qtb, n, frb);
            for (int k = 0; k < 3; ++k) xrb[k] = C.kr * frb[k] + bar.xr[k];
            // xr = rsc p, rsc = capr / |p| when capped, capr = mu_r |fn| / k_r
            if (rcapped) {
                const double sb = vdot(xrb, prr);
                const double caprb = sb / prm;
                const double prmb = -sb * capr / (prm * prm);
                for (int k = 0; k < 3; ++k) prb[k] = rsc * xrb[k] + prmb * prr[k] / prm;
                fnb += (fn > 0.0 ? 1.0 : (fn < 0.0 ? -1.0 : 0.0)) * C.mu_r / C.kr * caprb;
            } else {
                for (int k = 0; k < 3; ++k) prb[k] = xrb[k];
            }
            // p = q - (q.n) n
            const double pbn = vdot(prb, n);
            for (int k = 0; k < 3; ++k) {
                qb2[k] = prb[k] - pbn * n[k];
                nb[k] += -pbn * qrr[k] - qrn * prb[k];
            }
            // q = xro + abar (n x dw) dt
            for (int k = 0; k < 3; ++k) {
                g.xro[k] += qb2[k];
                urb[k] = abar * C.dt * qb2[k];
            }
            vcross(dwr, urb, t2);
            vaxpy(1.0, t2, nb);
            vcross(urb, n, dwb);
            for (int k = 0; k < 3; ++k) {
                g.wi[k] += dwb[k];
                g.wj[k] -= dwb[k];
            }
        }
        double xpb[3] = {0.0, 0.0, 0.0};
        if (C.kt > 0.0) {
            double xppb[3];
            for (int k = 0; k < 3; ++k) xppb[k] = C.kt * Ftb[k] + bar.xi[k];
            if (capped) {
                // xpp = xp cap / |xp|, cap = mu |fn| / kt
                const double scb = vdot(xppb, xp);
                const double capb = scb / xm;
                const double xmb = -scb * cap / (xm * xm);
                for (int k = 0; k < 3; ++k) xpb[k] = sc * xppb[k] + xmb * xp[k] / xm;
                g.mu += fabs(fn) / C.kt * capb;
                fnb += (fn > 0.0 ? 1.0 : (fn < 0.0 ? -1.0 : 0.0)) * C.mu / C.kt * capb;
            } else {
                for (int k = 0; k < 3; ++k) xpb[k] = xppb[k];
            }
        }
        // xp = xs - (xs.n) n
        const double xpn = vdot(xpb, n);
        double xsb[3];
        for (int k = 0; k < 3; ++k) {
            xsb[k] = xpb[k] - xpn * n[k];
            nb[k] += -xpn * xs[k] - xsn * xpb[k];
        }
        // xs = xo + (t - (t.n) n) dt
        for (int k = 0; k < 3; ++k) g.xo[k] += xsb[k];
        double yb[3] = {C.dt * xsb[0], C.dt * xsb[1], C.dt * xsb[2]};
        const double ybn = vdot(yb, n);
        double tb[3];
        for (int k = 0; k < 3; ++k) {
            tb[k] = yb[k] - ybn * n[k];
            nb[k] += -ybn * t[k] - tn * yb[k];
        }
        // t = D - q, q = sv x n, sv = a_i w_i + a_j w_j
        double Db[3] = {tb[0], tb[1], tb[2]};
        const double qb[3] = {-tb[0], -tb[1], -tb[2]};
        double svb[3];
        vcross(n, qb, svb);
        vcross(qb, sv, tmp);
        vaxpy(1.0, tmp, nb);
        for (int k = 0; k < 3; ++k) {
            g.wi[k] += ai * svb[k];
            g.wj[k] += aj * svb[k];
        }
        // fn = kn h + gn (D.n)
        hb += C.kn * fnb;
        const double unb = C.gn * fnb;
        vaxpy(unb, n, Db);
        vaxpy(unb, D, nb);
        // D = (dux + gd r_y, duy, duz)
        duxb += Db[0];
        rb[1] += gd * Db[0];
        duyb += Db[1];
        duzb += Db[2];
    }
    // lubrication torques
    {
        double nvb[3], tib[3], tjb[3];
        for (int k = 0; k < 3; ++k) {
            nvb[k] = -YBi * Tib[k] + YBj * Tjb[k];
            tib[k] = -YCii * Tib[k] - YCij * Tjb[k];
            tjb[k] = -YCij * Tib[k] - YCjj * Tjb[k];
        }
        double YBib = -vdot(Tib, nv), YBjb = vdot(Tjb, nv);
        const double YCiib = -vdot(Tib, ti), YCijb = -(vdot(Tib, tj) + vdot(Tjb, ti)), YCjjb = -vdot(Tjb, tj);
        // ti = wi - (wi.n) n
        const double tin = vdot(tib, n), tjn = vdot(tjb, n);
        for (int k = 0; k < 3; ++k) {
            wib[k] += tib[k] - tin * n[k];
            wjb[k] += tjb[k] - tjn * n[k];
            nb[k] += -tin * wi[k] - win * tib[k] - tjn * wj[k] - wjn * tjb[k];
        }
        // nv = n x v
        double vb[3], tmp[3];
        vcross(v, nvb, tmp);
        vaxpy(1.0, tmp, nb);
        vcross(nvb, n, vb);
        // FL = XA vn n + YA (v - vn n) - YBi ci + YBj cj
        const double FLn = vdot(FLb, n);
        const double XAb = vn * FLn;
        const double YAb = vdot(FLb, v) - vn * FLn;
        YBib += -vdot(FLb, ci);
        YBjb += vdot(FLb, cj);
        const double vnb = (XA - YA) * FLn;
        vaxpy((XA - YA) * vn, FLb, nb);
        vaxpy(YA, FLb, vb);
        double cib[3], cjb[3];
        for (int k = 0; k < 3; ++k) {
            cib[k] = -YBi * FLb[k];
            cjb[k] = YBj * FLb[k];
        }
        // c = n x w
        vcross(wi, cib, tmp);
        vaxpy(1.0, tmp, nb);
        vcross(wj, cjb, tmp);
        vaxpy(1.0, tmp, nb);
        vcross(cib, n, tmp);
        vaxpy(1.0, tmp, wib);
        vcross(cjb, n, tmp);
        vaxpy(1.0, tmp, wjb);
        // vn = v.n
        vaxpy(vnb, n, vb);
        vaxpy(vnb, v, nb);
        // v = (dux + s gd n_y / 2, duy + s gd n_x / 2, duz)
        duxb += vb[0];
        nb[1] += 0.5 * s * gd * vb[0];
        duyb += vb[1];
        nb[0] += 0.5 * s * gd * vb[1];
        duzb += vb[2];
        // coefficients: X = c invg, Y = c lg, invg = 1 / g, lg = -log g, g = max(2h/s, 0) + eps
        const double invgb = cXA * XAb;
        const double lgb = cYA * YAb + cYBi * YBib + cYBj * YBjb + cYCii * YCiib + cYCij * YCijb + cYCjj * YCjjb;
        const double ggb = lub_on ? -invg * invg * invgb - lgb / gg : 0.0;
        if (dpos) hb += 2.0 / s * ggb;
    }
    // w' = w + (0, 0, gd / 2)
    for (int k = 0; k < 3; ++k) {
        g.wi[k] += wib[k];
        g.wj[k] += wjb[k];
    }
    // du = (u_j - gd y_j x) - (u_i - gd y_i x)
    g.uj[0] += duxb;
    g.ui[0] -= duxb;
    g.yj += -gd * duxb;
    g.yi += gd * duxb;
    g.uj[1] += duyb;
    g.ui[1] -= duyb;
    g.uj[2] += duzb;
    g.ui[2] -= duzb;
    // n = r / |r|, h = |r| - a_i - a_j
    const double nn = vdot(nb, n);
    for (int k = 0; k < 3; ++k) g.r[k] += rb[k] + (nb[k] - nn * n[k]) * inv_d + hb * n[k];
}

}  // namespace dss
