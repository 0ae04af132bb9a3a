// dss_adjoint.hpp -- kernels of the discrete adjoint of the time step.
//
// The forward step (Sec. 2.1, numerical algorithm) is, per particle,
//   uh_{n+1} = uh_n + c_n dt F_n / m     (c = 1/2 on the first step from a state u^n, else 1)
//   x_{n+1}  = x_n + dt uh_{n+1}         (the Lees-Edwards wrap shifts by constants)
//   (F, T, Sigma, xi)_{n+1} = pair and Stokes terms at (x_{n+1}, uh_{n+1}, wh_{n+1}, xi_n)
// and the same for the rotation with T / I.  With the pair set, contact states and
// Coulomb-cap states of the forward run held fixed, the reverse sweep carries the adjoints
// of x, uh, wh (by particle id) and of the contact stretches (in canonical history rows)
// backwards one step at a time.  Everything here works on the recorded run ("tape") by
// particle id: positions, half-step velocities, the listed pairs (id_min, id_max) and the
// contact history in canonical rows (row of the smaller id, sorted by partner id).
#pragma once

#include "dss_kernels.hpp"
#include "pair_vjp.hpp"

namespace dss {

// Position of contact (a < b) in canonical rows, or -1 (keys carry the cap flag in bit 30).
__device__ __forceinline__ long long canon_find(const int *__restrict__ key, const int *__restrict__ cnt, int M, int a,
                                                int b)
{
    const int n = cnt[a];
    const int *kr = key + (long long)a * M;
    for (int k = 0; k < n; ++k) {
        const int kk = kr[k] & kKeyMask;
        if (kk == b) return (long long)a * M + k;
        if (kk > b) break;
    }
    return -1;
}

// Committed history rows (slot rows with owner ids and partner keys, stretch oriented from
// the smaller to the larger id) -> canonical rows by id.  Pass 1 appends each contact to the
// row of its smaller id; pass 2 sorts every row by partner id.  ccnt must be zero on entry.
template <int sw>
__global__ void __launch_bounds__(kBlock) k_canon_fill(int N, int M, const int *__restrict__ own,
                                                       const int *__restrict__ key, const double *__restrict__ xi,
                                                       const double *__restrict__ xr, const int *__restrict__ cnt,
                                                       int *__restrict__ ckey, double *__restrict__ cxi,
                                                       int *__restrict__ ccnt, DevClock *__restrict__ clk)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int id = own[p];
    const int n = cnt[p];
    for (int k = 0; k < n; ++k) {
        const int kw = key[(long long)p * M + k];
        const int partner = kw & kKeyMask;
        const int a = id < partner ? id : partner, b = id < partner ? partner : id;
        const int s = atomicAdd(&ccnt[a], 1);
        if (s < M) {
            ckey[(long long)a * M + s] = b | (kw & (kCapBit | kRollCapBit));
            const double *x = xi + ((long long)p * M + k) * 3;
            double *y = cxi + ((long long)a * M + s) * sw;
            y[0] = x[0];
            y[1] = x[1];
            y[2] = x[2];
            if (sw == 6) {
                // the rolling stretch has no orientation: it is stored as it is
                const double *z = xr + ((long long)p * M + k) * 3;
                y[3] = z[0];
                y[4] = z[1];
                y[5] = z[2];
            }
        } else {
            atomicOr(&clk->err, kErrRowOverflow);
        }
    }
}

template <int sw>
__global__ void __launch_bounds__(kBlock) k_canon_sort(int N, int M, int *__restrict__ ckey, double *__restrict__ cxi,
                                                       int *__restrict__ ccnt)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    int n = ccnt[a];
    n = n < M ? n : M;
    ccnt[a] = n;
    int *kr = ckey + (long long)a * M;
    double *xr = cxi + (long long)a * M * sw;
    for (int i = 1; i < n; ++i) {
        const int k = kr[i];
        double v[6];
        for (int c = 0; c < sw; ++c) v[c] = xr[sw * i + c];
        int j = i - 1;
        while (j >= 0 && (kr[j] & kKeyMask) > (k & kKeyMask)) {
            kr[j + 1] = kr[j];
            for (int c = 0; c < sw; ++c) xr[sw * (j + 1) + c] = xr[sw * j + c];
            --j;
        }
        kr[j + 1] = k;
        for (int c = 0; c < sw; ++c) xr[sw * (j + 1) + c] = v[c];
    }
}

// Stretch adjoints from canonical rows A to canonical rows B (the same contacts, possibly
// laid out differently): every contact of B takes the adjoint of its match in A, or 0.
template <int sw>
__global__ void __launch_bounds__(kBlock) k_canon_rekey(int N, int M, const int *__restrict__ keyA,
                                                        const int *__restrict__ cntA, const double *__restrict__ gA,
                                                        const int *__restrict__ keyB, const int *__restrict__ cntB,
                                                        double *__restrict__ gB)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const int n = cntB[a];
    for (int k = 0; k < n; ++k) {
        const long long q = (long long)a * M + k;
        const long long s = canon_find(keyA, cntA, M, a, keyB[q] & kKeyMask);
        for (int c = 0; c < sw; ++c) gB[sw * q + c] = s >= 0 ? gA[sw * s + c] : 0.0;
    }
}

// Clear the stretch adjoints of the contacts in canonical rows (the entries that exist).
template <int sw>
__global__ void __launch_bounds__(kBlock) k_canon_zero(int N, int M, const int *__restrict__ cnt,
                                                       double *__restrict__ g)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const int n = cnt[a];
    double *r = g + (long long)a * M * sw;
    for (int k = 0; k < sw * n; ++k) r[k] = 0.0;
}

// ----------------------------------------------------------------------------------
// k_pairs_vjp: reverse of the pair terms of one force evaluation (time index `step`).
// For a listed pair (a, b), a < b, r = x_b - x_a (Lees-Edwards minimum image), the
// stretch before the step is looked up in the canonical rows of the previous history, the
// cotangents of the pair's outputs are gathered (force cotangent Fb_a - Fb_b since
// F_b = -F_a, torque cotangents, the stretch cotangent from the rows after the step, the
// stress weights), and pair_vjp pulls them back (vjp_of_pair), one lane per pair.  The
// cotangents of both particles' x, u, w are stored with the pair (18 doubles, plain
// stores), and k_pairs_vjp_sum adds them to each particle over its recorded pairs (a list of
// integer codes per particle, of fixed capacity, written by this kernel; the codes beyond a
// full list go to an overflow list whose entries k_pairs_vjp_sum adds with FP64 atomics, so
// there are none on the common path); the old-stretch adjoint is stored at the
// contact's position in the previous rows, and the parameter gradients (mu, F_ER) are summed
// per workgroup, then added once.
// ----------------------------------------------------------------------------------
struct VjpTape {
    const int *pairs;       // 2 x npairs (id_min, id_max)
    const double *x, *u, *w, *rad;   // by id: positions, evaluation velocities, radii
    const int *key_old, *cnt_old;    // canonical rows before the step (null: empty)
    const double *xi_old;
    const int *key_new, *cnt_new;    // canonical rows after the step (null: not committed)
    int sw;                          // stretch entries per contact: 3, or 6 with the rolling stretch
};

// The reverse pass of recorded pair k of a tape entry: its ids (a < b), the position of its
// stretch in the previous canonical rows (or -1), and its PairGrad.
__device__ __forceinline__ void vjp_of_pair(const DevParams &P, const BoxParams &G, long long step, int k,
                                            const VjpTape &tp, const double *__restrict__ xib_new,
                                            const double *__restrict__ Fb, const double *__restrict__ Tb,
                                            const double *__restrict__ Sb, int &a, int &b, long long &pold,
                                            PairGrad &g)
{
    a = tp.pairs[2 * k];
    b = tp.pairs[2 * k + 1];
    const double delta = le_offset(P, G, step);
    const double *xa = tp.x + 3LL * a, *xb = tp.x + 3LL * b;
    double r[3];
    min_image(G, delta, xa[0], xa[1], xa[2], xb[0], xb[1], xb[2], r[0], r[1], r[2]);
    const int sw = tp.sw;
    double xo[3] = {0.0, 0.0, 0.0}, xro[3] = {0.0, 0.0, 0.0};
    pold = -1;
    if (tp.key_old) {
        pold = canon_find(tp.key_old, tp.cnt_old, P.M, a, b);
        if (pold >= 0)
            for (int c = 0; c < 3; ++c) {
                xo[c] = tp.xi_old[sw * pold + c];
                if (sw == 6) xro[c] = tp.xi_old[sw * pold + 3 + c];
            }
    }
    PairBar bar;
    for (int c = 0; c < 3; ++c) {
        bar.Fi[c] = Fb[3LL * a + c] - Fb[3LL * b + c];
        bar.Ti[c] = Tb[3LL * a + c];
        bar.Tj[c] = Tb[3LL * b + c];
        bar.xi[c] = 0.0;
        bar.xr[c] = 0.0;
    }
    // branch of the forward run: a pair is a contact after the step iff its rows hold it,
    // and the rows record whether its Coulomb cap and its rolling limit were active (at the
    // initial evaluation, which commits no rows, the branch is recomputed)
    int f_contact = -1, f_capped = -1, f_rcapped = -1;
    if (tp.key_new) {
        const long long pn = canon_find(tp.key_new, tp.cnt_new, P.M, a, b);
        f_contact = pn >= 0 ? 1 : 0;
        f_capped = pn >= 0 ? ((tp.key_new[pn] & kCapBit) ? 1 : 0) : 0;
        f_rcapped = pn >= 0 ? ((tp.key_new[pn] & kRollCapBit) ? 1 : 0) : 0;
        if (pn >= 0 && xib_new)
            for (int c = 0; c < 3; ++c) {
                bar.xi[c] = xib_new[sw * pn + c];
                if (sw == 6) bar.xr[c] = xib_new[sw * pn + 3 + c];
            }
    }
    for (int c = 0; c < 9; ++c) bar.S[c] = Sb ? Sb[c] : 0.0;
    PairConst C;
    C.k6 = P.k6; C.kn = P.kn; C.kt = P.kt; C.gn = P.gn; C.mu = P.mu; C.fer = P.fer; C.a0 = P.a0;
    C.lamd = P.lamd; C.ham = P.ham; C.eps_vdw = P.eps_vdw; C.eps_lub = P.eps_lub; C.dt = P.dt;
    C.ec = P.ec; C.cf = P.cf; C.rep_rng = P.rep_rng; C.att_rng = P.att_rng;
    C.roll = sw == 6 ? 1 : 0; C.kr = P.kr; C.mu_r = P.mu_r;
    pair_vjp(C, G.gd, r, tp.rad[a], tp.rad[b], xa[1], xb[1], tp.u + 3LL * a, tp.u + 3LL * b, tp.w + 3LL * a,
             tp.w + 3LL * b, xo, bar, g, nullptr, f_contact, f_capped, xro, f_rcapped);
}

// Lists of the recorded pairs of a tape entry by particle: each pair's code 2 k + side (side 0:
// the smaller id a, 1: b) goes to the list of each of its ids, list p holding at most cap
// codes at adj[p cap ..] (pos[p] counts them, zero on entry; k_pairs_vjp_sum clears it); a
// code beyond a full list goes, with its id, to the overflow list (ovf_n entries, zero on
// entry; k_integrate_vjp clears the count).
// The order inside a list depends on scheduling; so does the order of the sums below it, as
// with any floating-point accumulation on the GPU.
constexpr int kAdjCap = 32;  // default capacity of a particle's list

__device__ __forceinline__ void adj_push(int id, int code, int cap, int *__restrict__ pos, int *__restrict__ adj,
                                         unsigned *__restrict__ ovf_n, int2 *__restrict__ ovf)
{
    const int slot = atomicAdd(&pos[id], 1);
    if (slot < cap)
        adj[(long long)id * cap + slot] = code;
    else
        ovf[atomicAdd(ovf_n, 1u)] = make_int2(id, code);
}

__global__ void __launch_bounds__(kBlock) k_pairs_vjp(DevParams P, BoxParams G, long long step, int npairs,
                                                      VjpTape tp, const double *__restrict__ xib_new,
                                                      double *__restrict__ xib_old, const double *__restrict__ Fb,
                                                      const double *__restrict__ Tb, const double *__restrict__ Sb,
                                                      double *__restrict__ gpair, double *__restrict__ theta_b,
                                                      int cap, int *__restrict__ pos, int *__restrict__ adj,
                                                      unsigned *__restrict__ ovf_n, int2 *__restrict__ ovf)
{
    __shared__ double red[kBlock / 64][2];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double gmu = 0.0, gfer = 0.0;
    if (k < npairs) {
        // the pair's entries in the lists of its two ids (their atomics overlap the pair's
        // arithmetic)
        adj_push(tp.pairs[2 * k], 2 * k, cap, pos, adj, ovf_n, ovf);
        adj_push(tp.pairs[2 * k + 1], 2 * k + 1, cap, pos, adj, ovf_n, ovf);
        int a, b;
        long long pold;
        PairGrad g = {};
        vjp_of_pair(P, G, step, k, tp, xib_new, Fb, Tb, Sb, a, b, pold, g);
        // the two sides: (x, u, w) cotangents of a, then of b
        const double o[18] = {-g.r[0], -g.r[1] + g.yi, -g.r[2], g.ui[0], g.ui[1], g.ui[2], g.wi[0], g.wi[1], g.wi[2],
                              g.r[0],  g.r[1] + g.yj,  g.r[2],  g.uj[0], g.uj[1], g.uj[2], g.wj[0], g.wj[1], g.wj[2]};
        double2 *q = reinterpret_cast<double2 *>(gpair + 18LL * k);
#pragma unroll
        for (int c = 0; c < 9; ++c) q[c] = make_double2(o[2 * c], o[2 * c + 1]);
        if (pold >= 0 && xib_old)
            for (int c = 0; c < 3; ++c) {
                xib_old[tp.sw * pold + c] = g.xo[c];
                if (tp.sw == 6) xib_old[tp.sw * pold + 3 + c] = g.xro[c];
            }
        gmu = g.mu;
        gfer = g.fer;
    }
    gmu = warp_sum(gmu);
    gfer = warp_sum(gfer);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[wid][0] = gmu;
        red[wid][1] = gfer;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int q = 0; q < kBlock / 64; ++q) {
            s0 += red[q][0];
            s1 += red[q][1];
        }
        atomicAdd(theta_b, s0);
        atomicAdd(theta_b + 1, s1);
    }
}

// Per particle: the cotangents of its listed codes added in list order to its adjoints (the
// list positions cleared for the next evaluation); the codes of the overflow list, beyond full
// lists, are added by the same grid with FP64 atomics, and so are the list sums of the
// particles that overflowed, whose adjoints have more than one writer.  k_integrate_vjp
// clears the overflow count afterwards.
__global__ void __launch_bounds__(kBlock) k_pairs_vjp_sum(int N, int cap, int *__restrict__ pos,
                                                          const int *__restrict__ adj,
                                                          const unsigned *__restrict__ ovf_n,
                                                          const int2 *__restrict__ ovf,
                                                          const double *__restrict__ gpair, double *__restrict__ ax,
                                                          double *__restrict__ au, double *__restrict__ aw)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned no = *ovf_n;
    for (unsigned e = p; e < no; e += gridDim.x * blockDim.x) {
        const int2 v = ovf[e];
        const double *g = gpair + 18LL * (v.y >> 1) + 9 * (v.y & 1);
        for (int c = 0; c < 3; ++c) {
            atomicAdd(&ax[3LL * v.x + c], g[c]);
            atomicAdd(&au[3LL * v.x + c], g[3 + c]);
            atomicAdd(&aw[3LL * v.x + c], g[6 + c]);
        }
    }
    if (p >= N) return;
    const int m = pos[p];
    pos[p] = 0;
    const int n = m < cap ? m : cap;
    double s[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int *lst = adj + (long long)p * cap;
    for (int e = 0; e < n; ++e) {
        const int code = lst[e];
        const double *g = gpair + 18LL * (code >> 1) + 9 * (code & 1);
#pragma unroll
        for (int c = 0; c < 9; ++c) s[c] += g[c];
    }
    if (m > cap) {
        for (int c = 0; c < 3; ++c) {
            atomicAdd(&ax[3LL * p + c], s[c]);
            atomicAdd(&au[3LL * p + c], s[3 + c]);
            atomicAdd(&aw[3LL * p + c], s[6 + c]);
        }
    } else {
        for (int c = 0; c < 3; ++c) {
            ax[3LL * p + c] += s[c];
            au[3LL * p + c] += s[3 + c];
            aw[3LL * p + c] += s[6 + c];
        }
    }
}

// ----------------------------------------------------------------------------------
// k_integrate_vjp: per particle, the reverse of the Stokes terms of the evaluation at
// step n (F^S = -6 pi eta0 a (uh - gd y e_x), T^S = -8 pi eta0 a^3 (wh + gd/2 e_z)), then
// of the drift and kick that produced x_n, uh_n:
//   xb' = xb + ax,  ub' = ub + au + dt xb',  wb' = wb + aw,
//   Fb_{n-1} = c dt ub' / m,  Tb_{n-1} = c dt wb' / I
// (xb, ub, wb in: adjoints of x_n, uh_{n+1}, wh_{n+1} from the later steps; out: of x_{n-1},
// uh_n, wh_n).  final != 0: the evaluation at the initial state; the adjoints of the
// initial x, u, w are xb + ax, ub + au, wb + aw.  ax, au, aw are cleared.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_integrate_vjp(DevParams P, double gd, int N, double c, int final,
                                                          const double *__restrict__ rad,
                                                          const double *__restrict__ Fb, const double *__restrict__ Tb,
                                                          double *__restrict__ ax, double *__restrict__ au,
                                                          double *__restrict__ aw, double *__restrict__ xb,
                                                          double *__restrict__ ub, double *__restrict__ wb,
                                                          double *__restrict__ Fb_prev, double *__restrict__ Tb_prev,
                                                          unsigned *__restrict__ ovf_n, const int *__restrict__ zcnt,
                                                          double *__restrict__ zbuf, int M, int sw)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *ovf_n = 0u;  // the pair sums of this evaluation are complete
    if (p >= N) return;
    // the stretch adjoints that the next reverse step writes, cleared over the canonical rows
    // of its earlier history (the buffer this step's pair VJP has finished reading)
    if (zcnt) {
        double *r = zbuf + (long long)p * M * sw;
        const int n = sw * zcnt[p];
        for (int k = 0; k < n; ++k) r[k] = 0.0;
    }
    const double a = rad[p];
    const double K = P.k6 * a, KR = P.k8 * a * a * a;
    const double m = pmass(P, a), I = 0.4 * m * a * a;
    const double dt = P.dt;
    double gx[3], gu[3], gw[3];
    for (int k = 0; k < 3; ++k) {
        const long long q = 3LL * p + k;
        gx[k] = ax[q];
        gu[k] = au[q] - K * Fb[q];
        gw[k] = aw[q] - KR * Tb[q];
        ax[q] = 0.0;
        au[q] = 0.0;
        aw[q] = 0.0;
    }
    gx[1] += K * gd * Fb[3LL * p];
    for (int k = 0; k < 3; ++k) {
        const long long q = 3LL * p + k;
        if (final) {
            xb[q] += gx[k];
            ub[q] += gu[k];
            wb[q] += gw[k];
        } else {
            const double X = xb[q] + gx[k];
            const double U = ub[q] + gu[k] + dt * X;
            const double W = wb[q] + gw[k];
            xb[q] = X;
            ub[q] = U;
            wb[q] = W;
            Fb_prev[q] = c * dt * U / m;
            Tb_prev[q] = c * dt * W / I;
        }
    }
}

}  // namespace dss

namespace dss {

// Radius of every particle by id.
__global__ void __launch_bounds__(kBlock) k_rad_by_id(int N, const double4 *__restrict__ pa,
                                                      const double4 *__restrict__ omg, double *__restrict__ rad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    rad[(int)omg[p].w] = pa[p].w;
}

}  // namespace dss
