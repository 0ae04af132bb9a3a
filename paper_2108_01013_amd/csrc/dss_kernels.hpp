// dss_kernels.hpp -- HIP kernels of one dense-suspension time step on CDNA4 (gfx950).
//
// Data layout (all in sorted order = cell-major order of the last counting sort):
//   pa  double4 [N]  (x, y, z, radius)
//   vel double4 [N]  (u_x, u_y, u_z, 0): the velocity the last forces were evaluated with
//   omg double4 [N]  (w_x, w_y, w_z, id): angular velocity and the particle id (as a double)
//   frc double4 [N]  (F_x, F_y, F_z, 0), trq double4 [N]: totals of the last evaluation
// One 32-byte record per particle and quantity, so a neighbour gather is one 32-byte
// access per array; streaming kernels read them as two 16-byte loads per lane.
//
// Step kernels: k_predict (kick/drift, Lees-Edwards wrap, cell id, histogram rank),
// k_scan (exclusive scan of the cell counts), k_scatter (reorder), k_pairs (half-shell
// search + pair physics + history rows + stress).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dss {

constexpr double kPi = 3.14159265358979323846;
constexpr int kBlock = 256;

// error flag bits (device word)
constexpr unsigned kErrRowOverflow = 1u;
constexpr unsigned kErrNonFinite = 2u;
constexpr unsigned kErrPairBuffer = 4u;

struct DevParams {
    double L[3];
    double gd, eta0, rho, kn, kt, gn, mu, fer, lamd, a0, ham, eps_vdw, eps_lub, cf, dt;
    double cw[3];      // cell widths L/n
    int nc[3];         // cells per dimension
    int ncell;
    int N;
    int M;             // history row capacity
    int record_pairs;
    long long pair_cap;
};

// Device-side clock and per-evaluation counters.  step = time index of the state.
struct DevClock {
    long long step;
    unsigned long long n_pairs;
    unsigned long long n_contacts;
    int max_fill;
    unsigned err;
};

// Run descriptor of a dss_step call: stress sampling schedule.
struct DevRun {
    long long sample_every;   // 0: no sampling
    long long sample_first;   // first sampled time index of this call
    long long sample_cap;     // number of sample slots
    double *samples;          // sample_cap x 9
    double *sigma_last;       // 9: pair part of the stress of the last evaluation
};

// ----------------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------------
__device__ __forceinline__ double le_offset(const DevParams &P, long long step)
{
#pragma clang fp contract(off)
    double t = (double)step * P.dt;
    double s = P.gd * P.L[1] * t;
    return fmod(s, P.L[0]);
}

__device__ __forceinline__ int cell_coord(double xd, double cw, int n)
{
    int c = (int)(xd / cw);
    c = c < 0 ? 0 : c;
    c = c > n - 1 ? n - 1 : c;
    return c;
}

// Nearest image of b seen from a under Lees-Edwards shear; r = x_b - x_a.  Evaluated
// without contraction so that the listed-pair test is the IEEE expression as written.
__device__ __forceinline__ void min_image(const DevParams &P, double delta, double xa, double ya, double za,
                                          double xb, double yb, double zb, double &dx, double &dy, double &dz)
{
#pragma clang fp contract(off)
    dx = xb - xa;
    dy = yb - ya;
    dz = zb - za;
    if (dy > 0.5 * P.L[1]) {
        dy -= P.L[1];
        dx -= delta;
    } else if (dy < -0.5 * P.L[1]) {
        dy += P.L[1];
        dx += delta;
    }
    dx -= P.L[0] * rint(dx / P.L[0]);
    dz -= P.L[2] * rint(dz / P.L[2]);
}

__device__ __forceinline__ bool listed(const DevParams &P, double dx, double dy, double dz, double aa, double ab,
                                       double &r2)
{
#pragma clang fp contract(off)
    r2 = (dx * dx + dy * dy) + dz * dz;
    double rc = P.cf * (aa + ab);
    return r2 < rc * rc;
}

__device__ __forceinline__ double pmass(const DevParams &P, double a)
{
#pragma clang fp contract(off)
    return P.rho * (4.0 / 3.0) * kPi * a * a * a;
}

__device__ __forceinline__ double warp_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ long long warp_sum_ll(long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int warp_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) {
        int w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// ----------------------------------------------------------------------------------
// k_predict: velocity-Verlet drift + half kick (advance = 1) or velocity completion
// only (advance = 0), Lees-Edwards wrap at t_{n+1}, cell id and histogram rank.
//   vel_is_half = 1: vel holds the half-step velocity u^{n-1/2} of the forces frc, and
//   u^n = u^{n-1/2} + dt/2 F^n / m completes the previous step.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_predict(DevParams P, double4 *__restrict__ pa, double4 *__restrict__ vel,
                                                     double4 *__restrict__ omg, const double4 *__restrict__ frc,
                                                     const double4 *__restrict__ trq, int vel_is_half, int advance,
                                                     const DevClock *__restrict__ clk, int *__restrict__ cell,
                                                     int *__restrict__ rank, int *__restrict__ count)
{
#pragma clang fp contract(off)
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.N) return;
    double4 X = pa[p];
    double4 V = vel[p];
    double4 W = omg[p];
    const double dt = P.dt;
    double a = X.w;
    double m = pmass(P, a);
    double I = 0.4 * m * a * a;
    double4 Fp = frc[p];
    double4 Tp = trq[p];
    double ax = Fp.x / m, ay = Fp.y / m, az = Fp.z / m;
    double bx = Tp.x / I, by = Tp.y / I, bz = Tp.z / I;
    if (vel_is_half) {  // finish the previous step: u^n = u^{n-1/2} + dt/2 alpha^n
        V.x = V.x + 0.5 * dt * ax;
        V.y = V.y + 0.5 * dt * ay;
        V.z = V.z + 0.5 * dt * az;
        W.x = W.x + 0.5 * dt * bx;
        W.y = W.y + 0.5 * dt * by;
        W.z = W.z + 0.5 * dt * bz;
    }
    if (advance) {
        X.x = X.x + dt * V.x + 0.5 * dt * dt * ax;
        X.y = X.y + dt * V.y + 0.5 * dt * dt * ay;
        X.z = X.z + dt * V.z + 0.5 * dt * dt * az;
        V.x = V.x + 0.5 * dt * ax;
        V.y = V.y + 0.5 * dt * ay;
        V.z = V.z + 0.5 * dt * az;
        W.x = W.x + 0.5 * dt * bx;
        W.y = W.y + 0.5 * dt * by;
        W.z = W.z + 0.5 * dt * bz;
        // Lees-Edwards wrap at t_{n+1}
        double delta = le_offset(P, clk->step + 1);
        if (X.y >= P.L[1]) {
            X.y -= P.L[1];
            X.x -= delta;
            V.x -= P.gd * P.L[1];
        } else if (X.y < 0.0) {
            X.y += P.L[1];
            X.x += delta;
            V.x += P.gd * P.L[1];
        }
        X.x -= P.L[0] * floor(X.x / P.L[0]);
        X.z -= P.L[2] * floor(X.z / P.L[2]);
        pa[p] = X;
    }
    vel[p] = V;
    omg[p] = W;
    int cx = cell_coord(X.x, P.cw[0], P.nc[0]);
    int cy = cell_coord(X.y, P.cw[1], P.nc[1]);
    int cz = cell_coord(X.z, P.cw[2], P.nc[2]);
    int c = (cz * P.nc[1] + cy) * P.nc[0] + cx;
    cell[p] = c;
    rank[p] = atomicAdd(&count[c], 1);
}

// ----------------------------------------------------------------------------------
// k_scan: cell_start = exclusive scan of count (ncell + 1 entries), count reset to 0,
// per-evaluation counters reset, clock advanced.  One workgroup of 1024 lanes; each lane
// owns a contiguous chunk, chunk sums are scanned across the 16 wavefronts.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_scan(int ncell, int *__restrict__ count, int *__restrict__ cell_start,
                                               DevClock *__restrict__ clk, int advance, DevRun *__restrict__ run)
{
    __shared__ int wsum[16];
    const int t = threadIdx.x;
    const int chunk = (ncell + 1023) / 1024;
    const int lo = t * chunk;
    const int hi = min(lo + chunk, ncell);
    int s = 0;
    for (int c = lo; c < hi; ++c) s += count[c];
    // inclusive scan of s across the wavefront
    int lane = t & 63, wid = t >> 6;
    int v = s;
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) wsum[wid] = v;
    __syncthreads();
    if (wid == 0) {
        int w = lane < 16 ? wsum[lane] : 0;
        for (int o = 1; o < 16; o <<= 1) {
            int u = __shfl_up(w, o, 64);
            if (lane >= o) w += u;
        }
        if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    int base = v - s + (wid > 0 ? wsum[wid - 1] : 0);
    for (int c = lo; c < hi; ++c) {
        int k = count[c];
        cell_start[c] = base;
        base += k;
        count[c] = 0;
    }
    if (t == 1023) cell_start[ncell] = base;
    if (t == 0) {
        if (advance) clk->step += 1;
        clk->n_pairs = 0;
        clk->n_contacts = 0;
        clk->max_fill = 0;
        for (int k = 0; k < 9; ++k) run->sigma_last[k] = 0.0;
    }
}

// ----------------------------------------------------------------------------------
// k_scatter: move every particle to its sorted slot, record id -> slot, clear forces.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_scatter(int N, const int *__restrict__ cell, const int *__restrict__ rank,
                                                     const int *__restrict__ cell_start,
                                                     const double4 *__restrict__ pa_in,
                                                     const double4 *__restrict__ vel_in,
                                                     const double4 *__restrict__ omg_in, double4 *__restrict__ pa_out,
                                                     double4 *__restrict__ vel_out, double4 *__restrict__ omg_out,
                                                     double4 *__restrict__ frc_out, double4 *__restrict__ trq_out,
                                                     int *__restrict__ inv)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    int dst = cell_start[cell[p]] + rank[p];
    double4 W = omg_in[p];
    pa_out[dst] = pa_in[p];
    vel_out[dst] = vel_in[p];
    omg_out[dst] = W;
    frc_out[dst] = make_double4(0.0, 0.0, 0.0, 0.0);
    trq_out[dst] = make_double4(0.0, 0.0, 0.0, 0.0);
    inv[(int)W.w] = dst;
}

// ----------------------------------------------------------------------------------
// Pair physics of one listed pair (i, j), r = x_j - x_i.  Lubrication in the reduced
// form of the resistance matrices of Appendix A: with v = (u'_j - u'_i) + (a_i + a_j) E n
// (the ambient-strain rows of R'(E) add exactly the affine velocity of the gap),
//   F_i = X^A (v.n) n + Y^A T v - Y^B_ii n x w'_i + Y^B_jj n x w'_j,   F_j = -F_i
//   T_i = -Y^B_ii n x v - Y^C_ii T w'_i - Y^C_ij T w'_j
//   T_j =  Y^B_jj n x v - Y^C_ij T w'_i - Y^C_jj T w'_j
// with X^A = 6 pi eta0 2 a_i^2 a_j^2 / s^3 / (d* + eps), s = a_i + a_j, and the Y's
// 6 pi eta0 g^Y log(1 / (d* + eps)) from the g table written in a_i, a_j.
// ----------------------------------------------------------------------------------
struct PairOut {
    double Fi[3];   // total pair force on i (F_j = -F_i)
    double Ti[3];   // torque on i
    double Tj[3];   // torque on j
    double S[9];    // stresslet r (x) F summed over kinds (lubrication part symmetrised)
    double xi[3];   // new tangential stretch, oriented i -> j
    bool contact;
};

__device__ __forceinline__ void pair_physics(const DevParams &P, double dx, double dy, double dz, double r2,
                                             double ai, double aj, double yi, double yj, const double4 &Vi,
                                             const double4 &Vj, const double4 &Wi, const double4 &Wj,
                                             const double xo[3], bool want_stress, PairOut &o)
{
    const double dist = sqrt(r2);
    const double inv_d = 1.0 / dist;
    const double nx = dx * inv_d, ny = dy * inv_d, nz = dz * inv_d;
    const double h = dist - ai - aj;
    const double s = ai + aj;
    const double gd = P.gd;
    // fluctuation velocities u' = u - U_inf(x); w' = w - Omega_inf
    const double dux = (Vj.x - gd * yj) - (Vi.x - gd * yi);
    const double duy = Vj.y - Vi.y;
    const double duz = Vj.z - Vi.z;
    const double wix = Wi.x, wiy = Wi.y, wiz = Wi.z + 0.5 * gd;
    const double wjx = Wj.x, wjy = Wj.y, wjz = Wj.z + 0.5 * gd;

    // ---------------- lubrication
    double dstar = 2.0 * h / s;
    dstar = dstar > 0.0 ? dstar : 0.0;
    const double g = dstar + P.eps_lub;
    const double invg = 1.0 / g;
    const double lg = -log(g);
    const double K = 6.0 * kPi * P.eta0;
    const double ai2 = ai * ai, aj2 = aj * aj;
    const double is = 1.0 / s;
    const double is2 = is * is, is3 = is2 * is;
    const double XA = K * 2.0 * ai2 * aj2 * is3 * invg;
    const double YA = K * (4.0 / 15.0) * ai * aj * (2.0 * ai2 + ai * aj + 2.0 * aj2) * is3 * lg;
    const double YBi = -K * (2.0 / 15.0) * ai2 * aj * (4.0 * ai + aj) * is2 * lg;
    const double YBj = K * (2.0 / 15.0) * ai * aj2 * (ai + 4.0 * aj) * is2 * lg;
    const double YCii = K * (8.0 / 15.0) * ai2 * ai * aj * is * lg;
    const double YCij = K * (2.0 / 15.0) * ai2 * aj2 * is * lg;
    const double YCjj = K * (8.0 / 15.0) * ai * aj2 * aj * is * lg;
    // v = du + s E n, E n = gd/2 (n_y, n_x, 0)
    const double vx = dux + s * 0.5 * gd * ny;
    const double vy = duy + s * 0.5 * gd * nx;
    const double vz = duz;
    const double vn = vx * nx + vy * ny + vz * nz;
    // n x w'
    const double cix = ny * wiz - nz * wiy, ciy = nz * wix - nx * wiz, ciz = nx * wiy - ny * wix;
    const double cjx = ny * wjz - nz * wjy, cjy = nz * wjx - nx * wjz, cjz = nx * wjy - ny * wjx;
    double FLx = XA * vn * nx + YA * (vx - vn * nx) - YBi * cix + YBj * cjx;
    double FLy = XA * vn * ny + YA * (vy - vn * ny) - YBi * ciy + YBj * cjy;
    double FLz = XA * vn * nz + YA * (vz - vn * nz) - YBi * ciz + YBj * cjz;
    // n x v
    const double nvx = ny * vz - nz * vy, nvy = nz * vx - nx * vz, nvz = nx * vy - ny * vx;
    // T w' = w' - (w'.n) n
    const double win = wix * nx + wiy * ny + wiz * nz;
    const double wjn = wjx * nx + wjy * ny + wjz * nz;
    const double tix = wix - win * nx, tiy = wiy - win * ny, tiz = wiz - win * nz;
    const double tjx = wjx - wjn * nx, tjy = wjy - wjn * ny, tjz = wjz - wjn * nz;
    o.Ti[0] = -YBi * nvx - YCii * tix - YCij * tjx;
    o.Ti[1] = -YBi * nvy - YCii * tiy - YCij * tjy;
    o.Ti[2] = -YBi * nvz - YCii * tiz - YCij * tjz;
    o.Tj[0] = YBj * nvx - YCij * tix - YCjj * tjx;
    o.Tj[1] = YBj * nvy - YCij * tiy - YCjj * tjy;
    o.Tj[2] = YBj * nvz - YCij * tiz - YCjj * tjz;

    // ---------------- electro-chemical (central): repulsion eq. rep, attraction eq. att
    const double abar = 2.0 * ai * aj * is;
    double fe = 0.0;
    if (P.fer != 0.0) fe -= P.fer * (abar / P.a0) * (h >= 0.0 ? (P.lamd > 0.0 ? exp(-h / P.lamd) : 0.0) : 1.0);
    if (P.ham != 0.0) {
        const double e = P.eps_vdw * abar;
        fe += P.ham * abar / (12.0 * ((h >= 0.0 ? h * h : 0.0) + e * e));
    }

    // ---------------- contact eqs. contact0, csi
    double FCx = 0.0, FCy = 0.0, FCz = 0.0;
    o.contact = h < 0.0;
    o.xi[0] = o.xi[1] = o.xi[2] = 0.0;
    if (o.contact) {
        // true relative velocity of the image pair: ambient difference gd r_y along x
        const double Dx = dux + gd * dy, Dy = duy, Dz = duz;
        const double un = Dx * nx + Dy * ny + Dz * nz;
        const double fn = P.kn * h + P.gn * un;
        const double Fnx = fn * nx, Fny = fn * ny, Fnz = fn * nz;
        const double sx = ai * Wi.x + aj * Wj.x, sy = ai * Wi.y + aj * Wj.y, sz = ai * Wi.z + aj * Wj.z;
        // (a_i w_i + a_j w_j) x n
        const double qx = sy * nz - sz * ny, qy = sz * nx - sx * nz, qz = sx * ny - sy * nx;
        const double tx = Dx - qx, ty = Dy - qy, tz = Dz - qz;
        const double tn = tx * nx + ty * ny + tz * nz;
        double xx = xo[0] + (tx - tn * nx) * P.dt;
        double xy = xo[1] + (ty - tn * ny) * P.dt;
        double xz = xo[2] + (tz - tn * nz) * P.dt;
        const double xn = xx * nx + xy * ny + xz * nz;
        xx -= xn * nx;
        xy -= xn * ny;
        xz -= xn * nz;
        double Ftx = 0.0, Fty = 0.0, Ftz = 0.0;
        if (P.kt > 0.0) {
            const double cap = P.mu * fabs(fn) / P.kt;
            const double xm = sqrt(xx * xx + xy * xy + xz * xz);
            if (xm >= cap && xm > 0.0) {
                const double sc = cap / xm;
                xx *= sc;
                xy *= sc;
                xz *= sc;
            }
            Ftx = P.kt * xx;
            Fty = P.kt * xy;
            Ftz = P.kt * xz;
        } else {
            xx = xy = xz = 0.0;
        }
        o.xi[0] = xx;
        o.xi[1] = xy;
        o.xi[2] = xz;
        FCx = Fnx + Ftx;
        FCy = Fny + Fty;
        FCz = Fnz + Ftz;
        // T_i = a_i n x F_t, T_j = a_j n x F_t
        const double mx = ny * Ftz - nz * Fty, my = nz * Ftx - nx * Ftz, mz = nx * Fty - ny * Ftx;
        o.Ti[0] += ai * mx;
        o.Ti[1] += ai * my;
        o.Ti[2] += ai * mz;
        o.Tj[0] += aj * mx;
        o.Tj[1] += aj * my;
        o.Tj[2] += aj * mz;
    }
    const double Fex = fe * nx, Fey = fe * ny, Fez = fe * nz;
    o.Fi[0] = FLx + FCx + Fex;
    o.Fi[1] = FLy + FCy + Fey;
    o.Fi[2] = FLz + FCz + Fez;
    if (want_stress) {
        const double r[3] = {dx, dy, dz};
        const double FL[3] = {FLx, FLy, FLz};
        const double FO[3] = {FCx + Fex, FCy + Fey, FCz + Fez};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) o.S[3 * a + b] = 0.5 * (r[a] * FL[b] + r[b] * FL[a]) + r[a] * FO[b];
    }
}

// ----------------------------------------------------------------------------------
// History lookup: row of the particle that was at sorted slot p in the previous
// evaluation; rows are sorted by partner id, so the scan stops at the first larger key.
// ----------------------------------------------------------------------------------
__device__ __forceinline__ bool row_find(const int *__restrict__ hkey, const double *__restrict__ hxi,
                                         const int *__restrict__ hcnt, int M, int p, int key, double out[3])
{
    const int n = hcnt[p];
    const int *kr = hkey + (long long)p * M;
    for (int k = 0; k < n; ++k) {
        int kk = kr[k];
        if (kk == key) {
            const double *x = hxi + ((long long)p * M + k) * 3;
            out[0] = x[0];
            out[1] = x[1];
            out[2] = x[2];
            return true;
        }
        if (kk > key) break;
    }
    return false;
}

struct HistView {
    const int *key_old;
    const double *xi_old;
    const int *cnt_old;
    const int *inv_old;
    int *key_new;
    double *xi_new;
    int *cnt_new;
    int *own_new;   // owner id of each new row
};

// ----------------------------------------------------------------------------------
// k_pairs: one lane per sorted particle i.  Scans its own cell (later slots only) and
// the 13 forward cells of the half shell: (dz > 0) or (dz = 0, dy > 0) or
// (dz = dy = 0, dx > 0).  A row reached across a y face is a window of 4 x-cells
// around the Lees-Edwards-shifted position.  Cells with consecutive cx are contiguous
// in sorted order, so each row is one or two contiguous slot ranges.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_pairs(DevParams P, const int *__restrict__ cell_start,
                                                   const double4 *__restrict__ pa, const double4 *__restrict__ vel,
                                                   const double4 *__restrict__ omg, double4 *__restrict__ frc,
                                                   double4 *__restrict__ trq, HistView H, DevClock *__restrict__ clk,
                                                   DevRun *__restrict__ run, int *__restrict__ pair_out,
                                                   unsigned long long *__restrict__ pair_count)
{
    __shared__ double red[kBlock / 64][12];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const long long step = clk->step;
    const bool want_stress = true;
    const double delta = le_offset(P, step);
    double Fi[3] = {0, 0, 0}, Ti[3] = {0, 0, 0}, S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    long long npair = 0, ncont = 0;
    int fill = 0;
    if (i < P.N) {
        const double4 Xi = pa[i];
        const double4 Vi = vel[i];
        const double4 Wi = omg[i];
        const int idi = (int)Wi.w;
        const int cx = cell_coord(Xi.x, P.cw[0], P.nc[0]);
        const int cy = cell_coord(Xi.y, P.cw[1], P.nc[1]);
        const int cz = cell_coord(Xi.z, P.cw[2], P.nc[2]);
        const int nxc = P.nc[0], nyc = P.nc[1], nzc = P.nc[2];
        int *krow = H.key_new + (long long)i * P.M;
        double *xrow = H.xi_new + (long long)i * P.M * 3;
        const int pi_old = H.inv_old[idi];

        // rows of the half shell: (dz, dy) with x window [xlo, xhi] (may wrap)
        // row 0: own row, cells cx .. cx+1 with j > i in the own cell
        for (int row = 0; row < 5; ++row) {
            int dz, dy;
            if (row == 0) { dz = 0; dy = 0; }
            else if (row == 1) { dz = 0; dy = 1; }
            else { dz = 1; dy = row - 3; }
            int yy = cy + dy;
            int zz = cz + dz;
            zz = zz >= nzc ? zz - nzc : zz;
            int xlo, xhi;
            if (yy < 0 || yy >= nyc) {
                // across a y face: images displaced by +delta (top) / -delta (bottom)
                double sh = yy >= nyc ? -delta : delta;
                int k0 = (int)floor(((double)cx * P.cw[0] + sh) / P.cw[0]);
                xlo = k0 - 1;
                xhi = k0 + 2;
                yy = yy < 0 ? yy + nyc : yy - nyc;
            } else if (row == 0) {
                xlo = cx;
                xhi = cx + 1;
            } else {
                xlo = cx - 1;
                xhi = cx + 1;
            }
            const int rbase = (zz * nyc + yy) * nxc;
            // split the window into at most two contiguous cell ranges
            int xl = ((xlo % nxc) + nxc) % nxc;
            int span = xhi - xlo + 1;
            for (int part = 0; part < 2 && span > 0; ++part) {
                int len = (xl + span <= nxc) ? span : nxc - xl;
                int jb = cell_start[rbase + xl];
                int je = cell_start[rbase + xl + len];
                if (row == 0 && part == 0) jb = i + 1;  // own cell first: only later slots
                for (int j = jb; j < je; ++j) {
                    const double4 Xj = pa[j];
                    double dx, dy2, dz2, r2;
                    min_image(P, delta, Xi.x, Xi.y, Xi.z, Xj.x, Xj.y, Xj.z, dx, dy2, dz2);
                    if (!listed(P, dx, dy2, dz2, Xi.w, Xj.w, r2)) continue;
                    const double4 Vj = vel[j];
                    const double4 Wj = omg[j];
                    const int idj = (int)Wj.w;
                    ++npair;
                    if (P.record_pairs) {
                        unsigned long long k = atomicAdd(pair_count, 1ull);
                        if ((long long)k < P.pair_cap) {
                            pair_out[2 * k] = idi < idj ? idi : idj;
                            pair_out[2 * k + 1] = idi < idj ? idj : idi;
                        } else {
                            atomicOr(&clk->err, kErrPairBuffer);
                        }
                    }
                    // stored stretch, canonical orientation min id -> max id
                    double xo[3] = {0.0, 0.0, 0.0};
                    const double rc_h = sqrt(r2) - Xi.w - Xj.w;
                    if (rc_h < 0.0) {
                        bool found = row_find(H.key_old, H.xi_old, H.cnt_old, P.M, pi_old, idj, xo);
                        if (!found) found = row_find(H.key_old, H.xi_old, H.cnt_old, P.M, H.inv_old[idj], idi, xo);
                        if (found && idi > idj) {
                            xo[0] = -xo[0];
                            xo[1] = -xo[1];
                            xo[2] = -xo[2];
                        }
                    }
                    PairOut o;
                    pair_physics(P, dx, dy2, dz2, r2, Xi.w, Xj.w, Xi.y, Xj.y, Vi, Vj, Wi, Wj, xo, want_stress, o);
                    Fi[0] += o.Fi[0];
                    Fi[1] += o.Fi[1];
                    Fi[2] += o.Fi[2];
                    Ti[0] += o.Ti[0];
                    Ti[1] += o.Ti[1];
                    Ti[2] += o.Ti[2];
                    atomicAdd(&frc[j].x, -o.Fi[0]);
                    atomicAdd(&frc[j].y, -o.Fi[1]);
                    atomicAdd(&frc[j].z, -o.Fi[2]);
                    atomicAdd(&trq[j].x, o.Tj[0]);
                    atomicAdd(&trq[j].y, o.Tj[1]);
                    atomicAdd(&trq[j].z, o.Tj[2]);
#pragma unroll
                    for (int k = 0; k < 9; ++k) S[k] += o.S[k];
                    if (o.contact) {
                        ++ncont;
                        if (fill < P.M) {
                            const double sg = idi < idj ? 1.0 : -1.0;
                            krow[fill] = idj;
                            xrow[3 * fill + 0] = sg * o.xi[0];
                            xrow[3 * fill + 1] = sg * o.xi[1];
                            xrow[3 * fill + 2] = sg * o.xi[2];
                        } else {
                            atomicOr(&clk->err, kErrRowOverflow);
                        }
                        ++fill;
                    }
                }
                xl = 0;
                span -= len;
            }
        }
        // sort the new row by partner id (insertion sort; rows are short)
        const int nrow = fill < P.M ? fill : P.M;
        for (int a = 1; a < nrow; ++a) {
            int key = krow[a];
            double x0 = xrow[3 * a], x1 = xrow[3 * a + 1], x2 = xrow[3 * a + 2];
            int b = a - 1;
            while (b >= 0 && krow[b] > key) {
                krow[b + 1] = krow[b];
                xrow[3 * (b + 1)] = xrow[3 * b];
                xrow[3 * (b + 1) + 1] = xrow[3 * b + 1];
                xrow[3 * (b + 1) + 2] = xrow[3 * b + 2];
                --b;
            }
            krow[b + 1] = key;
            xrow[3 * (b + 1)] = x0;
            xrow[3 * (b + 1) + 1] = x1;
            xrow[3 * (b + 1) + 2] = x2;
        }
        H.cnt_new[i] = nrow;
        H.own_new[i] = idi;

        // per-particle terms: Stokes drag and rotational drag (eq. rst)
        const double K = 6.0 * kPi * P.eta0;
        Fi[0] += -K * Xi.w * (Vi.x - P.gd * Xi.y);
        Fi[1] += -K * Xi.w * Vi.y;
        Fi[2] += -K * Xi.w * Vi.z;
        const double KR = 8.0 * kPi * P.eta0 * Xi.w * Xi.w * Xi.w;
        Ti[0] += -KR * Wi.x;
        Ti[1] += -KR * Wi.y;
        Ti[2] += -KR * (Wi.z + 0.5 * P.gd);
        atomicAdd(&frc[i].x, Fi[0]);
        atomicAdd(&frc[i].y, Fi[1]);
        atomicAdd(&frc[i].z, Fi[2]);
        atomicAdd(&trq[i].x, Ti[0]);
        atomicAdd(&trq[i].y, Ti[1]);
        atomicAdd(&trq[i].z, Ti[2]);
        if (!(isfinite(Fi[0]) && isfinite(Fi[1]) && isfinite(Fi[2]) && isfinite(Ti[0]) && isfinite(Ti[1]) &&
              isfinite(Ti[2])))
            atomicOr(&clk->err, kErrNonFinite);
    }
    // block reduction of the stress and the counters
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double v = warp_sum(S[k]);
        if (lane == 0) red[wid][k] = v;
    }
    long long np_ = warp_sum_ll(npair), nc_ = warp_sum_ll(ncont);
    int mf = warp_max(fill);
    if (lane == 0) {
        red[wid][9] = (double)np_;
        red[wid][10] = (double)nc_;
        red[wid][11] = (double)mf;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        const int k = threadIdx.x;
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) v = (k == 11) ? fmax(v, red[w][k]) : v + red[w][k];
        if (k < 9) {
            atomicAdd(&run->sigma_last[k], v);
        } else if (k == 9) {
            atomicAdd(&clk->n_pairs, (unsigned long long)v);
        } else if (k == 10) {
            atomicAdd(&clk->n_contacts, (unsigned long long)v);
        } else {
            atomicMax(&clk->max_fill, (int)v);
        }
    }
}

// ----------------------------------------------------------------------------------
// k_sample: copy the pair part of the stress of this evaluation into the sample slot of
// the current time index, when the schedule asks for it.  One lane.
// ----------------------------------------------------------------------------------
__global__ void k_sample(const DevClock *__restrict__ clk, DevRun *__restrict__ run)
{
    if (threadIdx.x >= 9) return;
    const long long n = clk->step;
    if (run->sample_every <= 0 || n % run->sample_every != 0 || n < run->sample_first) return;
    const long long slot = (n - run->sample_first) / run->sample_every;
    if (slot >= run->sample_cap) return;
    run->samples[slot * 9 + threadIdx.x] = run->sigma_last[threadIdx.x];
}

// ----------------------------------------------------------------------------------
// k_unsort: state by particle id.  Completes u^n = vel + dt/2 F/m when vel holds the
// half-step velocity.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_unsort(DevParams P, const double4 *__restrict__ pa,
                                                    const double4 *__restrict__ vel, const double4 *__restrict__ omg,
                                                    const double4 *__restrict__ frc, const double4 *__restrict__ trq,
                                                    int vel_is_half, int complete, double *__restrict__ x,
                                                    double *__restrict__ u, double *__restrict__ w,
                                                    double *__restrict__ F, double *__restrict__ T)
{
#pragma clang fp contract(off)
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.N) return;
    double4 X = pa[p], V = vel[p], W = omg[p], Fp = frc[p], Tp = trq[p];
    int id = (int)W.w;
    if (vel_is_half && complete) {
        double m = pmass(P, X.w);
        double I = 0.4 * m * X.w * X.w;
        const double dt = P.dt;
        V.x = V.x + 0.5 * dt * (Fp.x / m);
        V.y = V.y + 0.5 * dt * (Fp.y / m);
        V.z = V.z + 0.5 * dt * (Fp.z / m);
        W.x = W.x + 0.5 * dt * (Tp.x / I);
        W.y = W.y + 0.5 * dt * (Tp.y / I);
        W.z = W.z + 0.5 * dt * (Tp.z / I);
    }
    if (x) { x[3 * id] = X.x; x[3 * id + 1] = X.y; x[3 * id + 2] = X.z; }
    if (u) { u[3 * id] = V.x; u[3 * id + 1] = V.y; u[3 * id + 2] = V.z; }
    if (w) { w[3 * id] = W.x; w[3 * id + 1] = W.y; w[3 * id + 2] = W.z; }
    if (F) { F[3 * id] = Fp.x; F[3 * id + 1] = Fp.y; F[3 * id + 2] = Fp.z; }
    if (T) { T[3 * id] = Tp.x; T[3 * id + 1] = Tp.y; T[3 * id + 2] = Tp.z; }
}

// k_load: particles by id -> unsorted records (slot = id).
__global__ void __launch_bounds__(kBlock) k_load(int N, const double *__restrict__ x, const double *__restrict__ rad,
                                                  const double *__restrict__ u, const double *__restrict__ w,
                                                  double gd, double4 *__restrict__ pa, double4 *__restrict__ vel,
                                                  double4 *__restrict__ omg, double4 *__restrict__ frc,
                                                  double4 *__restrict__ trq, int *__restrict__ inv)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    pa[p] = make_double4(x[3 * p], x[3 * p + 1], x[3 * p + 2], rad[p]);
    if (u)
        vel[p] = make_double4(u[3 * p], u[3 * p + 1], u[3 * p + 2], 0.0);
    else
        vel[p] = make_double4(gd * x[3 * p + 1], 0.0, 0.0, 0.0);
    if (w)
        omg[p] = make_double4(w[3 * p], w[3 * p + 1], w[3 * p + 2], (double)p);
    else
        omg[p] = make_double4(0.0, 0.0, -0.5 * gd, (double)p);
    frc[p] = make_double4(0.0, 0.0, 0.0, 0.0);
    trq[p] = make_double4(0.0, 0.0, 0.0, 0.0);
    inv[p] = p;
}

// k_history_export: rows -> (id_min, id_max, xi) list in canonical orientation.
__global__ void __launch_bounds__(kBlock) k_history_export(int N, int M, const int *__restrict__ own,
                                                            const int *__restrict__ key, const double *__restrict__ xi,
                                                            const int *__restrict__ cnt, long long cap,
                                                            int *__restrict__ out_pairs, double *__restrict__ out_xi,
                                                            unsigned long long *__restrict__ n_out)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    int id = own[p];
    int n = cnt[p];
    for (int k = 0; k < n; ++k) {
        int partner = key[(long long)p * M + k];
        unsigned long long s = atomicAdd(n_out, 1ull);
        if ((long long)s < cap) {
            out_pairs[2 * s] = id < partner ? id : partner;
            out_pairs[2 * s + 1] = id < partner ? partner : id;
            const double *x = xi + ((long long)p * M + k) * 3;
            out_xi[3 * s] = x[0];
            out_xi[3 * s + 1] = x[1];
            out_xi[3 * s + 2] = x[2];
        }
    }
}

}  // namespace dss
