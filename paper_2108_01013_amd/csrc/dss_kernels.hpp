// dss_kernels.hpp -- HIP kernels of one dense-suspension time step on CDNA4 (gfx950).
//
// Data layout (all in sorted order = cell-major order of the last counting sort):
//   pa  double4 [N]  (x, y, z, radius)
//   vel double4 [N]  (u_x, u_y, u_z, box): the velocity the last forces were evaluated with,
//                    and the index of the particle's box
//   omg double4 [N]  (w_x, w_y, w_z, id): angular velocity and the particle id (as a double)
//   force records: 6 doubles (F, T) per particle in six buffers (see ForceBufs)
// One 32-byte record per particle and quantity, so a neighbour gather is one 32-byte
// access per array; streaming kernels read them as two 16-byte loads per lane.
//
// Step kernels: k_predict (kick/drift, Lees-Edwards wrap, cell id, histogram rank),
// k_scan (exclusive scan of the counts), k_scatter (reorder), k_pairs (half-shell
// search + pair physics + history rows + stress), k_finish (stress and counters).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace dss {

constexpr double kPi = 3.14159265358979323846;
constexpr int kBlock = 256;

// error flag bits (device word)
constexpr unsigned kErrRowOverflow = 1u;
constexpr unsigned kErrNonFinite = 2u;
constexpr unsigned kErrPairBuffer = 4u;

// A history entry's key is the partner id (below 2^29) with bit 30 set when the contact's
// Coulomb cap was active at the step that wrote it and bit 29 when its rolling limit was (the
// stick/slip branch of the step, read by the adjoint).
constexpr int kKeyMask = 0x1fffffff;
constexpr int kRollCapBit = 0x20000000;
constexpr int kCapBit = 0x40000000;

// Physical constants and capacities shared by all boxes of a handle.
struct DevParams {
    double eta0, rho, kn, kt, gn, mu, fer, lamd, a0, ham, eps_vdw, eps_lub, cf, dt;
    double k6, k8;     // 6 pi eta0, 8 pi eta0
    double inv_lamd;   // 1 / lambda_D (0 if lambda_D <= 0)
    double fer_a0;     // F_ER / a0
    int nbox;          // number of independent boxes
    int N;             // particles over all boxes
    int M;             // history row capacity
    int record_pairs;
    long long pair_cap;
    int own_cap, stage_cap, qcap;   // row-tile capacities of k_pairs
    int tiled;                      // 0: every row takes the per-particle path
    int pstride;                    // stride of the partial records (1024 R)
    int sized;                      // 1: size-class stencils (class-major cell numbering)
    int ncls;                       // size classes (stencil radius of class k: k + 1 cells)
    int wave_cls;                   // classes from this one up take a wavefront per particle
    double cls_mul, cls_add;        // class of radius a: floor(a cls_mul + cls_add)
    int ec;                         // 1: electro-chemical forces over their own ranges
    double rext;                    // with ec: longest active range (pair set |r| < max(c s, s + rext))
    double rep_rng, att_rng;        // with ec: surface-distance ranges of repulsion and attraction
    double kr, mu_r;                // rolling spring stiffness and Coulomb coefficient (kr = 0: off)
    double inv_kt, inv_kr;          // 1 / kt, 1 / kr (0 when the spring is off)
    double wave_amp;                // amplitude W of the wavy shear, eq. uinf (0: simple shear)
    int ec_split;                   // with ec: the lattice and the pair kernels cover the lubrication
                                    //   list c (a_i + a_j); k_pairs_ec takes the pairs beyond it
    int ec_ry, ec_rz;               // with ec_split: reach of k_pairs_ec in cell rows along y and z
    double ec_amax;                 // with ec_split: largest radius
    float pf_m2;                    // margin on r^2 of the FP32 candidate pre-test of k_pairs
};

// One box: its geometry, shear rate, cell lattice and its ranges in the global numbering
// (cells, cell rows and particle ids of all boxes are numbered box after box, so one
// counting sort orders every box and each box is a contiguous range of sorted slots).
struct BoxParams {
    double L[3];       // box lengths
    double gd;         // shear rate
    double cw[3];      // cell widths L / nc
    int nc[3];         // cells per dimension
    int cell_off;      // first cell of the box
    int row_off;       // first cell row (nc[1] nc[2] rows per box)
    int part_off;      // first particle id of the box
    int n_part;        // particles of the box
    int nrec;          // stress partial records of the box (from row_off; its cell rows when tiled)
    double wk;         // wave number 2 pi n / L_y of the wavy shear
};

// Device-side clock and error flags.  step = time index of the state.
struct DevClock {
    long long step;
    unsigned err;
    int deferred;   // 1: the atomic force record is in use (rows of k_pairs on the per-particle
                    // path, size-class stencils); cleared by k_scatter
};

// Run descriptor of a dss_step call: stress sampling schedule.
struct DevRun {
    long long sample_every;   // 0: no sampling
    long long sample_first;   // first sampled time index of this call
    long long sample_cap;     // number of sample slots
    double *samples;          // sample_cap x nbox x 9
    double *sigma_last;       // nbox x 9: pair part of the stress of the last evaluation
    double *box_diag;         // nbox x 3: listed pairs, contacts, largest history row
};

// ----------------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------------
__device__ __forceinline__ double le_offset(const DevParams &P, const BoxParams &G, long long step)
{
#pragma clang fp contract(off)
    double t = (double)step * P.dt;
    double s = G.gd * G.L[1] * t;
    return fmod(s, G.L[0]);
}

__device__ __forceinline__ int cell_coord(double xd, double cw, int n)
{
    int c = (int)(xd / cw);
    c = c < 0 ? 0 : c;
    c = c > n - 1 ? n - 1 : c;
    return c;
}

// Local shear rate dU/dy of the ambient flow at height y: gdot, plus W k cos(k y) in the
// wavy shear U_inf = (gdot y + W sin(k y), 0, 0) of eq. uinf.
__device__ __forceinline__ double shear_at(const DevParams &P, double gd, double wk, double y)
{
    return P.wave_amp != 0.0 ? gd + P.wave_amp * wk * cos(wk * y) : gd;
}

// Size class of radius a under size-class stencils (stencil radius class + 1 cells).
__device__ __forceinline__ int size_class(const DevParams &P, double a)
{
#pragma clang fp contract(off)
    const int k = (int)floor(a * P.cls_mul + P.cls_add);
    return k < 0 ? 0 : (k > P.ncls - 1 ? P.ncls - 1 : k);
}

// Nearest image of b seen from a under Lees-Edwards shear; r = x_b - x_a.  Rows above /
// below are displaced by +delta / -delta along x.  Periodic wraps by comparison: for every
// pair closer than L/2 along x and z this equals r - L round(r / L) bit for bit (the
// subtractions of L and 2 L are exact by Sterbenz's lemma), so the listed-pair test is the
// IEEE expression as written.  Evaluated without contraction.
__device__ __forceinline__ void min_image(const BoxParams &P, double delta, double xa, double ya, double za,
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
    const double hx = 0.5 * P.L[0];
    if (dx > hx) {
        dx -= P.L[0];
        if (dx > hx) dx -= P.L[0];
    } else if (dx < -hx) {
        dx += P.L[0];
        if (dx < -hx) dx += P.L[0];
    }
    if (dz > 0.5 * P.L[2])
        dz -= P.L[2];
    else if (dz < -0.5 * P.L[2])
        dz += P.L[2];
}

__device__ __forceinline__ bool listed(const DevParams &P, double dx, double dy, double dz, double aa, double ab,
                                       double &r2)
{
#pragma clang fp contract(off)
    r2 = (dx * dx + dy * dy) + dz * dz;
    double rc = P.cf * (aa + ab);
    if (P.ec && !P.ec_split) rc = fmax(rc, (aa + ab) + P.rext);
    return r2 < rc * rc;
}

__device__ __forceinline__ double pmass(const DevParams &P, double a)
{
#pragma clang fp contract(off)
    return P.rho * (4.0 / 3.0) * kPi * a * a * a;
}

// 1/x from the hardware reciprocal refined by two Newton steps (relative error ~1e-16);
// used in the pair physics only, never in the listed-pair test.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
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
// Force records.  The totals of one evaluation are the sum of six 48-byte records per
// particle (sorted order): the workgroup that owns the particle's cell row writes its own
// part (own row pairs + Stokes terms), and for each of the four other rows of the half
// shell exactly one workgroup writes the partner-side part it accumulated (nb[0..3]);
// ft_x receives atomic additions only from rows evaluated by the per-particle path.
// All plain stores: no atomics on the hot path, every record written every evaluation.
// ----------------------------------------------------------------------------------
struct ForceBufs {
    double *own;     // N x 6
    double *nb;      // 4 x N x 6
    double *x;       // N x 6, atomic accumulation, cleared by k_predict after use
    long long n;     // N (stride of nb)
    int nnb;         // partner records in use (4 on the row tiles, 0 with size-class stencils)
};

__device__ __forceinline__ void load_ft(const double *__restrict__ rec, double f[6])
{
    const double2 *q = reinterpret_cast<const double2 *>(rec);
    double2 a = q[0], b = q[1], c = q[2];
    f[0] = a.x; f[1] = a.y; f[2] = b.x; f[3] = b.y; f[4] = c.x; f[5] = c.y;
}

__device__ __forceinline__ void store_ft(double *__restrict__ rec, const double f[6])
{
    double2 *q = reinterpret_cast<double2 *>(rec);
    q[0] = make_double2(f[0], f[1]);
    q[1] = make_double2(f[2], f[3]);
    q[2] = make_double2(f[4], f[5]);
}

// Total force (f[0..2]) and torque (f[3..5]) of slot p, summed in a fixed order.  with_x = 0
// leaves out the atomic record (all zero when no row took the per-particle path).
__device__ __forceinline__ void total_ft(const ForceBufs &B, int p, double f[6], bool with_x = true)
{
    double a[6];
    load_ft(B.own + 6LL * p, f);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r >= B.nnb) break;
        load_ft(B.nb + 6LL * (r * B.n + p), a);
#pragma unroll
        for (int k = 0; k < 6; ++k) f[k] += a[k];
    }
    if (!with_x) return;
    load_ft(B.x + 6LL * p, a);
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k] += a[k];
}

// ----------------------------------------------------------------------------------
// k_scan: exclusive scan of the cell counts by one workgroup of 1024 lanes, cell_start =
// exscan(count), count reset to 0, clock advanced.  The counts are read as C4 tiles of
// 1024 int4 chunks (lane t holds chunk k 1024 + t of every tile k: each load instruction
// of a wavefront covers one contiguous KB).  Prefix of a chunk = totals of the earlier
// tiles + the lanes before it in its tile (wavefront shuffles, then the 16 wavefront
// totals through LDS).  count and cell_start are padded to 4096 C4 entries (padding
// counts stay 0), so the entry at index n_cells receives the total.
// Lattices beyond one workgroup (many boxes): each workgroup scans its own 4096 C4 counts
// and leaves its total in tile_sum; k_scan_add then adds the totals of the earlier
// workgroups and advances the clock.
// ----------------------------------------------------------------------------------
template <int C4>
__global__ void __launch_bounds__(1024) k_scan(int *__restrict__ count, int *__restrict__ cell_start,
                                               DevClock *__restrict__ clk, int advance, int *__restrict__ tile_sum)
{
    static_assert(C4 >= 1 && C4 <= 16, "one wavefront scans at most 256 wavefront totals");
    __shared__ int wsum[C4][16];
    __shared__ int wpre[C4][16];
    const int t = threadIdx.x;
    const int lane = t & 63, wid = t >> 6;
    int4 *cnt4 = reinterpret_cast<int4 *>(count) + (size_t)blockIdx.x * (C4 * 1024);
    int4 *out4 = reinterpret_cast<int4 *>(cell_start) + (size_t)blockIdx.x * (C4 * 1024);
    int4 v[C4];
#pragma unroll
    for (int k = 0; k < C4; ++k) v[k] = cnt4[k * 1024 + t];
    int s[C4], incl[C4];
#pragma unroll
    for (int k = 0; k < C4; ++k) {
        s[k] = v[k].x + v[k].y + v[k].z + v[k].w;
        incl[k] = s[k];
    }
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int k = 0; k < C4; ++k) {
            const int u = __shfl_up(incl[k], o, 64);
            if (lane >= o) incl[k] += u;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < C4; ++k) wsum[k][wid] = incl[k];
    }
    __syncthreads();
    if (wid == 0) {
        // prefix of the C4 x 16 wavefront totals (flat order k 16 + w): four per lane, then
        // one wavefront scan of the lane sums
        const int *ws = &wsum[0][0];
        int *wp = &wpre[0][0];
        int loc[4], sum = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = 4 * lane + e;
            loc[e] = q < C4 * 16 ? ws[q] : 0;
            sum += loc[e];
        }
        int incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        int run = incl - sum;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = 4 * lane + e;
            if (q < C4 * 16) wp[q] = run;
            run += loc[e];
        }
        if (tile_sum && lane == 63) tile_sum[blockIdx.x] = incl;
    }
    __syncthreads();
    const int4 zero = make_int4(0, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < C4; ++k) {
        int4 o;
        o.x = wpre[k][wid] + incl[k] - s[k];
        o.y = o.x + v[k].x;
        o.z = o.y + v[k].y;
        o.w = o.z + v[k].z;
        out4[k * 1024 + t] = o;
        cnt4[k * 1024 + t] = zero;
    }
    if (t == 0 && advance && !tile_sum) clk->step += 1;
}

// Second pass of the multi-workgroup scan: workgroup b adds the totals of workgroups
// 0 .. b-1 to its chunk of cell_start (chunks int4 entries per workgroup).
__global__ void __launch_bounds__(1024) k_scan_add(int *__restrict__ cell_start, const int *__restrict__ tile_sum,
                                                   int chunks, DevClock *__restrict__ clk, int advance)
{
    __shared__ int red[16];
    const int t = threadIdx.x, b = blockIdx.x;
    if (b == 0) {
        if (t == 0 && advance) clk->step += 1;
        return;
    }
    int part = 0;
    for (int k = t; k < b; k += 1024) part += tile_sum[k];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((t & 63) == 0) red[t >> 6] = part;
    __syncthreads();
    int off = 0;
    for (int w = 0; w < 16; ++w) off += red[w];
    int4 *out4 = reinterpret_cast<int4 *>(cell_start) + (size_t)b * chunks;
    for (int k = t; k < chunks; k += 1024) {
        int4 v = out4[k];
        v.x += off;
        v.y += off;
        v.z += off;
        v.w += off;
        out4[k] = v;
    }
}

// ----------------------------------------------------------------------------------
// k_predict: velocity-Verlet drift + half kick (advance = 1) or velocity completion
// only (advance = 0), Lees-Edwards wrap at t_{n+1}, cell id and histogram rank.
//   vel_is_half = 1: vel holds the half-step velocity u^{n-1/2} of the forces, and
//   u^n = u^{n-1/2} + dt/2 F^n / m completes the previous step.
// The atomic force record is read, and cleared for the next evaluation, only when the last
// evaluation took rows on the per-particle path (clk->deferred > 0) or k_pairs_ec wrote
// it (ec_split); otherwise it is already zero.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_predict(DevParams P, const BoxParams *__restrict__ boxes,
                                                     double4 *__restrict__ pa, double4 *__restrict__ vel,
                                                     double4 *__restrict__ omg, ForceBufs B, int vel_is_half,
                                                     int advance, const DevClock *__restrict__ clk,
                                                     int *__restrict__ cell, int *__restrict__ rank,
                                                     int *__restrict__ count, int *__restrict__ img, BoxParams G0,
                                                     unsigned long long *__restrict__ pair_count,
                                                     double *__restrict__ tx, double *__restrict__ tu,
                                                     double *__restrict__ tw, int *__restrict__ tz)
{
#pragma clang fp contract(off)
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && pair_count) *pair_count = 0;  // the pairs this step's pair kernels record
    if (tz && p < P.N) tz[p] = 0;  // counts the adjoint's tape fills after this evaluation
    const bool active = p < P.N;
    int c = -1;
    if (active) {
    double4 X = pa[p];
    double4 V = vel[p];
    double4 W = omg[p];
    if (tx) {
        // the state as read, by id (the adjoint's tape of the previous evaluation)
        const long long id = (long long)W.w;
        tx[3 * id] = X.x; tx[3 * id + 1] = X.y; tx[3 * id + 2] = X.z;
        tu[3 * id] = V.x; tu[3 * id + 1] = V.y; tu[3 * id + 2] = V.z;
        tw[3 * id] = W.x; tw[3 * id + 1] = W.y; tw[3 * id + 2] = W.z;
    }
    // the box of the particle: the table entry of a batch, else the kernel argument (no
    // load that waits for the particle record)
    auto body = [&](const BoxParams &G) {
    const double dt = P.dt;
    double a = X.w;
    double m = pmass(P, a);
    double I = 0.4 * m * a * a;
    double f[6];
    total_ft(B, p, f, false);
    if (clk->deferred || P.ec_split) {
        double e[6];
        load_ft(B.x + 6LL * p, e);
#pragma unroll
        for (int k = 0; k < 6; ++k) f[k] += e[k];
        const double z[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        store_ft(B.x + 6LL * p, z);
    }
    double ax = f[0] / m, ay = f[1] / m, az = f[2] / m;
    double bx = f[3] / I, by = f[4] / I, bz = f[5] / I;
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
        double delta = le_offset(P, G, clk->step + 1);
        if (X.y >= G.L[1]) {
            X.y -= G.L[1];
            X.x -= delta;
            V.x -= G.gd * G.L[1];
            img[(int)W.w] += 1;  // y-face crossings, for the unwrapped shear-wise position
        } else if (X.y < 0.0) {
            X.y += G.L[1];
            X.x += delta;
            V.x += G.gd * G.L[1];
            img[(int)W.w] -= 1;
        }
        X.x -= G.L[0] * floor(X.x / G.L[0]);
        X.z -= G.L[2] * floor(X.z / G.L[2]);
        pa[p] = X;
    }
    vel[p] = V;
    omg[p] = W;
    int cx = cell_coord(X.x, G.cw[0], G.nc[0]);
    int cy = cell_coord(X.y, G.cw[1], G.nc[1]);
    int cz = cell_coord(X.z, G.cw[2], G.nc[2]);
    c = G.cell_off + (cz * G.nc[1] + cy) * G.nc[0] + cx;
    if (P.sized) c += size_class(P, X.w) * (G.nc[0] * G.nc[1] * G.nc[2]);
    };
    if (P.nbox > 1)
        body(boxes[(int)V.w]);
    else
        body(G0);
    }
    // histogram rank: lanes of a wavefront with equal consecutive cell ids (the input is
    // sorted by the previous step's cells) form runs; the first lane of a run claims the
    // run's slots with one atomic and the others take consecutive ranks
    const int lane = threadIdx.x & 63;
    const int cprev = __shfl_up(c, 1, 64);
    const unsigned long long starts = __ballot(lane == 0 || c != cprev);
    const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int rs = 63 - __clzll(starts & upto);
    const unsigned long long after = starts & ~upto;
    const int re = after ? __ffsll((long long)after) - 1 : 64;
    int base = 0;
    if (active && lane == rs) base = atomicAdd(&count[c], re - rs);
    base = __shfl(base, rs, 64);
    if (active) {
        cell[p] = c;
        rank[p] = base + (lane - rs);
    }
}

// k_complete: vel <- u^n = u^{n-1/2} + dt/2 F^n/m in place (an evaluation at the current
// state, without a re-sort).
__global__ void __launch_bounds__(kBlock) k_complete(DevParams P, const double4 *__restrict__ pa,
                                                      double4 *__restrict__ vel, double4 *__restrict__ omg,
                                                      ForceBufs B)
{
#pragma clang fp contract(off)
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.N) return;
    const double a = pa[p].w;
    const double m = pmass(P, a);
    const double I = 0.4 * m * a * a;
    const double dt = P.dt;
    double f[6];
    total_ft(B, p, f);
    double4 V = vel[p];
    double4 W = omg[p];
    V.x = V.x + 0.5 * dt * (f[0] / m);
    V.y = V.y + 0.5 * dt * (f[1] / m);
    V.z = V.z + 0.5 * dt * (f[2] / m);
    W.x = W.x + 0.5 * dt * (f[3] / I);
    W.y = W.y + 0.5 * dt * (f[4] / I);
    W.z = W.z + 0.5 * dt * (f[5] / I);
    vel[p] = V;
    omg[p] = W;
}

// ----------------------------------------------------------------------------------
// k_scatter: move every particle to its sorted slot, remember its previous slot (where
// its contact-history row of the last step lives).
// With ntile > 0 (at most 16 tiles of 4096 cells) the counts were scanned tile by tile in
// parallel (cs_local, tile totals in tile_sum): every workgroup forms the tile offsets
// (one wavefront scan), slots are cs_local + offset, the workgroups write the final
// cell_start over a grid stride, and the clock advances here.  With ntile = 0 cs_local is
// the final cell_start.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_scatter(int N, const int *__restrict__ cell, const int *__restrict__ rank,
                                                     const int *__restrict__ cs_local,
                                                     const int *__restrict__ tile_sum, int ntile, int ncell1,
                                                     int *__restrict__ cell_start, DevClock *__restrict__ clk,
                                                     int advance, const double4 *__restrict__ pa_in,
                                                     const double4 *__restrict__ vel_in,
                                                     const double4 *__restrict__ omg_in, double4 *__restrict__ pa_out,
                                                     double4 *__restrict__ vel_out, double4 *__restrict__ omg_out,
                                                     int *__restrict__ prev)
{
    __shared__ int off[16];
    const int t = threadIdx.x;
    if (blockIdx.x == 0 && t == 0) clk->deferred = 0;  // set again by the rows of this step's pair kernels
    if (ntile > 0) {
        if (t < 64) {
            const int v = t < ntile ? tile_sum[t] : 0;
            int incl = v;
            for (int o = 1; o < 16; o <<= 1) {
                const int u = __shfl_up(incl, o, 64);
                if ((t & 63) >= o) incl += u;
            }
            if (t < 16) off[t] = incl - v;
        }
        __syncthreads();
        if (blockIdx.x == 0 && t == 0 && advance) clk->step += 1;
        for (int q = blockIdx.x * blockDim.x + t; q < ncell1; q += gridDim.x * blockDim.x)
            cell_start[q] = cs_local[q] + off[q >> 12];
    }
    int p = blockIdx.x * blockDim.x + t;
    if (p >= N) return;
    const int c = cell[p];
    int dst = (ntile > 0 ? cs_local[c] + off[c >> 12] : cs_local[c]) + rank[p];
    pa_out[dst] = pa_in[p];
    vel_out[dst] = vel_in[p];
    omg_out[dst] = omg_in[p];
    prev[dst] = p;
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
    double xi[3];   // new tangential stretch, oriented i -> j
    double xr[3];   // new rolling stretch (no orientation), with rolling resistance
    bool contact;
    bool capped;    // the Coulomb cap rescaled the stretch
    bool rcapped;   // the rolling limit rescaled the rolling stretch
};

// Arithmetic of the pair physics in type Real: double (FP64 mode) or float (mixed mode).
__device__ __forceinline__ double rcp_r(double x) { return rcp_nr(x); }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double log_r(double x) { return log(x); }
__device__ __forceinline__ float log_r(float x) { return __logf(x); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
__device__ __forceinline__ float exp_r(float x) { return __expf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_sqrtf(x); }

// Pair physics.  In FP64 mode (Real = double) everything is FP64.  In mixed mode (Real =
// float) the gap h, the lubrication argument d* + eps and its reciprocal, and the velocity
// differences (which cancel the large ambient-flow values) are formed in FP64 and rounded
// once; the unit vector, coefficients, log/exp, contact model and stresslet are FP32; the
// results are accumulated in FP64 by the caller.
template <typename Real, bool Roll = false, bool Wave = false>
__device__ __forceinline__ void pair_physics(const DevParams &P, double gd_d, double wk, double dx_d, double dy_d,
                                             double dz_d, double dist,
                                             double ai_d, double aj_d, double yi, double yj, const double4 &Vi,
                                             const double4 &Vj, const double4 &Wi, const double4 &Wj,
                                             const double xo[3], const double xro[3], double *S, PairOut &o)
{
    // ---------------- FP64 in both modes: gap, lubrication argument, velocity differences
    const double h_d = dist - ai_d - aj_d;
    const double s_d = ai_d + aj_d;
    double dstar = 2.0 * h_d / s_d;
    dstar = dstar > 0.0 ? dstar : 0.0;
    const double g_d = dstar + P.eps_lub;
    Real invg = (Real)rcp_nr(g_d);
    Real lg = -log_r((Real)g_d);
    // electro-chemical ranges: the list reaches beyond the lubrication range, where every
    // lubrication coefficient is zero; each electro-chemical force has its own range
    bool rep_on = true, att_on = true;
    if (P.ec) {
#pragma clang fp contract(off)
        const double r2 = (dx_d * dx_d + dy_d * dy_d) + dz_d * dz_d;
        const double rl = P.cf * s_d;
        if (!(r2 < rl * rl)) {
            invg = (Real)0.0;
            lg = (Real)0.0;
        }
        rep_on = h_d < P.rep_rng;
        att_on = h_d < P.att_rng;
    }
    // wavy shear: the ambient flow, rotation and strain at each particle's own height
    constexpr bool wavy = Wave;
    double si = gd_d, sj = gd_d, wvi = 0.0, wvj = 0.0;
    double uxi = Vi.x - gd_d * yi, uxj = Vj.x - gd_d * yj;
    if (wavy) {
        si = shear_at(P, gd_d, wk, yi);
        sj = shear_at(P, gd_d, wk, yj);
        wvi = P.wave_amp * sin(wk * yi);
        wvj = P.wave_amp * sin(wk * yj);
        uxi -= wvi;
        uxj -= wvj;
    }
    const Real dux = (Real)(uxj - uxi);
    const Real duy = (Real)(Vj.y - Vi.y);
    const Real duz = (Real)(Vj.z - Vi.z);
    const Real h = (Real)h_d;

    // ---------------- type Real from here
    const Real dx = (Real)dx_d, dy = (Real)dy_d, dz = (Real)dz_d;
    const Real inv_d = rcp_r((Real)dist);
    const Real nx = dx * inv_d, ny = dy * inv_d, nz = dz * inv_d;
    const Real ai = (Real)ai_d, aj = (Real)aj_d;
    const Real s = ai + aj;
    const Real gd = (Real)gd_d;
    const Real gbar = wavy ? (Real)(0.5 * (si + sj)) : gd;  // shear of the mean strain (E_i + E_j) / 2
    const Real wix = (Real)Wi.x, wiy = (Real)Wi.y, wiz = (Real)(Wi.z + 0.5 * si);
    const Real wjx = (Real)Wj.x, wjy = (Real)Wj.y, wjz = (Real)(Wj.z + 0.5 * sj);

    // ---------------- lubrication
    const Real K = (Real)P.k6;
    const Real ai2 = ai * ai, aj2 = aj * aj;
    const Real is = rcp_r(s);
    const Real is2 = is * is, is3 = is2 * is;
    const Real XA = K * (Real)2.0 * ai2 * aj2 * is3 * invg;
    const Real YA = K * (Real)(4.0 / 15.0) * ai * aj * ((Real)2.0 * ai2 + ai * aj + (Real)2.0 * aj2) * is3 * lg;
    const Real YBi = -K * (Real)(2.0 / 15.0) * ai2 * aj * ((Real)4.0 * ai + aj) * is2 * lg;
    const Real YBj = K * (Real)(2.0 / 15.0) * ai * aj2 * (ai + (Real)4.0 * aj) * is2 * lg;
    const Real YCii = K * (Real)(8.0 / 15.0) * ai2 * ai * aj * is * lg;
    const Real YCij = K * (Real)(2.0 / 15.0) * ai2 * aj2 * is * lg;
    const Real YCjj = K * (Real)(8.0 / 15.0) * ai * aj2 * aj * is * lg;
    // v = du + s E n, E n = gd/2 (n_y, n_x, 0) (the mean strain in the wavy shear)
    const Real vx = dux + s * (Real)0.5 * gbar * ny;
    const Real vy = duy + s * (Real)0.5 * gbar * nx;
    const Real vz = duz;
    const Real vn = vx * nx + vy * ny + vz * nz;
    // n x w'
    const Real cix = ny * wiz - nz * wiy, ciy = nz * wix - nx * wiz, ciz = nx * wiy - ny * wix;
    const Real cjx = ny * wjz - nz * wjy, cjy = nz * wjx - nx * wjz, cjz = nx * wjy - ny * wjx;
    const Real FLx = XA * vn * nx + YA * (vx - vn * nx) - YBi * cix + YBj * cjx;
    const Real FLy = XA * vn * ny + YA * (vy - vn * ny) - YBi * ciy + YBj * cjy;
    const Real FLz = XA * vn * nz + YA * (vz - vn * nz) - YBi * ciz + YBj * cjz;
    // n x v
    const Real nvx = ny * vz - nz * vy, nvy = nz * vx - nx * vz, nvz = nx * vy - ny * vx;
    // T w' = w' - (w'.n) n
    const Real win = wix * nx + wiy * ny + wiz * nz;
    const Real wjn = wjx * nx + wjy * ny + wjz * nz;
    const Real tix = wix - win * nx, tiy = wiy - win * ny, tiz = wiz - win * nz;
    const Real tjx = wjx - wjn * nx, tjy = wjy - wjn * ny, tjz = wjz - wjn * nz;
    Real Ti0 = -YBi * nvx - YCii * tix - YCij * tjx;
    Real Ti1 = -YBi * nvy - YCii * tiy - YCij * tjy;
    Real Ti2 = -YBi * nvz - YCii * tiz - YCij * tjz;
    Real Tj0 = YBj * nvx - YCij * tix - YCjj * tjx;
    Real Tj1 = YBj * nvy - YCij * tiy - YCjj * tjy;
    Real Tj2 = YBj * nvz - YCij * tiz - YCjj * tjz;
    Real FLxw = FLx, FLyw = FLy, FLzw = FLz;
    if (wavy) {
        // strain difference D = (E_j - E_i) / 2, D_xy = (s_j - s_i) / 4: the columns of R'(E)
        // taken at their own particles differ from the mean-strain form by
        //   dF_i = (X^G_ji - X^G_ii) P(D) n + (Y^G_ji - Y^G_ii) Q(D) n = -dF_j,
        //   dT_i = (Y^H_ji - Y^H_ii) n_perp(D),  dT_j = (Y^H_jj - Y^H_ij) n_perp(D),
        // with the coefficient differences of the Appendix A table in a_i, alpha = a_j / a_i
        const Real d = (Real)(0.25 * (sj - si));
        const Real Dnx = d * ny, Dny = d * nx;                   // D n
        const Real PD = (Real)2.0 * d * nx * ny;                 // n.D.n (Tr D = 0)
        const Real QDx = (Real)2.0 * (Dnx - PD * nx), QDy = (Real)2.0 * (Dny - PD * ny), QDz = (Real)-2.0 * PD * nz;
        const Real pnx = (Real)2.0 * (-nz * Dny), pny = (Real)2.0 * (nz * Dnx), pnz = (Real)2.0 * (nx * Dny - ny * Dnx);
        const Real al = aj * rcp_r(ai), op = (Real)1.0 + al;
        const Real op2 = op * op, op3 = op2 * op;
        const Real dXG = K * (Real)2.0 * ai2 * aj2 * (aj - ai) * is3 * invg;
        const Real dYG = K * (Real)(4.0 / 15.0) * ai2 * al * (al - (Real)1.0) * (al * al - al + (Real)1.0) *
                         rcp_r(op3) * lg;
        const Real a3 = ai2 * ai;
        const Real dHi = K * (Real)(1.0 / 15.0) * a3 * al * (al * al + (Real)9.0 * al - (Real)4.0) * rcp_r(op2) * lg;
        const Real dHj = K * (Real)(1.0 / 15.0) * a3 * al * al * ((Real)4.0 * al * al - (Real)9.0 * al - (Real)1.0) *
                         rcp_r(op2) * lg;
        FLxw += dXG * PD * nx + dYG * QDx;
        FLyw += dXG * PD * ny + dYG * QDy;
        FLzw += dXG * PD * nz + dYG * QDz;
        Ti0 += dHi * pnx;
        Ti1 += dHi * pny;
        Ti2 += dHi * pnz;
        Tj0 += dHj * pnx;
        Tj1 += dHj * pny;
        Tj2 += dHj * pnz;
    }

    // ---------------- electro-chemical (central): repulsion eq. rep, attraction eq. att
    const Real abar = (Real)2.0 * ai * aj * is;
    Real fe = (Real)0.0;
    if (P.fer != 0.0 && rep_on)
        fe -= (Real)P.fer_a0 * abar *
              (h >= (Real)0.0 ? (P.lamd > 0.0 ? exp_r(-h * (Real)P.inv_lamd) : (Real)0.0) : (Real)1.0);
    if (P.ham != 0.0 && att_on) {
        const Real e = (Real)P.eps_vdw * abar;
        fe += (Real)P.ham * abar * rcp_r((Real)12.0 * ((h >= (Real)0.0 ? h * h : (Real)0.0) + e * e));
    }

    // ---------------- contact eqs. contact0, csi
    Real FCx = 0, FCy = 0, FCz = 0;
    o.contact = h_d < 0.0;
    o.capped = false;
    o.rcapped = false;
    o.xi[0] = o.xi[1] = o.xi[2] = 0.0;
    if (o.contact) {
        // true relative velocity of the image pair: ambient difference gd r_y along x
        // (plus the wave's difference at the two heights)
        const Real Dx = dux + gd * dy + (Real)(wvj - wvi), Dy = duy, Dz = duz;
        const Real un = Dx * nx + Dy * ny + Dz * nz;
        const Real fn = (Real)P.kn * h + (Real)P.gn * un;
        const Real Fnx = fn * nx, Fny = fn * ny, Fnz = fn * nz;
        const Real sx = (Real)(ai_d * Wi.x + aj_d * Wj.x), sy = (Real)(ai_d * Wi.y + aj_d * Wj.y),
                   sz = (Real)(ai_d * Wi.z + aj_d * Wj.z);
        // (a_i w_i + a_j w_j) x n
        const Real qx = sy * nz - sz * ny, qy = sz * nx - sx * nz, qz = sx * ny - sy * nx;
        const Real tx = Dx - qx, ty = Dy - qy, tz = Dz - qz;
        const Real tn = tx * nx + ty * ny + tz * nz;
        const Real dtR = (Real)P.dt;
        Real xx = (Real)xo[0] + (tx - tn * nx) * dtR;
        Real xy = (Real)xo[1] + (ty - tn * ny) * dtR;
        Real xz = (Real)xo[2] + (tz - tn * nz) * dtR;
        const Real xn = xx * nx + xy * ny + xz * nz;
        xx -= xn * nx;
        xy -= xn * ny;
        xz -= xn * nz;
        Real Ftx = 0, Fty = 0, Ftz = 0;
        if (P.kt > 0.0) {
            const Real cap = (Real)P.mu * fabs(fn) * (Real)P.inv_kt;
            const Real xm = sqrt_r(xx * xx + xy * xy + xz * xz);
            if (xm >= cap && xm > (Real)0.0) {
                o.capped = true;
                const Real sc = cap * rcp_r(xm);
                xx *= sc;
                xy *= sc;
                xz *= sc;
            }
            Ftx = (Real)P.kt * xx;
            Fty = (Real)P.kt * xy;
            Ftz = (Real)P.kt * xz;
        } else {
            xx = xy = xz = 0;
        }
        o.xi[0] = xx;
        o.xi[1] = xy;
        o.xi[2] = xz;
        FCx = Fnx + Ftx;
        FCy = Fny + Fty;
        FCz = Fnz + Ftz;
        // T_i = a_i n x F_t, T_j = a_j n x F_t
        const Real mx = ny * Ftz - nz * Fty, my = nz * Ftx - nx * Ftz, mz = nx * Fty - ny * Ftx;
        Ti0 += ai * mx;
        Ti1 += ai * my;
        Ti2 += ai * mz;
        Tj0 += aj * mx;
        Tj1 += aj * my;
        Tj2 += aj * mz;
        if constexpr (Roll) {
            // rolling resistance (Appendix roll): a second spring on the rolling velocity
            // u_r = a_ij n x (w_i - w_j), a_ij = abar; the same Coulomb limitation with mu_r;
            // torques T_i = a_ij n x k_r xi^r, T_j = -T_i, no force, no stress
            const Real dwx = (Real)(Wi.x - Wj.x), dwy = (Real)(Wi.y - Wj.y), dwz = (Real)(Wi.z - Wj.z);
            const Real urx = abar * (ny * dwz - nz * dwy), ury = abar * (nz * dwx - nx * dwz),
                       urz = abar * (nx * dwy - ny * dwx);
            Real rx = (Real)xro[0] + urx * dtR, ry = (Real)xro[1] + ury * dtR, rz = (Real)xro[2] + urz * dtR;
            const Real rn = rx * nx + ry * ny + rz * nz;
            rx -= rn * nx;
            ry -= rn * ny;
            rz -= rn * nz;
            const Real capr = (Real)P.mu_r * fabs(fn) * (Real)P.inv_kr;
            const Real rm = sqrt_r(rx * rx + ry * ry + rz * rz);
            if (rm >= capr && rm > (Real)0.0) {
                const Real sc = capr * rcp_r(rm);
                rx *= sc;
                ry *= sc;
                rz *= sc;
                o.rcapped = true;
            }
            o.xr[0] = rx;
            o.xr[1] = ry;
            o.xr[2] = rz;
            const Real frx = (Real)P.kr * rx, fry = (Real)P.kr * ry, frz = (Real)P.kr * rz;
            const Real qrx = abar * (ny * frz - nz * fry), qry = abar * (nz * frx - nx * frz),
                       qrz = abar * (nx * fry - ny * frx);
            Ti0 += qrx;
            Ti1 += qry;
            Ti2 += qrz;
            Tj0 -= qrx;
            Tj1 -= qry;
            Tj2 -= qrz;
        }
    }
    const Real Fex = fe * nx, Fey = fe * ny, Fez = fe * nz;
    o.Fi[0] = FLxw + FCx + Fex;
    o.Fi[1] = FLyw + FCy + Fey;
    o.Fi[2] = FLzw + FCz + Fez;
    o.Ti[0] = Ti0;
    o.Ti[1] = Ti1;
    o.Ti[2] = Ti2;
    o.Tj[0] = Tj0;
    o.Tj[1] = Tj1;
    o.Tj[2] = Tj2;
    // stresslet r (x) F_i of the pair, the lubrication part symmetrised (eq. stresslet)
    {
        const Real r[3] = {dx, dy, dz};
        const Real FL[3] = {FLxw, FLyw, FLzw};
        const Real FO[3] = {FCx + Fex, FCy + Fey, FCz + Fez};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) S[3 * a + b] += (double)((Real)0.5 * (r[a] * FL[b] + r[b] * FL[a]) + r[a] * FO[b]);
    }
}

// ----------------------------------------------------------------------------------
// History lookup (Sec. 2.1, memory paragraph: a stored stretch is sought over the sorted row).
// The row of the particle at sorted slot p of the previous evaluation holds n = hcnt[p]
// entries sorted by partner id.  The first kRowHead keys are read together with the count
// (independent loads, in flight at once, clamped into the row's capacity); a key beyond them,
// in a row longer than kRowHead, is found by bisection over the sorted rest.
// ----------------------------------------------------------------------------------
constexpr int kRowHead = 8;

struct RowHead {
    int n;
    int key[kRowHead];
};

__device__ __forceinline__ void row_head(const int *__restrict__ hkey, const int *__restrict__ hcnt, int M, int p,
                                         RowHead &r)
{
    const int *kr = hkey + (long long)p * M;
#pragma unroll
    for (int k = 0; k < kRowHead; ++k) r.key[k] = kr[k < M ? k : M - 1];
    r.n = hcnt[p];
}

// Entry index of partner `key` in the row read into r (row of slot p), or -1.
__device__ __forceinline__ int row_index(const int *__restrict__ hkey, int M, int p, const RowHead &r, int key)
{
    int idx = -1;
#pragma unroll
    for (int k = 0; k < kRowHead; ++k)
        if (k < r.n && (r.key[k] & kKeyMask) == key) idx = k;
    if (idx < 0 && r.n > kRowHead && (r.key[kRowHead - 1] & kKeyMask) < key) {
        const int *kr = hkey + (long long)p * M;
        int lo = kRowHead, hi = r.n;   // the key, if present, is in [lo, hi)
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int km = kr[mid] & kKeyMask;
            if (km == key) {
                idx = mid;
                break;
            }
            if (km < key)
                lo = mid + 1;
            else
                hi = mid;
        }
    }
    return idx;
}

__device__ __forceinline__ bool row_find(const int *__restrict__ hkey, const double *__restrict__ hxi,
                                         const int *__restrict__ hcnt, int M, int p, int key, double out[3],
                                         const double *__restrict__ hxr = nullptr, double *outr = nullptr)
{
    RowHead r;
    row_head(hkey, hcnt, M, p, r);
    const int k = row_index(hkey, M, p, r, key);
    if (k < 0) return false;
    const double *x = hxi + ((long long)p * M + k) * 3;
    out[0] = x[0];
    out[1] = x[1];
    out[2] = x[2];
    if (hxr) {
        const double *y = hxr + ((long long)p * M + k) * 3;
        outr[0] = y[0];
        outr[1] = y[1];
        outr[2] = y[2];
    }
    return true;
}

// Entry index of partner `key` in a row whose head h = (slot, count, key 0, key 1) was read
// before, or -1: the first two entries from the head, the rest (sorted) by bisection.
__device__ __forceinline__ int head_index(const int *__restrict__ hkey, int M, const int4 &h, int key)
{
    if (h.y > 0 && (h.z & kKeyMask) == key) return 0;
    if (h.y > 1 && (h.w & kKeyMask) == key) return 1;
    if (h.y > 2 && (h.w & kKeyMask) < key) {
        const int *kr = hkey + (long long)h.x * M;
        int lo = 2, hi = h.y;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int km = kr[mid] & kKeyMask;
            if (km == key) return mid;
            if (km < key)
                lo = mid + 1;
            else
                hi = mid;
        }
    }
    return -1;
}

struct HistView {
    const int *key_old;    // rows of the committed history, at the slots of the last step
    const double *xi_old;
    const int *cnt_old;
    const int *prev;       // slot -> slot of the same particle at the last step (null: same slot)
    int *key_new;
    double *xi_new;
    int *cnt_new;
    int *own_new;          // owner id of each new row
    const double *xr_old;  // rolling stretches beside xi (null without rolling resistance)
    double *xr_new;
};

// ----------------------------------------------------------------------------------
// Half shell of a cell (cx, cy, cz): its own cell (later slots only) and the 13 forward
// cells (dz > 0) or (dz = 0, dy > 0) or (dz = dy = 0, dx > 0).  Grouped by (dz, dy) into
// five x-rows:  r = 0 (0, 0) cells cx..cx+1;  r = 1 (0, +1);  r = 2 (+1, -1);
// r = 3 (+1, 0);  r = 4 (+1, +1), each cells cx-1..cx+1.  A row reached across a y face
// (images displaced by the Lees-Edwards offset) is the window of 4 x-cells around the
// shifted position instead.  Cells with consecutive cx are contiguous in sorted order,
// so a window is one or two contiguous slot ranges (two when it wraps in x).
// ----------------------------------------------------------------------------------
__device__ __forceinline__ void shell_row(int r, int &dz, int &dy)
{
    dz = r >= 2 ? 1 : 0;
    dy = r == 0 ? 0 : (r == 1 ? 1 : r - 3);
}

// x window [xlo, xhi] (unwrapped) of row r for a particle in cell column cx, given whether
// the row is reached across the top (+1) or bottom (-1) face (0: interior).
__device__ __forceinline__ void shell_window(const BoxParams &P, int r, int cx, int cross, double delta, int &xlo,
                                             int &xhi)
{
    if (cross != 0) {
        // top face: images displaced by +delta, so look around x - delta; bottom: x + delta
        const double sh = cross > 0 ? -delta : delta;
        const int k0 = (int)floor(((double)cx * P.cw[0] + sh) / P.cw[0]);
        xlo = k0 - 1;
        xhi = k0 + 2;
    } else if (r == 0) {
        xlo = cx;
        xhi = cx + 1;
    } else {
        xlo = cx - 1;
        xhi = cx + 1;
    }
}

// Evaluate one listed pair (i at slot gi, j at slot gj): history lookup (stored stretch
// of this pair in the row of either particle, canonical orientation min id -> max id) and
// the pair physics.
template <typename Real, bool Roll = false, bool Wave = false>
__device__ __forceinline__ void evaluate_pair(const DevParams &P, double gd, double wk, const HistView &H, int gi,
                                              int gj, int idi, int idj,
                                              const double4 &Xi, const double4 &Xj, const double4 &Vi,
                                              const double4 &Wi, const double4 &Vj, const double4 &Wj, double dx,
                                              double dy, double dz, double r2, double *S, PairOut &o)
{
    double xo[3] = {0.0, 0.0, 0.0};
    double xro[3] = {0.0, 0.0, 0.0};  // the rolling stretch has no orientation
    const double dist = sqrt(r2);
    if (dist - Xi.w - Xj.w < 0.0) {
        // the stored stretch is in the row of i (partner j) or, when the owner changed with the
        // cells, in the row of j (partner i): both row heads are read at once
        const int pi_ = H.prev ? H.prev[gi] : gi;
        const int pj_ = H.prev ? H.prev[gj] : gj;
        RowHead ri, rj;
        row_head(H.key_old, H.cnt_old, P.M, pi_, ri);
        row_head(H.key_old, H.cnt_old, P.M, pj_, rj);
        int p = pi_;
        int k = row_index(H.key_old, P.M, pi_, ri, idj);
        if (k < 0) {
            p = pj_;
            k = row_index(H.key_old, P.M, pj_, rj, idi);
        }
        if (k >= 0) {
            const double sg = idi > idj ? -1.0 : 1.0;
            const double *x = H.xi_old + ((long long)p * P.M + k) * 3;
            xo[0] = sg * x[0];
            xo[1] = sg * x[1];
            xo[2] = sg * x[2];
            if constexpr (Roll) {
                const double *y = H.xr_old + ((long long)p * P.M + k) * 3;
                xro[0] = y[0];
                xro[1] = y[1];
                xro[2] = y[2];
            }
        }
    }
    pair_physics<Real, Roll, Wave>(P, gd, wk, dx, dy, dz, dist, Xi.w, Xj.w, Xi.y, Xj.y, Vi, Vj, Wi, Wj, xo, xro, S, o);
}

__device__ __forceinline__ void record_pair(const DevParams &P, int idi, int idj, int *pair_out,
                                            unsigned long long *pair_count, DevClock *clk)
{
    unsigned long long k = atomicAdd(pair_count, 1ull);
    if ((long long)k < P.pair_cap) {
        pair_out[2 * k] = idi < idj ? idi : idj;
        pair_out[2 * k + 1] = idi < idj ? idj : idi;
    } else {
        atomicOr(&clk->err, kErrPairBuffer);
    }
}

template <bool Roll = false>
__device__ __forceinline__ void store_history(const HistView &H, int M, int gi, int slot, int idi, int idj,
                                              const PairOut &o, DevClock *clk)
{
    if (slot < M) {
        const double sg = idi < idj ? 1.0 : -1.0;
        H.key_new[(long long)gi * M + slot] = idj | (o.capped ? kCapBit : 0) | (o.rcapped ? kRollCapBit : 0);
        if constexpr (Roll) {
            double *y = H.xr_new + ((long long)gi * M + slot) * 3;
            y[0] = o.xr[0];
            y[1] = o.xr[1];
            y[2] = o.xr[2];
        }
        double *x = H.xi_new + ((long long)gi * M + slot) * 3;
        x[0] = sg * o.xi[0];
        x[1] = sg * o.xi[1];
        x[2] = sg * o.xi[2];
    } else {
        atomicOr(&clk->err, kErrRowOverflow);
    }
}

// Heap sort of the n entries of a history row by partner id, in place: O(n log n) key
// reads and entry moves (partner ids in a row are distinct).  The stretches, and the rolling
// stretches when rrow is set, move with their keys.
template <bool Roll>
__device__ __forceinline__ void heap_sort_row(int *krow, double *xrow, double *rrow, int n)
{
    auto swap_e = [&](int a, int b) {
        const int tk = krow[a];
        krow[a] = krow[b];
        krow[b] = tk;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double tx = xrow[3 * a + c];
            xrow[3 * a + c] = xrow[3 * b + c];
            xrow[3 * b + c] = tx;
            if constexpr (Roll) {
                const double ty = rrow[3 * a + c];
                rrow[3 * a + c] = rrow[3 * b + c];
                rrow[3 * b + c] = ty;
            }
        }
    };
    // sift the entry at `root` down the max-heap of the first `end` entries
    auto sift = [&](int root, int end) {
        int kr = krow[root] & kKeyMask;
        for (;;) {
            int c = 2 * root + 1;
            if (c >= end) break;
            int kc = krow[c] & kKeyMask;
            if (c + 1 < end) {
                const int k2 = krow[c + 1] & kKeyMask;
                if (k2 > kc) {
                    ++c;
                    kc = k2;
                }
            }
            if (kr >= kc) break;
            swap_e(root, c);
            root = c;
        }
    };
    for (int r = n / 2 - 1; r >= 0; --r) sift(r, n);
    for (int e = n - 1; e > 0; --e) {
        swap_e(0, e);
        sift(0, e);
    }
}

// Stretches of a history row in the order idx (n <= 16 entries): entry idx[a] is gathered
// into entry t0 + a of the free end of the row (t0 >= n), eight at a time, then the n entries
// are copied back to the front; the two ranges never overlap.
template <bool Roll>
__device__ __forceinline__ void permute_row_entries(double *xrow, double *rrow, const int idx[16], int n, int t0)
{
    constexpr int kBatch = Roll ? 4 : 8;
#pragma unroll
    for (int b0 = 0; b0 < 16; b0 += kBatch) {
        const double *__restrict__ src = xrow;
        double *__restrict__ dst = xrow + 3 * t0;
        double v[kBatch][3];
#pragma unroll
        for (int a = 0; a < kBatch; ++a) {
            const int e = b0 + a < n ? idx[b0 + a] : 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) v[a][c] = src[3 * e + c];
        }
#pragma unroll
        for (int a = 0; a < kBatch; ++a)
            if (b0 + a < n)
#pragma unroll
                for (int c = 0; c < 3; ++c) dst[3 * (b0 + a) + c] = v[a][c];
        if constexpr (Roll) {
            const double *__restrict__ rs = rrow;
            double *__restrict__ rd = rrow + 3 * t0;
#pragma unroll
            for (int a = 0; a < kBatch; ++a) {
                const int e = b0 + a < n ? idx[b0 + a] : 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) v[a][c] = rs[3 * e + c];
            }
#pragma unroll
            for (int a = 0; a < kBatch; ++a)
                if (b0 + a < n)
#pragma unroll
                    for (int c = 0; c < 3; ++c) rd[3 * (b0 + a) + c] = v[a][c];
        }
    }
#pragma unroll
    for (int b0 = 0; b0 < 16; b0 += kBatch) {
        const double *__restrict__ src = xrow + 3 * t0;
        double *__restrict__ dst = xrow;
        double v[kBatch][3];
#pragma unroll
        for (int a = 0; a < kBatch; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[a][c] = b0 + a < n ? src[3 * (b0 + a) + c] : 0.0;
#pragma unroll
        for (int a = 0; a < kBatch; ++a)
            if (b0 + a < n)
#pragma unroll
                for (int c = 0; c < 3; ++c) dst[3 * (b0 + a) + c] = v[a][c];
        if constexpr (Roll) {
            const double *__restrict__ rs = rrow + 3 * t0;
            double *__restrict__ rd = rrow;
#pragma unroll
            for (int a = 0; a < kBatch; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) v[a][c] = b0 + a < n ? rs[3 * (b0 + a) + c] : 0.0;
#pragma unroll
            for (int a = 0; a < kBatch; ++a)
                if (b0 + a < n)
#pragma unroll
                    for (int c = 0; c < 3; ++c) rd[3 * (b0 + a) + c] = v[a][c];
        }
    }
}

// Stretches of a history row in the order idx (n <= 16 entries) through a buffer of the
// lane's own in LDS (row_pool_doubles, rolling stretches in its second half): the whole row
// is loaded at once and parked in the buffer, then written back gathered in the new order, so
// the row costs one round of global loads instead of the two passes through its free end.
template <bool Roll>
constexpr int row_pool_doubles()
{
    return (Roll ? 2 : 1) * 16 * 3;
}

template <bool Roll>
__device__ __forceinline__ void permute_row_entries_lds(double *xrow, double *rrow, const int idx[16], int n,
                                                        double *buf)
{
#pragma unroll
    for (int part = 0; part < (Roll ? 2 : 1); ++part) {
        double *row = part ? rrow : xrow;
        double *b = buf + part * 48;
#pragma unroll
        for (int b0 = 0; b0 < 16; b0 += 8) {
            double v[8][3];
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) v[a][c] = b0 + a < n ? row[3 * (b0 + a) + c] : 0.0;
#pragma unroll
            for (int a = 0; a < 8; ++a)
                if (b0 + a < n)
#pragma unroll
                    for (int c = 0; c < 3; ++c) b[3 * (b0 + a) + c] = v[a][c];
        }
#pragma unroll
        for (int a = 0; a < 16; ++a)
            if (a < n)
#pragma unroll
                for (int c = 0; c < 3; ++c) row[3 * a + c] = b[3 * idx[a] + c];
    }
}

// Sort history row gi by partner id and publish it (the per-row sort of the contact
// map).  Rows of up to 8 entries are read at once and sorted in registers (odd-even
// transposition on the (key, stretch) tuples); rows of up to 16 (at most half the capacity) by
// their keys and entry indices in registers, the stretches then moved through a buffer in LDS
// when the caller gives a pool of them and one is free (pool_next counts the buffers taken),
// else through the free end of the row; longer rows by a heap sort in place.  With rolling
// resistance the rolling stretches move with their entries.
template <bool Roll = false>
__device__ __forceinline__ void finish_row(const HistView &H, int M, int gi, int fill, int idi,
                                           double *pool = nullptr, int *pool_next = nullptr, int pool_bufs = 0)
{
    int *krow = H.key_new + (long long)gi * M;
    double *xrow = H.xi_new + (long long)gi * M * 3;
    double *rrow = Roll ? H.xr_new + (long long)gi * M * 3 : nullptr;
    const int nrow = fill < M ? fill : M;
    if (nrow >= 2 && nrow <= 8) {
        // keys and stretches of the whole row read at once, sorted as tuples in registers
        // (odd-even transposition), written back
        int key[8];
        double x[8][3], y[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int e = a < nrow ? a : 0;
            key[a] = a < nrow ? krow[e] : 0x7fffffff;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                x[a][c] = xrow[3 * e + c];
                if constexpr (Roll) y[a][c] = rrow[3 * e + c];
            }
        }
#pragma unroll
        for (int round = 0; round < 8; ++round) {
#pragma unroll
            for (int a = round & 1; a + 1 < 8; a += 2) {
                if ((key[a] & kKeyMask) > (key[a + 1] & kKeyMask)) {
                    const int tk = key[a];
                    key[a] = key[a + 1];
                    key[a + 1] = tk;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double tx = x[a][c];
                        x[a][c] = x[a + 1][c];
                        x[a + 1][c] = tx;
                        if constexpr (Roll) {
                            const double ty = y[a][c];
                            y[a][c] = y[a + 1][c];
                            y[a + 1][c] = ty;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 8; ++a)
            if (a < nrow) {
                krow[a] = key[a];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xrow[3 * a + c] = x[a][c];
                    if constexpr (Roll) rrow[3 * a + c] = y[a][c];
                }
            }
    } else if (nrow > 8 && nrow <= 16 && (pool_bufs > 0 || 2 * nrow <= M)) {
        // keys sorted with their entry indices in registers (odd-even transposition); the
        // entries are gathered in the new order through an LDS buffer, or into the free end of
        // the row and then copied back (disjoint ranges: the loads of a batch are in flight
        // together)
        int key[16], idx[16];
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            key[a] = a < nrow ? krow[a] : 0x7fffffff;
            idx[a] = a;
        }
#pragma unroll
        for (int round = 0; round < 16; ++round) {
#pragma unroll
            for (int a = round & 1; a + 1 < 16; a += 2) {
                if ((key[a] & kKeyMask) > (key[a + 1] & kKeyMask)) {
                    const int tk = key[a];
                    key[a] = key[a + 1];
                    key[a + 1] = tk;
                    const int ti = idx[a];
                    idx[a] = idx[a + 1];
                    idx[a + 1] = ti;
                }
            }
        }
        const int buf = pool_bufs > 0 ? atomicAdd(pool_next, 1) : pool_bufs;
        if (buf < pool_bufs)
            permute_row_entries_lds<Roll>(xrow, rrow, idx, nrow, pool + (size_t)buf * row_pool_doubles<Roll>());
        else if (2 * nrow <= M)
            permute_row_entries<Roll>(xrow, rrow, idx, nrow, M - nrow);
        else
            heap_sort_row<Roll>(krow, xrow, rrow, nrow);
#pragma unroll
        for (int a = 0; a < 16; ++a)
            if (a < nrow) krow[a] = key[a];
    } else if (nrow > 16) {
        heap_sort_row<Roll>(krow, xrow, rrow, nrow);
    }
    H.cnt_new[gi] = nrow;
    H.own_new[gi] = idi;
}

// Stokes drag and rotational drag of one particle (eq. rst), added to f (force 0..2,
// torque 3..5).
// In the wavy shear the drag takes the Faxen term, F = -6 pi eta0 a [u - U_inf - a^2/6 lap U_inf]
// (lap U_inf = (-W k^2 sin(k y), 0, 0)), the torque the local rotation, and the Stokes stresslet
// (1 + a^2/10 lap) E_inf(y) (lap E_xy = -W k^3 cos(k y) / 2) adds its deviation from the uniform
// 20/3 pi eta0 a^3 gdot/2 (which the host adds for every particle) to S.
template <bool Wave>
__device__ __forceinline__ void stokes_terms(const DevParams &P, const BoxParams &G, const double4 &Xi,
                                             const double4 &Vi, const double4 &Wi, double f[6], double *S)
{
    const double K = P.k6;
    const double gd = G.gd;
    double ux = Vi.x - gd * Xi.y, sy = gd;
    if constexpr (Wave) {
        const double a = Xi.w, k = G.wk, sn = sin(k * Xi.y), cs = cos(k * Xi.y);
        ux -= P.wave_amp * sn * (1.0 - a * a * k * k / 6.0);
        sy = gd + P.wave_amp * k * cs;
        const double ss = (20.0 / 3.0) * kPi * P.eta0 * a * a * a *
                          (0.5 * (sy - gd) + a * a / 10.0 * (-0.5 * P.wave_amp * k * k * k * cs));
        S[1] += ss;
        S[3] += ss;
    }
    f[0] += -K * Xi.w * ux;
    f[1] += -K * Xi.w * Vi.y;
    f[2] += -K * Xi.w * Vi.z;
    const double KR = P.k8 * Xi.w * Xi.w * Xi.w;
    f[3] += -KR * Wi.x;
    f[4] += -KR * Wi.y;
    f[5] += -KR * (Wi.z + 0.5 * sy);
}

__device__ __forceinline__ bool finite6(const double f[6])
{
    return isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2]) && isfinite(f[3]) && isfinite(f[4]) &&
           isfinite(f[5]);
}

struct PairTally {
    double S[9];
    long long npair, ncont;
    int fill;
};

// ----------------------------------------------------------------------------------
// Per-particle path, for a cell row too large for the LDS tile: one lane walks the half
// shell of particle i, keeps its own side in registers (stored into its own record) and
// adds the partner side atomically to ft_x.
// ----------------------------------------------------------------------------------
template <typename Real, bool Roll, bool Wave>
__device__ __forceinline__ void particle_pairs_global(const DevParams &P, const BoxParams &G, int i, double delta,
                                      const int *__restrict__ cell_start,
                                      const double4 *__restrict__ pa, const double4 *__restrict__ vel,
                                      const double4 *__restrict__ omg, const ForceBufs &B, const HistView &H,
                                      DevClock *clk, int *pair_out, unsigned long long *pair_count,
                                      PairTally &tally)
{
    const double4 Xi = pa[i];
    const double4 Vi = vel[i];
    const double4 Wi = omg[i];
    const int idi = (int)Wi.w;
    const int cx = cell_coord(Xi.x, G.cw[0], G.nc[0]);
    const int cy = cell_coord(Xi.y, G.cw[1], G.nc[1]);
    const int cz = cell_coord(Xi.z, G.cw[2], G.nc[2]);
    const int nxc = G.nc[0], nyc = G.nc[1], nzc = G.nc[2];
    double f[6] = {0, 0, 0, 0, 0, 0};
    int fill = 0;
    for (int r = 0; r < 5; ++r) {
        int dz, dy;
        shell_row(r, dz, dy);
        int yy = cy + dy;
        int zz = cz + dz;
        zz = zz >= nzc ? zz - nzc : zz;
        const int cross = yy >= nyc ? 1 : (yy < 0 ? -1 : 0);
        yy = yy < 0 ? yy + nyc : (yy >= nyc ? yy - nyc : yy);
        int xlo, xhi;
        shell_window(G, r, cx, cross, delta, xlo, xhi);
        const int rbase = G.cell_off + (zz * nyc + yy) * nxc;
        int xl = ((xlo % nxc) + nxc) % nxc;
        int span = xhi - xlo + 1;
        for (int part = 0; part < 2 && span > 0; ++part) {
            const int len = (xl + span <= nxc) ? span : nxc - xl;
            int jb = cell_start[rbase + xl];
            const int je = cell_start[rbase + xl + len];
            if (r == 0 && part == 0) jb = i + 1;
            for (int j = jb; j < je; ++j) {
                const double4 Xj = pa[j];
                double dx, dy2, dz2, r2;
                min_image(G, delta, Xi.x, Xi.y, Xi.z, Xj.x, Xj.y, Xj.z, dx, dy2, dz2);
                if (!listed(P, dx, dy2, dz2, Xi.w, Xj.w, r2)) continue;
                const double4 Vj = vel[j];
                const double4 Wj = omg[j];
                const int idj = (int)Wj.w;
                ++tally.npair;
                if (P.record_pairs) record_pair(P, idi, idj, pair_out, pair_count, clk);
                PairOut o;
                evaluate_pair<Real, Roll, Wave>(P, G.gd, G.wk, H, i, j, idi, idj, Xi, Xj, Vi, Wi, Vj, Wj, dx, dy2, dz2, r2, tally.S, o);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    f[k] += o.Fi[k];
                    f[3 + k] += o.Ti[k];
                }
                double *xr = B.x + 6LL * j;
                atomicAdd(xr + 0, -o.Fi[0]);
                atomicAdd(xr + 1, -o.Fi[1]);
                atomicAdd(xr + 2, -o.Fi[2]);
                atomicAdd(xr + 3, o.Tj[0]);
                atomicAdd(xr + 4, o.Tj[1]);
                atomicAdd(xr + 5, o.Tj[2]);
                if (o.contact) {
                    ++tally.ncont;
                    store_history<Roll>(H, P.M, i, fill, idi, idj, o, clk);
                    ++fill;
                }
            }
            xl = 0;
            span -= len;
        }
    }
    finish_row<Roll>(H, P.M, i, fill, idi);
    tally.fill = max(tally.fill, fill);
    stokes_terms<Wave>(P, G, Xi, Vi, Wi, f, tally.S);
    store_ft(B.own + 6LL * i, f);
    if (!finite6(f)) atomicOr(&clk->err, kErrNonFinite);
}

// Block reduction of the stress and counters of a workgroup into its partial record
// (12 doubles: 9 stress components, pairs, contacts, largest row; component k of workgroup
// w at partials[k pstride + w]), summed by k_finish.
__device__ __forceinline__ void reduce_tally(PairTally &tally, double (*red)[12], double *__restrict__ partials,
                                             int pstride, int rec)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double v = warp_sum(tally.S[k]);
        if (lane == 0) red[wid][k] = v;
    }
    long long np_ = warp_sum_ll(tally.npair), nc_ = warp_sum_ll(tally.ncont);
    int mf = warp_max(tally.fill);
    if (lane == 0) {
        red[wid][9] = (double)np_;
        red[wid][10] = (double)nc_;
        red[wid][11] = (double)mf;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        const int k = threadIdx.x;
        double v = 0.0;
        const int nw = (int)(blockDim.x >> 6);
        for (int w = 0; w < nw; ++w) v = (k == 11) ? fmax(v, red[w][k]) : v + red[w][k];
        partials[(long long)k * pstride + rec] = v;
    }
}

// The two parts of reduce_tally for a kernel that knows its sums before its rows: the sums
// (9 stress components, pairs, contacts; components 0..10), then the largest row (11).
__device__ __forceinline__ void reduce_sums(const PairTally &tally, double (*red)[12], double *__restrict__ partials,
                                            int pstride, int rec)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double v = warp_sum(tally.S[k]);
        if (lane == 0) red[wid][k] = v;
    }
    long long np_ = warp_sum_ll(tally.npair), nc_ = warp_sum_ll(tally.ncont);
    if (lane == 0) {
        red[wid][9] = (double)np_;
        red[wid][10] = (double)nc_;
    }
    __syncthreads();
    if (threadIdx.x < 11) {
        const int k = threadIdx.x;
        double v = 0.0;
        const int nw = (int)(blockDim.x >> 6);
        for (int w = 0; w < nw; ++w) v += red[w][k];
        partials[(long long)k * pstride + rec] = v;
    }
}

__device__ __forceinline__ void reduce_fill(int fill, double (*red)[12], double *__restrict__ partials, int pstride,
                                            int rec)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int mf = warp_max(fill);
    if (lane == 0) red[wid][11] = (double)mf;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        const int nw = (int)(blockDim.x >> 6);
        for (int w = 0; w < nw; ++w) v = fmax(v, red[w][11]);
        partials[11LL * pstride + rec] = v;
    }
}

// ----------------------------------------------------------------------------------
// k_pairs: one workgroup of kPairBlock lanes per x-row of cells (cz, cy).  The particles of
// the five rows of the half shell are staged in LDS as FP32 (x, y, z, a) records, which
// only pre-select candidates; every decision and every pair quantity is FP64, from the
// particle records in global memory.
//   A1  every (particle, shell row) task appends the staged indices of its window (at most
//       two ranges) to one flat candidate list;
//   A2  every lane pre-tests its share of the candidates in FP32 with a margin that covers
//       the rounding of FP32 coordinates (no listed pair is lost), and queues the survivors
//       in LDS (probable contacts last);
//   H   the history row head (slot at the last step, count, first two keys) of every staged
//       particle replaces its FP32 record;
//   B   all lanes take the queued pairs: the FP64 nearest image and listed test decide,
//       then the pair physics with the stored stretch found from the row heads; both sides
//       accumulate in LDS (FP64 LDS atomics), history rows of the own particles get their
//       slots from LDS counters;
//   C   own particles: Stokes terms, own force record, history row sorted by partner id;
//       particles of the other four shell rows: partner-side force records.
// LDS: the candidate list and the staged slots at the last step live in the force
// accumulators' space (cleared after H), the row heads in that of the FP32 records, and the
// cell starts of the five rows (read by A1) in that of the pair queue, so that four
// workgroups fit in the 160 KB of a CU; with 3 wavefronts each they hold 12 wavefronts per CU
// (the register file holds three per SIMD), one cell row per workgroup slot (the host keeps
// the rows of one box below the slots).  The row heads are requested before A2, whose
// barriers order LDS only, so their loads overlap the candidate tests.
// Tile capacities (P.own_cap, P.stage_cap, P.qcap) are sized from the mean row occupancy; a
// row beyond them takes the per-particle path, by its own workgroup.  Sum: the row's stress and
// counters are reduced into its partial record.  Steps whose stress is not summed take
// Sum = false, and the compiler drops the stresslet arithmetic and its accumulators (the
// forces, torques and history are the same).
// ----------------------------------------------------------------------------------
constexpr int kPairBlock = 192;

// The k_pairs instantiation that inlines the per-particle path of a row beyond the tile
// capacities: the mixed kernel without rolling resistance and wavy shear, whose FP32 physics
// leaves the registers for it; the others call it out of line (row_per_particle).
template <typename Real, bool Roll, bool Wave>
__host__ __device__ constexpr bool rows_inlined()
{
    return std::is_same<Real, float>::value && !Roll && !Wave;
}
constexpr int kPairWaves = kPairBlock / 64;
constexpr int kHeadPre = 3;  // row heads per lane requested before A2

struct TileShared {
    int rs[5], re[5], ro[6], rbase[5], rcross[5];
    int qn;
    int nc;             // candidates listed by k_pairs
    int ovf;            // tile overflow: the row is redone on the per-particle path
    int rpool;          // LDS row buffers taken in C (in the pair queue's space)
    int wsum[kBlock / 64];
    double red[kBlock / 64][12];
};

struct TileView {
    float4 *sp;         // stage_cap: FP32 (x, y, z, a) of the staged particles; from B on the
    int4 *heads;        //   history row heads of the staged particles (slot, count, key 0, key 1)
    double *acc;        // stage_cap x 6 FP64 accumulators; during A1-A2 the candidate list
    unsigned *queue;    // qcap pairs
    int *rowcnt;        // own_cap history-row fill
    int *owncx;         // own_cap cell column of each own particle
    int *prevs;         // stage_cap: slot of each staged particle at the last step (the end
                        //   of the accumulators' space, beyond the candidate list)
};

__host__ __device__ inline size_t tile_lds_bytes(int own_cap, int stage_cap, int qcap)
{
    return (size_t)stage_cap * 16 + (size_t)stage_cap * 48 + ((size_t)qcap * 4 + 7) / 8 * 8 + (size_t)own_cap * 4 +
           (size_t)own_cap * 4;
}

// FP32 pre-test of a candidate with the image shifts of its range: 0 surely not listed, 1
// possibly listed, 2 possibly listed and probably in contact.  m2 bounds the error of r^2
// from FP32 coordinates (host: from the largest box length); the FP64 test decides later.
__device__ __forceinline__ int image_class_f32(const float4 &Xi, const float4 &Xj, float sy, float sxd, float sx,
                                               float sz, float cf, float rext, float m2)
{
    float dx = Xj.x - Xi.x, dy = Xj.y - Xi.y, dz = Xj.z - Xi.z;
    dy = dy + sy;
    dx = dx + sxd;
    dx = dx + sx;
    dz = dz + sz;
    const float r2 = (dx * dx + dy * dy) + dz * dz;
    const float s = Xi.w + Xj.w;
    float rc = cf * s;
    if (rext > 0.0f) rc = fmaxf(rc, s + rext);
    return r2 < rc * rc + m2 ? (r2 < s * s + m2 ? 2 : 1) : 0;
}

// One queued pair (i = own particle il, j = staged particle jl): the FP64 nearest image and
// listed test (the definition; the FP32 pre-test only selected it), then the pair physics.
template <typename Real, bool Roll, bool Wave>
__device__ __forceinline__ void tile_pair(const DevParams &P, const BoxParams &G, const HistView &H, const TileShared &T,
                                          const TileView &V, int il, int jl, double delta,
                                          const double4 *__restrict__ pa, const double4 *__restrict__ vel,
                                          const double4 *__restrict__ omg, DevClock *clk, int *pair_out,
                                          unsigned long long *pair_count, PairTally &tally)
{
    const int r = (jl >= T.ro[1]) + (jl >= T.ro[2]) + (jl >= T.ro[3]) + (jl >= T.ro[4]);
    const int gi = T.rs[0] + il;
    const int gj = T.rs[r] + (jl - T.ro[r]);
    const double4 Xi = pa[gi];
    const double4 Xj = pa[gj];
    const double4 Vi = vel[gi];
    const double4 Wi = omg[gi];
    const double4 Vj = vel[gj];
    const double4 Wj = omg[gj];
    double dx, dy, dz, r2;
    min_image(G, delta, Xi.x, Xi.y, Xi.z, Xj.x, Xj.y, Xj.z, dx, dy, dz);
    if (!listed(P, dx, dy, dz, Xi.w, Xj.w, r2)) return;
    const int idi = (int)Wi.w, idj = (int)Wj.w;
    ++tally.npair;
    if (P.record_pairs) record_pair(P, idi, idj, pair_out, pair_count, clk);
    // stored stretch of a contact: in the row of i (partner j) or, when the owner changed with
    // the cells, in the row of j (partner i), found from the staged row heads
    double xo[3] = {0.0, 0.0, 0.0};
    double xro[3] = {0.0, 0.0, 0.0};  // the rolling stretch has no orientation
    const double dist = sqrt(r2);
    if (dist - Xi.w - Xj.w < 0.0) {
        const int4 hi = V.heads[il], hj = V.heads[jl];
        int p = hi.x;
        int k = head_index(H.key_old, P.M, hi, idj);
        if (k < 0) {
            p = hj.x;
            k = head_index(H.key_old, P.M, hj, idi);
        }
        if (k >= 0) {
            const double sg = idi > idj ? -1.0 : 1.0;
            const double *x = H.xi_old + ((long long)p * P.M + k) * 3;
            xo[0] = sg * x[0];
            xo[1] = sg * x[1];
            xo[2] = sg * x[2];
            if constexpr (Roll) {
                const double *y = H.xr_old + ((long long)p * P.M + k) * 3;
                xro[0] = y[0];
                xro[1] = y[1];
                xro[2] = y[2];
            }
        }
    }
    PairOut o;
    pair_physics<Real, Roll, Wave>(P, G.gd, G.wk, dx, dy, dz, dist, Xi.w, Xj.w, Xi.y, Xj.y, Vi, Vj, Wi, Wj, xo, xro,
                                   tally.S, o);
    double *ai = V.acc + 6 * il;
    double *aj = V.acc + 6 * jl;
    atomicAdd(ai + 0, o.Fi[0]);
    atomicAdd(ai + 1, o.Fi[1]);
    atomicAdd(ai + 2, o.Fi[2]);
    atomicAdd(ai + 3, o.Ti[0]);
    atomicAdd(ai + 4, o.Ti[1]);
    atomicAdd(ai + 5, o.Ti[2]);
    atomicAdd(aj + 0, -o.Fi[0]);
    atomicAdd(aj + 1, -o.Fi[1]);
    atomicAdd(aj + 2, -o.Fi[2]);
    atomicAdd(aj + 3, o.Tj[0]);
    atomicAdd(aj + 4, o.Tj[1]);
    atomicAdd(aj + 5, o.Tj[2]);
    if (o.contact) {
        ++tally.ncont;
        const int slot = atomicAdd(&V.rowcnt[il], 1);
        store_history<Roll>(H, P.M, gi, slot, idi, idj, o, clk);
    }
}

// Slot ranges of the five half-shell rows of cell row `row` of box G (shared), with the
// y-face crossing of each row; ends with a barrier.
__device__ __forceinline__ void row_bounds(const BoxParams &G, int row, const int *__restrict__ cell_start,
                                           TileShared &T)
{
    const int t = threadIdx.x;
    const int nxc = G.nc[0], nyc = G.nc[1], nzc = G.nc[2];
    const int cz = row / nyc, cy = row - (row / nyc) * nyc;
    if (t < 5) {
        int dz, dy;
        shell_row(t, dz, dy);
        int zz = cz + dz;
        zz = zz >= nzc ? zz - nzc : zz;
        int yy = cy + dy;
        T.rcross[t] = yy >= nyc ? 1 : (yy < 0 ? -1 : 0);
        yy = yy < 0 ? yy + nyc : (yy >= nyc ? yy - nyc : yy);
        const int base = G.cell_off + (zz * nyc + yy) * nxc;
        T.rbase[t] = base;
        T.rs[t] = cell_start[base];
        T.re[t] = cell_start[base + nxc];
    }
    __syncthreads();
    if (t == 0) {
        int o = 0;
        for (int r = 0; r < 5; ++r) {
            T.ro[r] = o;
            o += T.re[r] - T.rs[r];
        }
        T.ro[5] = o;
        T.qn = 0;
        T.nc = 0;
        T.ovf = 0;
    }
    __syncthreads();
}

// row_bounds with the cell starts of the five rows staged in LDS (csl, 5 (n_x + 1) entries:
// row r's start of cell c at csl[r (n_x + 1) + c], its end at csl[r (n_x + 1) + n_x]), so that
// the windows of A1 are read from LDS.  Ends with a barrier.
__device__ __forceinline__ void row_bounds_staged(const BoxParams &G, int row, const int *__restrict__ cell_start,
                                                  TileShared &T, int *csl)
{
    const int t = threadIdx.x;
    const int nxc = G.nc[0], nyc = G.nc[1], nzc = G.nc[2];
    const int cz = row / nyc, cy = row - (row / nyc) * nyc;
    for (int k = t; k < 5 * (nxc + 1); k += blockDim.x) {
        const int r = k / (nxc + 1), c = k - r * (nxc + 1);
        int dz, dy;
        shell_row(r, dz, dy);
        int zz = cz + dz;
        zz = zz >= nzc ? zz - nzc : zz;
        int yy = cy + dy;
        const int cross = yy >= nyc ? 1 : (yy < 0 ? -1 : 0);
        yy = yy < 0 ? yy + nyc : (yy >= nyc ? yy - nyc : yy);
        const int base = G.cell_off + (zz * nyc + yy) * nxc;
        csl[k] = cell_start[base + c];
        if (c == 0) {
            T.rbase[r] = base;
            T.rcross[r] = cross;
        }
    }
    __syncthreads();
    if (t == 0) {
        int o = 0;
        for (int r = 0; r < 5; ++r) {
            T.rs[r] = csl[r * (nxc + 1)];
            T.re[r] = csl[r * (nxc + 1) + nxc];
            T.ro[r] = o;
            o += T.re[r] - T.rs[r];
        }
        T.ro[5] = o;
        T.qn = 0;
        T.nc = 0;
        T.ovf = 0;
    }
    __syncthreads();
}

// Workgroup barrier that orders LDS accesses only: global loads in flight stay in flight
// (__syncthreads also waits for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Cell row of workgroup b of n.  Workgroups are dispatched to the 8 XCDs in turn (b mod 8),
// each XCD with its own L2; this bijection gives every XCD one contiguous run of rows, so the
// shell rows a workgroup stages were mostly fetched into the same L2 by its neighbours.
__device__ __forceinline__ int xcd_row(int b, int n)
{
    constexpr int kXcd = 8;
    const int q = n / kXcd, r = n % kXcd;
    const int x = b % kXcd, k = b / kXcd;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Window of shell row r for an own particle in cell column cx: at most two runs of cells of
// the row, [xl0, xl0 + len0) and [0, len1), the first w box lengths L_x beyond the row in x
// and the second w + 1.
struct TaskWindow {
    int xl0, len0, len1, w;
};

__device__ __forceinline__ TaskWindow task_window(const BoxParams &G, const TileShared &T, int r, int cx, double delta)
{
    const int nxc = G.nc[0];
    int xlo, xhi;
    shell_window(G, r, cx, T.rcross[r], delta, xlo, xhi);
    const int w = xlo >= 0 ? xlo / nxc : -((-xlo + nxc - 1) / nxc);  // floor(xlo / nx)
    const int xl = xlo - w * nxc;
    const int span = xhi - xlo + 1;
    const int len0 = (xl + span <= nxc) ? span : nxc - xl;
    TaskWindow W;
    W.xl0 = xl;
    W.len0 = len0;
    W.len1 = span - len0;
    W.w = w;
    return W;
}

// The arguments of the per-particle path inside k_pairs, as a kernel argument of its own: the
// call reads them from the kernel's argument segment where it is made, while values passed from
// the tile path's own arguments were copied to memory at the kernel's start, on every row.
struct RowArgs {
    DevParams P;
    ForceBufs B;
    HistView H;
    const BoxParams *boxes;
    const int *row_box;
    const int *cell_start;
    const double4 *pa, *vel, *omg;
    DevClock *clk;
    double *partials;
    int *pair_out;
    unsigned long long *pair_count;
};

// One cell row on the per-particle path, taken by the k_pairs workgroup that found it beyond its
// tile (every kernel but the plain mixed one).  Kept out of line: the physics of a lane's whole
// half shell needs more registers than the tile path leaves, and as a call its spills stay on
// this rare path (nothing of the tile is live at the call), where inlined they spilled the
// tile path.
template <typename Real, bool Roll, bool Wave, bool Sum>
__device__ __noinline__ void row_per_particle(RowArgs R, int grow, TileShared &T)
{
    const DevParams &P = R.P;
    const int t = threadIdx.x;
    const BoxParams G = R.boxes[P.nbox > 1 ? R.row_box[grow] : 0];
    const double delta = le_offset(P, G, R.clk->step);
    PairTally tally;
#pragma unroll
    for (int k = 0; k < 9; ++k) tally.S[k] = 0.0;
    tally.npair = tally.ncont = 0;
    tally.fill = 0;
    for (int i = T.rs[0] + t; i < T.re[0]; i += kPairBlock)
        particle_pairs_global<Real, Roll, Wave>(P, G, i, delta, R.cell_start, R.pa, R.vel, R.omg, R.B, R.H, R.clk,
                                                R.pair_out, R.pair_count, tally);
    const double z[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = 1; r < 5; ++r)
        for (int g = T.rs[r] + t; g < T.re[r]; g += kPairBlock) store_ft(R.B.nb + 6LL * ((r - 1) * R.B.n + g), z);
    if (t == 0) R.clk->deferred = 1;
    if constexpr (Sum) reduce_tally(tally, T.red, R.partials, P.pstride, grow);
}

template <typename Real, bool Roll, bool Wave, bool Sum>
__global__ void __launch_bounds__(kPairBlock, 3) k_pairs(DevParams P, const BoxParams *__restrict__ boxes,
                                                          const int *__restrict__ row_box,
                                                          const int *__restrict__ cell_start,
                                                          const double4 *__restrict__ pa,
                                                          const double4 *__restrict__ vel,
                                                          const double4 *__restrict__ omg, ForceBufs B, HistView H,
                                                          DevClock *__restrict__ clk, double *__restrict__ partials,
                                                          int *__restrict__ pair_out,
                                                          unsigned long long *__restrict__ pair_count, RowArgs R)
{
    __shared__ TileShared T;
    extern __shared__ double4 dyn_lds[];
    TileView V;
    V.sp = reinterpret_cast<float4 *>(dyn_lds);
    V.heads = reinterpret_cast<int4 *>(dyn_lds);
    V.acc = reinterpret_cast<double *>(V.sp + P.stage_cap);
    V.queue = reinterpret_cast<unsigned *>(V.acc + 6 * P.stage_cap);
    V.rowcnt = reinterpret_cast<int *>(V.queue + (P.qcap + 1) / 2 * 2);
    V.owncx = V.rowcnt + P.own_cap;
    V.prevs = reinterpret_cast<int *>(V.acc) + 11 * P.stage_cap;

    const int t = threadIdx.x;
    const int lane = t & 63, wid = t >> 6;
    const int grow = xcd_row(blockIdx.x, gridDim.x);
    const BoxParams G = boxes[P.nbox > 1 ? row_box[grow] : 0];
    const int nxc = G.nc[0], nzc = G.nc[2];
    const int row = grow - G.row_off;  // cell row within the box
    const int cz = row / G.nc[1];
    const double delta = le_offset(P, G, clk->step);
    PairTally tally;
#pragma unroll
    for (int k = 0; k < 9; ++k) tally.S[k] = 0.0;
    tally.npair = tally.ncont = 0;
    tally.fill = 0;
    // the cell starts of the five rows in LDS (in the queue's space, free until A2) when they fit
    int *const csl = reinterpret_cast<int *>(V.queue);
    const bool cs_staged = 5 * (nxc + 1) <= P.qcap;
    if (cs_staged)
        row_bounds_staged(G, row, cell_start, T, csl);
    else
        row_bounds(G, row, cell_start, T);
    const int n_own = T.re[0] - T.rs[0];
    const int total = T.ro[5];
    // a row beyond the tile capacities (or one that hits a tile limit below) takes the
    // per-particle path by its own workgroup (the partner sides go to the atomic record, which
    // k_predict then reads; inlined in the plain mixed kernel, a call in the others); nothing
    // of the tile is written
    auto defer_row = [&]() {
        if constexpr (!rows_inlined<Real, Roll, Wave>()) {
            row_per_particle<Real, Roll, Wave, Sum>(R, grow, T);
        } else {
            for (int i = T.rs[0] + t; i < T.re[0]; i += kPairBlock)
                particle_pairs_global<Real, Roll, Wave>(P, G, i, delta, cell_start, pa, vel, omg, B, H, clk, pair_out,
                                                        pair_count, tally);
            const double z[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int r = 1; r < 5; ++r)
                for (int g = T.rs[r] + t; g < T.re[r]; g += kPairBlock) store_ft(B.nb + 6LL * ((r - 1) * B.n + g), z);
            if (t == 0) clk->deferred = 1;
            if constexpr (Sum) reduce_tally(tally, T.red, partials, P.pstride, grow);
        }
    };
    if (!P.tiled || n_own > P.own_cap || total > P.stage_cap) goto per_particle;
  {  // the tile path (every exit to per_particle is workgroup-uniform)
    // stage the shell rows (FP32) with their slots at the last step, and the cell column of
    // every own particle (from FP64)
    for (int k = t; k < total; k += kPairBlock) {
        const int r = (k >= T.ro[1]) + (k >= T.ro[2]) + (k >= T.ro[3]) + (k >= T.ro[4]);
        const int g = T.rs[r] + (k - T.ro[r]);
        const double4 X = pa[g];
        V.prevs[k] = H.prev ? H.prev[g] : g;
        V.sp[k] = make_float4((float)X.x, (float)X.y, (float)X.z, (float)X.w);
        if (k < n_own) {
            V.owncx[k] = cell_coord(X.x, G.cw[0], nxc);
            V.rowcnt[k] = 0;
        }
    }
    __syncthreads();

    // A1: every (particle, shell row) task turns its window into at most two ranges of staged
    // indices and appends their candidates to one flat list (a wavefront scan of the task
    // counts and one LDS atomic per wavefront place them; the order of the list does not
    // matter).  Candidate word: staged partner index jl (bits 0-13), il (bits 14-25), and the
    // image of its range (bits 26-31: y-face crossing + 1, x period w + 4, z wrap).  The list
    // lives in the LDS of the force accumulators.
    unsigned *const cand = reinterpret_cast<unsigned *>(V.acc);
    const int ccap = 11 * P.stage_cap < 64 * kPairBlock ? 11 * P.stage_cap : 64 * kPairBlock;
    const int ntask = 5 * n_own;
    constexpr int kTaskBatch = 4;  // tasks per lane whose cell-range loads are in flight together
    for (int task0 = 0; task0 < ntask; task0 += kTaskBatch * kPairBlock) {  // the same trip count in every lane
        int rr[kTaskBatch], ill[kTaskBatch], cs4[kTaskBatch][4];
        TaskWindow W[kTaskBatch];
#pragma unroll
        for (int u = 0; u < kTaskBatch; ++u) {
            const int task = task0 + u * kPairBlock + t;
            const bool on = task < ntask;
            rr[u] = on ? task / n_own : 0;
            ill[u] = on ? task - rr[u] * n_own : 0;
            W[u] = task_window(G, T, rr[u], V.owncx[ill[u]], delta);
            if (cs_staged) {
                const int *cr = csl + rr[u] * (nxc + 1);
                cs4[u][0] = cr[W[u].xl0];
                cs4[u][1] = cr[W[u].xl0 + W[u].len0];
                cs4[u][2] = cr[0];
                cs4[u][3] = cr[W[u].len1];
            } else {
                const int base = T.rbase[rr[u]];
                cs4[u][0] = cell_start[base + W[u].xl0];
                cs4[u][1] = cell_start[base + W[u].xl0 + W[u].len0];
                cs4[u][2] = cell_start[base];
                cs4[u][3] = cell_start[base + W[u].len1];
            }
        }
#pragma unroll
        for (int u = 0; u < kTaskBatch; ++u) {
            const int task = task0 + u * kPairBlock + t;
            const int r = rr[u], il = ill[u];
            int n0 = 0, n1 = 0, j0 = 0, j1 = 0;
            if (task < ntask) {
                const int jb = r == 0 ? T.rs[0] + il + 1 : cs4[u][0];
                n0 = cs4[u][1] > jb ? cs4[u][1] - jb : 0;
                j0 = T.ro[r] + (jb - T.rs[r]);
                if (W[u].len1 > 0) {
                    n1 = cs4[u][3] > cs4[u][2] ? cs4[u][3] - cs4[u][2] : 0;
                    j1 = T.ro[r] + (cs4[u][2] - T.rs[r]);
                }
                if (n0 > 2047 || n1 > 2047) T.ovf = 1;
            }
            const int n = n0 + n1;
            int incl = n;
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            int base = 0;
            if (lane == 63) base = atomicAdd(&T.nc, incl);
            base = __shfl(base, 63, 64) + incl - n;
            if (n > 0 && base + n <= ccap) {
                const unsigned common = ((unsigned)il << 14) | ((unsigned)(T.rcross[r] + 1) << 26) |
                                        ((r >= 2 && cz == nzc - 1) ? (1u << 31) : 0u);
                const unsigned c0 = common | ((unsigned)(W[u].w + 4) << 28);
                const unsigned c1 = common | ((unsigned)(W[u].w + 5) << 28);
                for (int o = 0; o < n0; ++o) cand[base + o] = c0 + (unsigned)(j0 + o);
                for (int o = 0; o < n1; ++o) cand[base + n0 + o] = c1 + (unsigned)(j1 + o);
            }
        }
    }
    __syncthreads();
    const int ncand = T.nc;
    if (T.ovf || ncand > ccap) goto per_particle;  // a tile limit was hit

    // the history row heads of the first kHeadPre staged particles of every lane are requested
    // now, so that their loads are in flight during A2; they are written over the FP32
    // records (which A2 still reads) after it
    int4 hpre[kHeadPre];
#pragma unroll
    for (int m = 0; m < kHeadPre; ++m) {
        const int k = t + m * kPairBlock;
        if (k < total) {
            const int p = V.prevs[k];
            const int *kr = H.key_old + (long long)p * P.M;
            hpre[m] = make_int4(p, H.cnt_old[p], kr[0], kr[P.M > 1 ? 1 : 0]);
        }
    }

    // A2: the candidates in lane-strided order (lane t pre-tests k = t + kPairBlock j, two per
    // pass), every lane running the same straight-line FP32 test with the shifts of the
    // candidate's range.  Survivors are kept as bit masks per lane (all, and the probable
    // contacts); a block scan of the two counts gives every lane its slots in the pair queue,
    // the other pairs first and the probable contacts last (no atomics).
    if (!T.ovf) {
        const float Lx = (float)G.L[0], Ly = (float)G.L[1], Lz = (float)G.L[2], dl = (float)delta;
        const float cf = (float)P.cf, rx = (P.ec && !P.ec_split) ? (float)P.rext : 0.0f, m2 = P.pf_m2;
        auto test = [&](unsigned wd) -> int {
            const int jl = (int)(wd & 0x3fffu);
            const int il = (int)((wd >> 14) & 0xfffu);
            const int cross = (int)((wd >> 26) & 3u) - 1;
            const float sy = cross > 0 ? Ly : (cross < 0 ? -Ly : 0.0f);
            const float sxd = cross > 0 ? dl : (cross < 0 ? -dl : 0.0f);
            const float sx = (float)((int)((wd >> 28) & 7u) - 4) * Lx;
            const float sz = (wd >> 31) ? Lz : 0.0f;
            return image_class_f32(V.sp[il], V.sp[jl], sy, sxd, sx, sz, cf, rx, m2);
        };
        unsigned long long bits = 0ull, cbits = 0ull;
        int j = 0;
        for (int k = t; k < ncand; k += 2 * kPairBlock, j += 2) {
            const int k2 = k + kPairBlock;
            const unsigned w0 = cand[k];
            const unsigned w1 = k2 < ncand ? cand[k2] : w0;
            const int h0 = test(w0);
            const int h1 = k2 < ncand ? test(w1) : 0;
            bits |= (unsigned long long)(h0 != 0) << j | (unsigned long long)(h1 != 0) << (j + 1);
            cbits |= (unsigned long long)(h0 == 2) << j | (unsigned long long)(h1 == 2) << (j + 1);
        }
        const int cc = __popcll(cbits);
        const int c = (__popcll(bits) - cc) | (cc << 16);
        int incl = c;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) T.wsum[wid] = incl;
        lds_barrier();  // the row heads requested above stay in flight
        int q = incl - c;
        int tot = 0;
        for (int w = 0; w < kPairWaves; ++w) {
            q += w < wid ? T.wsum[w] : 0;
            tot += T.wsum[w];
        }
        const int nfar = tot & 0xffff, nhit = nfar + (tot >> 16);
        if (nhit > P.qcap) {
            if (t == 0) T.ovf = 1;
        } else {
            int qf = q & 0xffff, qc = nfar + (q >> 16);
            while (bits) {
                const int jj = __ffsll((long long)bits) - 1;
                const bool ct = (cbits >> jj) & 1ull;
                bits &= bits - 1ull;
                const unsigned wd = cand[t + jj * kPairBlock];
                V.queue[ct ? qc++ : qf++] = (((wd >> 14) & 0xfffu) << 16) | (wd & 0x3fffu);
            }
            if (t == 0) T.qn = nhit;
        }
    }
    lds_barrier();
    if (T.ovf) goto per_particle;  // a tile limit was hit: the tile is discarded

    // the FP32 records are dead: the history row head of every staged particle (its slot at
    // the last step, row count, first two keys) takes their place, so that B finds most stored
    // stretches without a chain of global loads; the accumulators are cleared
#pragma unroll
    for (int m = 0; m < kHeadPre; ++m) {
        const int k = t + m * kPairBlock;
        if (k < total) V.heads[k] = hpre[m];
    }
    for (int k = t + kHeadPre * kPairBlock; k < total; k += kPairBlock) {
        const int p = V.prevs[k];
        const int *kr = H.key_old + (long long)p * P.M;
        V.heads[k] = make_int4(p, H.cnt_old[p], kr[0], kr[P.M > 1 ? 1 : 0]);
    }
    __syncthreads();   // the slots are read before the accumulators (their space) are cleared
    for (int k = t; k < 6 * total; k += kPairBlock) V.acc[k] = 0.0;
    __syncthreads();

    // B: evaluate the queued pairs
    const int nq = T.qn;
    for (int q = t; q < nq; q += kPairBlock) {
        const unsigned e = V.queue[q];
        tile_pair<Real, Roll, Wave>(P, G, H, T, V, (int)(e >> 16), (int)(e & 0xffffu), delta, pa, vel, omg, clk,
                                    pair_out, pair_count, tally);
    }
    // the records of the lane's first own particle of C are requested before the barrier
    double4 Xc = make_double4(0.0, 0.0, 0.0, 0.0), Vc = Xc, Wc = Xc;
    if (t < n_own) {
        Xc = pa[T.rs[0] + t];
        Vc = vel[T.rs[0] + t];
        Wc = omg[T.rs[0] + t];
    }
    // the sums are complete (C adds to the stress only in the wavy shear): reduced here, so that
    // their registers are free in C
    if constexpr (Sum && !Wave) reduce_sums(tally, T.red, partials, P.pstride, grow);
    if (t == 0) T.rpool = 0;
    __syncthreads();

    // C: own particles (Stokes terms, own record, history row), then partner records.  The
    // pair queue is dead: its space holds the LDS buffers of the history rows of 9-16 entries.
    double *const row_pool = reinterpret_cast<double *>(V.queue);
    const int row_bufs =
        (int)((size_t)(P.qcap + 1) / 2 * 2 * sizeof(unsigned) / (row_pool_doubles<Roll>() * sizeof(double)));
    for (int il = t; il < n_own; il += kPairBlock) {
        const int gi = T.rs[0] + il;
        const double4 Xi = il == t ? Xc : pa[gi];
        const double4 Vi = il == t ? Vc : vel[gi];
        const double4 Wi = il == t ? Wc : omg[gi];
        double f[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) f[c] = V.acc[6 * il + c];
        stokes_terms<Wave>(P, G, Xi, Vi, Wi, f, tally.S);
        store_ft(B.own + 6LL * gi, f);
        if (!finite6(f)) atomicOr(&clk->err, kErrNonFinite);
        const int fill = V.rowcnt[il];
        finish_row<Roll>(H, P.M, gi, fill, (int)Wi.w, row_pool, &T.rpool, row_bufs);
        tally.fill = max(tally.fill, fill);
    }
    for (int k = T.ro[1] + t; k < total; k += kPairBlock) {
        const int r = (k >= T.ro[2]) + (k >= T.ro[3]) + (k >= T.ro[4]) + 1;
        const int g = T.rs[r] + (k - T.ro[r]);
        double f[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) f[c] = V.acc[6 * k + c];
        store_ft(B.nb + 6LL * ((r - 1) * B.n + g), f);
    }
    if constexpr (Sum) {
        if constexpr (Wave)
            reduce_tally(tally, T.red, partials, P.pstride, grow);
        else
            reduce_fill(tally.fill, T.red, partials, P.pstride, grow);
    }
    return;
  }
per_particle:
    defer_row();
}

// ----------------------------------------------------------------------------------
// k_pairs_ec: with the electro-chemical ranges (Fig. elch: repulsion, eq. rep, while the
// surface distance is below 20 lambda_D, attraction, eq. att, below 4 a0) on a lattice sized
// for the lubrication list alone, the pairs beyond that list, c (a_i + a_j) <= |r| <
// a_i + a_j + rext.  Such a pair carries only the central electro-chemical force (no
// lubrication, no contact since c >= 1, no torque).  Each particle gathers its own force over
// the cell rows within its reach a_i + a_max + rext (rows whose y-z distance exceeds it are
// skipped; a row reached across a y face is searched around the x shifted by the
// Lees-Edwards offset, as in the half shell), so every pair is seen from both sides and
// nothing is accumulated across particles: the force goes to the atomic record by a plain
// store (the row tiles' deferred rows add to it afterwards).  kEcLanes consecutive lanes share
// a particle, each taking every kEcLanes-th row of its (2 R_z + 1) x (2 R_y + 1) rows, and
// their sums are combined by a fixed butterfly, so that enough wavefronts are in flight to
// cover the latency of the candidate loads.  A lane only tests its candidates (four loads in
// flight, each with the image of its window part) and keeps the far ones in LDS; their forces
// are taken when some lane of the wavefront could overflow its kEcBuf entries (and at the
// end), by all lanes at once, so the force arithmetic runs about once per far pair instead
// of once per candidate of the wavefront.  The split of the pair set is exact: the tiles take
// r^2 < (c s)^2 and this kernel (c s)^2 <= r^2 < (s + rext)^2 with the same FP64 r^2 (the
// nearest image is antisymmetric), whose union is the list r^2 < max(c s, s + rext)^2.  Each
// side adds half of the pair's stresslet r (x) F_i; the pair is counted and recorded by its
// smaller slot.  Sum: the stress and pair count of the workgroup go to partial record
// rec0 + block.
// ----------------------------------------------------------------------------------
constexpr int kEcLanes = 8;
constexpr int kEcBuf = 16;  // far partners a lane holds before their forces are taken
constexpr int kEcChunk = 4;  // candidate loads of a lane in flight together

// Central electro-chemical force of a far pair (i, j) on i, r = x_j - x_i (eqs. rep, att).
__device__ __forceinline__ double ec_far_force(const DevParams &P, double dist, double ai, double aj)
{
    const double h = dist - ai - aj;
    const double abar = 2.0 * ai * aj / (ai + aj);
    double fe = 0.0;
    if (P.fer != 0.0 && h < P.rep_rng) fe -= P.fer_a0 * abar * (P.lamd > 0.0 ? exp(-h * P.inv_lamd) : 0.0);
    if (P.ham != 0.0 && h < P.att_rng) {
        const double e = P.eps_vdw * abar;
        fe += P.ham * abar / (12.0 * (h * h + e * e));
    }
    return fe;
}

template <bool Sum>
__global__ void __launch_bounds__(kBlock) k_pairs_ec(DevParams P, const BoxParams *__restrict__ boxes,
                                                      const int *__restrict__ cell_start,
                                                      const double4 *__restrict__ pa,
                                                      const double4 *__restrict__ omg, double *__restrict__ fx,
                                                      DevClock *__restrict__ clk, double *__restrict__ partials,
                                                      int rec0, int *__restrict__ pair_out,
                                                      unsigned long long *__restrict__ pair_count)
{
    __shared__ double red[kBlock / 64][12];
    __shared__ int fbuf[kEcBuf][kBlock];  // far partners of each lane, taken in wavefront-uniform flushes
    const int t = threadIdx.x;
    const int sub = t & (kEcLanes - 1);
    const int i = (blockIdx.x * kBlock + t) / kEcLanes;
    const BoxParams G = boxes[0];
    PairTally tally;
#pragma unroll
    for (int k = 0; k < 9; ++k) tally.S[k] = 0.0;
    tally.npair = tally.ncont = 0;
    tally.fill = 0;
    double f[3] = {0.0, 0.0, 0.0};
    const bool on = i < P.N;
    const double4 Xi = on ? pa[i] : make_double4(0.0, 0.0, 0.0, 1.0);
    const double delta = le_offset(P, G, clk->step);
    const int idi = (on && P.record_pairs) ? (int)omg[i].w : 0;
    int nb = 0;
    // forces of the buffered far partners (every lane of the wavefront at once)
    auto flush = [&]() {
        for (int b = 0; b < nb; ++b) {
            const int j = fbuf[b][t];
            const double4 Xj = pa[j];
            double dx, dy_, dz_;
            min_image(G, delta, Xi.x, Xi.y, Xi.z, Xj.x, Xj.y, Xj.z, dx, dy_, dz_);
            double r2;
            {
#pragma clang fp contract(off)
                r2 = (dx * dx + dy_ * dy_) + dz_ * dz_;
            }
            const double dist = sqrt(r2);
            const double g = ec_far_force(P, dist, Xi.w, Xj.w) / dist;
            const double F[3] = {g * dx, g * dy_, g * dz_};
            f[0] += F[0];
            f[1] += F[1];
            f[2] += F[2];
            if constexpr (Sum) {
                const double r[3] = {dx, dy_, dz_};
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) tally.S[3 * a + c] += 0.5 * r[a] * F[c];
            }
            if (i < j) {
                ++tally.npair;
                if (P.record_pairs) record_pair(P, idi, (int)omg[j].w, pair_out, pair_count, clk);
            }
        }
        nb = 0;
    };
    const int nxc = G.nc[0], nyc = G.nc[1], nzc = G.nc[2];
    const int cy = cell_coord(Xi.y, G.cw[1], nyc), cz = cell_coord(Xi.z, G.cw[2], nzc);
    const double reach = Xi.w + P.ec_amax + P.rext;  // >= a_i + a_j + rext for every j
    const int ny = 2 * P.ec_ry + 1, nrows = on ? ny * (2 * P.ec_rz + 1) : 0;
    for (int q = sub; q < nrows; q += kEcLanes) {
        const int dz = q / ny - P.ec_rz, dy = q - (q / ny) * ny - P.ec_ry;
        const int zu = cz + dz, yu = cy + dy;
        const double zlo = (double)zu * G.cw[2], ylo = (double)yu * G.cw[1];
        const double ez = fmax(0.0, fmax(zlo - Xi.z, Xi.z - (zlo + G.cw[2])));
        const double ey = fmax(0.0, fmax(ylo - Xi.y, Xi.y - (ylo + G.cw[1])));
        const double e2 = ey * ey + ez * ez;
        if (e2 >= reach * reach) continue;
        const int zz = zu < 0 ? zu + nzc : (zu >= nzc ? zu - nzc : zu);
        const int cross = yu >= nyc ? 1 : (yu < 0 ? -1 : 0);
        const int yy = yu < 0 ? yu + nyc : (yu >= nyc ? yu - nyc : yu);
        // images across the top face are displaced by +delta: look around x - delta; a partner
        // within reach lies within sqrt(reach^2 - e^2) along x of the row at y-z distance e
        const double xs = Xi.x + (cross > 0 ? -delta : (cross < 0 ? delta : 0.0));
        const double hw = sqrt(reach * reach - e2);
        const int xlo = (int)floor((xs - hw) / G.cw[0]);
        const int xhi = (int)floor((xs + hw) / G.cw[0]);
        int span = xhi - xlo + 1;
        // a window of the whole row (never on a lattice that passes the host's check) takes the
        // nearest image candidate by candidate; otherwise every candidate of a part has the
        // image of the part: y and z shifts of the row, the Lees-Edwards shift of a row across
        // a y face, and the period of the part along x.  These are the operations min_image
        // applies to a partner within reach (the periodic shifts are exact), so r^2 is the same
        // to the bit; a partner beyond reach stays beyond it under either image.
        const bool whole = span >= nxc;
        span = whole ? nxc : span;
        const int w0 = xlo >= 0 ? xlo / nxc : -((-xlo + nxc - 1) / nxc);  // floor(xlo / n_x)
        int xl = xlo - w0 * nxc;
        const double sy = cross > 0 ? G.L[1] : (cross < 0 ? -G.L[1] : 0.0);
        const double sxd = cross > 0 ? delta : (cross < 0 ? -delta : 0.0);
        const double sz = zu >= nzc ? G.L[2] : (zu < 0 ? -G.L[2] : 0.0);
        const int rbase = G.cell_off + (zz * nyc + yy) * nxc;
        for (int part = 0; part < 2 && span > 0; ++part) {
            const int len = (xl + span <= nxc) ? span : nxc - xl;
            const int jb = cell_start[rbase + xl];
            const int je = cell_start[rbase + xl + len];
            const double sxw = (double)(w0 + part) * G.L[0];
            // candidates in chunks of kEcChunk whose loads are in flight together
            for (int j0 = jb; j0 < je; j0 += kEcChunk) {
                if (__any(nb > kEcBuf - kEcChunk)) flush();
                double4 Xc[kEcChunk];
#pragma unroll
                for (int u = 0; u < kEcChunk; ++u) Xc[u] = pa[j0 + u < je ? j0 + u : j0];
#pragma unroll
                for (int u = 0; u < kEcChunk; ++u) {
                    const int j = j0 + u;
                    bool far;
                    {
#pragma clang fp contract(off)
                        double dx, dy_, dz_;
                        if (whole) {
                            min_image(G, delta, Xi.x, Xi.y, Xi.z, Xc[u].x, Xc[u].y, Xc[u].z, dx, dy_, dz_);
                        } else {
                            dx = ((Xc[u].x - Xi.x) + sxd) + sxw;
                            dy_ = (Xc[u].y - Xi.y) + sy;
                            dz_ = (Xc[u].z - Xi.z) + sz;
                        }
                        const double r2 = (dx * dx + dy_ * dy_) + dz_ * dz_;
                        const double s = Xi.w + Xc[u].w;
                        const double rl = P.cf * s, re = s + P.rext;
                        far = j < je && j != i && !(r2 < rl * rl) && r2 < re * re;
                    }
                    if (far) fbuf[nb++][t] = j;
                }
            }
            xl = 0;
            span -= len;
        }
    }
    flush();
    // the particle's force: the kEcLanes partial sums combined in a fixed order
#pragma unroll
    for (int o = 1; o < kEcLanes; o <<= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c] += __shfl_xor(f[c], o, 64);
    }
    if (on && sub == 0) {
        const double out[6] = {f[0], f[1], f[2], 0.0, 0.0, 0.0};
        store_ft(fx + 6LL * i, out);
        if (!finite6(out)) atomicOr(&clk->err, kErrNonFinite);
    }
    if constexpr (Sum) reduce_tally(tally, red, partials, P.pstride, rec0 + blockIdx.x);
}

// ----------------------------------------------------------------------------------
// k_finish: one workgroup of kBlock lanes per (box, component) of the 12 partial-record
// components (9 stress components, listed pairs, contacts, largest history row): the sum
// (the maximum for the last) of the box's records in a fixed order (lane t takes records
// t, t + kBlock, ..., then the wavefronts and the waves in order), so the stress does not
// depend on scheduling; the workgroup publishes its component of the box's stress or
// counters, and the stress sample of the current time index when the schedule asks for it.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_finish(const BoxParams *__restrict__ boxes,
                                                    const double *__restrict__ partials, int pstride,
                                                    DevClock *__restrict__ clk, DevRun *__restrict__ run, int sample)
// partials: 12 components x pstride records
{
    __shared__ double red[kBlock / 64];
    const int t = threadIdx.x;
    const int b = blockIdx.x / 12, k = blockIdx.x - (blockIdx.x / 12) * 12;
    const BoxParams &G = boxes[b];
    const int r0 = G.row_off, nrow = G.nrec;
    const double *src = partials + (long long)k * pstride + r0;
    double acc = 0.0;
    if (k == 11) {
        for (int w = t; w < nrow; w += kBlock) acc = fmax(acc, src[w]);
        for (int o = 32; o > 0; o >>= 1) acc = fmax(acc, __shfl_xor(acc, o, 64));
    } else {
        for (int w = t; w < nrow; w += kBlock) acc += src[w];
        acc = warp_sum(acc);
    }
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t != 0) return;
    double x = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) x = (k == 11) ? fmax(x, red[w]) : x + red[w];
    if (k < 9) {
        run->sigma_last[9 * b + k] = x;
        const long long n = clk->step;
        if (sample && run->sample_every > 0 && n % run->sample_every == 0 && n >= run->sample_first) {
            const long long slot = (n - run->sample_first) / run->sample_every;
            if (slot < run->sample_cap) run->samples[(slot * (gridDim.x / 12) + b) * 9 + k] = x;
        }
    } else {
        run->box_diag[3 * b + (k - 9)] = x;
    }
}

// ----------------------------------------------------------------------------------
// k_history_move: after a counting sort without time advance, the committed contact history
// follows its particles to their new slots: row q of the new buffers = row prev[q] of the
// old ones (keys, stretches, rolling stretches when xr_old is set, fill, owner id).
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_history_move(int N, int M, const int *__restrict__ prev,
                                                          const int *__restrict__ key_old,
                                                          const double *__restrict__ xi_old,
                                                          const double *__restrict__ xr_old,
                                                          const int *__restrict__ cnt_old,
                                                          const int *__restrict__ own_old, int *__restrict__ key_new,
                                                          double *__restrict__ xi_new, double *__restrict__ xr_new,
                                                          int *__restrict__ cnt_new, int *__restrict__ own_new)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int p = prev[q];
    const int n = cnt_old[p];
    cnt_new[q] = n;
    own_new[q] = own_old[p];
    for (int k = 0; k < n; ++k) {
        const long long src = (long long)p * M + k, dst = (long long)q * M + k;
        key_new[dst] = key_old[src];
        xi_new[3 * dst] = xi_old[3 * src];
        xi_new[3 * dst + 1] = xi_old[3 * src + 1];
        xi_new[3 * dst + 2] = xi_old[3 * src + 2];
        if (xr_old) {
            xr_new[3 * dst] = xr_old[3 * src];
            xr_new[3 * dst + 1] = xr_old[3 * src + 1];
            xr_new[3 * dst + 2] = xr_old[3 * src + 2];
        }
    }
}

// ----------------------------------------------------------------------------------
// k_unsort: state by particle id.  Completes u^n = vel + dt/2 F/m when vel holds the
// half-step velocity and complete != 0.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_unsort(DevParams P, const double4 *__restrict__ pa,
                                                    const double4 *__restrict__ vel, const double4 *__restrict__ omg,
                                                    ForceBufs B, int vel_is_half, int complete,
                                                    double *__restrict__ x, double *__restrict__ u,
                                                    double *__restrict__ w, double *__restrict__ F,
                                                    double *__restrict__ T)
{
#pragma clang fp contract(off)
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.N) return;
    double4 X = pa[p], V = vel[p], W = omg[p];
    double f[6];
    total_ft(B, p, f);
    int id = (int)W.w;
    if (vel_is_half && complete) {
        double m = pmass(P, X.w);
        double I = 0.4 * m * X.w * X.w;
        const double dt = P.dt;
        V.x = V.x + 0.5 * dt * (f[0] / m);
        V.y = V.y + 0.5 * dt * (f[1] / m);
        V.z = V.z + 0.5 * dt * (f[2] / m);
        W.x = W.x + 0.5 * dt * (f[3] / I);
        W.y = W.y + 0.5 * dt * (f[4] / I);
        W.z = W.z + 0.5 * dt * (f[5] / I);
    }
    if (x) { x[3 * id] = X.x; x[3 * id + 1] = X.y; x[3 * id + 2] = X.z; }
    if (u) { u[3 * id] = V.x; u[3 * id + 1] = V.y; u[3 * id + 2] = V.z; }
    if (w) { w[3 * id] = W.x; w[3 * id + 1] = W.y; w[3 * id + 2] = W.z; }
    if (F) { F[3 * id] = f[0]; F[3 * id + 1] = f[1]; F[3 * id + 2] = f[2]; }
    if (T) { T[3 * id] = f[3]; T[3 * id + 1] = f[4]; T[3 * id + 2] = f[5]; }
}

// k_load: particles by id -> unsorted records (slot = id), force records cleared.
__global__ void __launch_bounds__(kBlock) k_load(int N, const double *__restrict__ x, const double *__restrict__ rad,
                                                  const double *__restrict__ u, const double *__restrict__ w,
                                                  const int *__restrict__ pbox, const BoxParams *__restrict__ boxes,
                                                  double4 *__restrict__ pa, double4 *__restrict__ vel,
                                                  double4 *__restrict__ omg, ForceBufs B, double wave_amp)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int b = pbox[p];
    const double gd = boxes[b].gd, wk = boxes[b].wk;
    const double y = x[3 * p + 1];
    // ambient velocity and rotation at the particle (with the wave of eq. uinf)
    const double Ux = wave_amp != 0.0 ? gd * y + wave_amp * sin(wk * y) : gd * y;
    const double Wz = wave_amp != 0.0 ? -0.5 * (gd + wave_amp * wk * cos(wk * y)) : -0.5 * gd;
    pa[p] = make_double4(x[3 * p], x[3 * p + 1], x[3 * p + 2], rad[p]);
    // vel.w carries the particle's box index through every reorder
    if (u)
        vel[p] = make_double4(u[3 * p], u[3 * p + 1], u[3 * p + 2], (double)b);
    else
        vel[p] = make_double4(Ux, 0.0, 0.0, (double)b);
    if (w)
        omg[p] = make_double4(w[3 * p], w[3 * p + 1], w[3 * p + 2], (double)p);
    else
        omg[p] = make_double4(0.0, 0.0, Wz, (double)p);
    const double z[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    store_ft(B.own + 6LL * p, z);
    store_ft(B.x + 6LL * p, z);
    for (int r = 0; r < 4; ++r) store_ft(B.nb + 6LL * (r * B.n + p), z);
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
        const int partner = key[(long long)p * M + k] & kKeyMask;
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
