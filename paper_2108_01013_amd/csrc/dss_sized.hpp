// Size-class stencils for boxes of high size ratio (the remedy named in Section 2.2 of the
// paper: a cell spacing suited to the smallest particles, with the search stencil widened
// for the larger ones, as in Hoetzlein's and LAMMPS's multi-size searches).
//
// Lattice: spacing cw >= cell_scale x 2 c a_min.  Particle i of radius a_i belongs to size
// class k_i = floor(a_i cls_mul), cls_mul = 2 c (1 + 1e-9) / min(cw); its stencil radius is
// R_i = k_i + 1 cells, so R_i cw > 2 c a_i >= c (a_i + a_j) for every partner j with
// a_j <= a_i.  The counting sort is class-major (cell id = k n_cells + cell), so the slots of
// class k are one contiguous, spatially sorted block, and a wavefront of consecutive slots
// holds one class (uniform stencil work).
//
// Ownership: a pair is found once, by its larger member under the key (a, slot): i scans
// classes 0 .. k_i of every cell of its (2 R_i + 1)^3 stencil (2 R_i + 2 x-cells in a row
// reached across a sheared y face), and within its own class only partners of smaller key.
// The owner keeps its side in registers (its own record, with the Stokes terms) and adds the
// partner side atomically to the atomic force record; the contact-history row of the pair is
// the owner's.  Classes from wave_cls up take one wavefront per particle (lanes split the
// stencil rows); the others one lane per particle; both in one launch.
//
// Requirements checked on the host: one box, n_x >= 2 R_max + 2, n_y, n_z >= 2 R_max + 1
// (no cell is reached twice), partial records at most 4096.
#pragma once

#include "dss_kernels.hpp"

namespace dss {

// Candidates of particle i (slot i, class ci) in stencil row (dz, dy): both pieces of the
// (wrapped) x window, classes 0 .. ci.  Calls visit(j, x_j) for every slot j of smaller key.
template <typename Visit>
__device__ __forceinline__ void sized_row(const BoxParams &G, const int *__restrict__ cell_start,
                                          const double4 *__restrict__ pa, int i, const double4 &Xi, int ci, int cx,
                                          int cy, int cz, int dy, int dz, double delta, Visit &&visit)
{
#pragma clang fp contract(off)
    const int nxc = G.nc[0], nyc = G.nc[1], nzc = G.nc[2];
    const int R = ci + 1;
    int zz = cz + dz;
    zz = zz < 0 ? zz + nzc : (zz >= nzc ? zz - nzc : zz);
    int yy = cy + dy;
    const int cross = yy >= nyc ? 1 : (yy < 0 ? -1 : 0);
    yy = yy < 0 ? yy + nyc : (yy >= nyc ? yy - nyc : yy);
    int xlo, xhi;
    if (cross != 0) {
        // top face: images displaced by +delta, so look around x - delta; bottom: x + delta
        const double sh = cross > 0 ? -delta : delta;
        const int k0 = (int)floor(((double)cx * G.cw[0] + sh) / G.cw[0]);
        xlo = k0 - R;
        xhi = k0 + R + 1;
    } else {
        xlo = cx - R;
        xhi = cx + R;
    }
    const int ncb = nxc * nyc * nzc;
    const int rowc = G.cell_off + (zz * nyc + yy) * nxc;
    int xl = ((xlo % nxc) + nxc) % nxc;
    int span = xhi - xlo + 1;
    for (int part = 0; part < 2 && span > 0; ++part) {
        const int len = (xl + span <= nxc) ? span : nxc - xl;
        for (int k = 0; k <= ci; ++k) {
            const int c0 = k * ncb + rowc + xl;
            const int jb = cell_start[c0];
            const int je = cell_start[c0 + len];
            for (int j = jb; j < je; ++j) {
                const double4 Xj = pa[j];
                if (k == ci && !(Xj.w < Xi.w || (Xj.w == Xi.w && j < i))) continue;
                visit(j, Xj);
            }
        }
        xl = 0;
        span -= len;
    }
}

// One listed-candidate test and, for a listed pair, its physics; partner side atomically.
template <typename Real, bool Roll, bool Wave>
__device__ __forceinline__ void sized_pair(const DevParams &P, const BoxParams &G, const HistView &H, int i, int j,
                                           int idi, const double4 &Xi, const double4 &Vi, const double4 &Wi,
                                           const double4 &Xj, double delta,
                                           const double4 *__restrict__ vel, const double4 *__restrict__ omg,
                                           const ForceBufs &B, DevClock *clk, int *pair_out,
                                           unsigned long long *pair_count, PairTally &tally, double f[6],
                                           int &contact_slot_needed, PairOut &o, int &idj)
{
    contact_slot_needed = 0;
    double dx, dy2, dz2, r2;
    min_image(G, delta, Xi.x, Xi.y, Xi.z, Xj.x, Xj.y, Xj.z, dx, dy2, dz2);
    if (!listed(P, dx, dy2, dz2, Xi.w, Xj.w, r2)) return;
    const double4 Vj = vel[j];
    const double4 Wj = omg[j];
    idj = (int)Wj.w;
    ++tally.npair;
    if (P.record_pairs) record_pair(P, idi, idj, pair_out, pair_count, clk);
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
        contact_slot_needed = 1;
    }
}

// ----------------------------------------------------------------------------------
// Lane path: one lane per particle of the classes below wave_cls (slots [0, n_lane), n_lane =
// first slot of class wave_cls), workgroup lb of nlb striding over the slots.
// ----------------------------------------------------------------------------------
template <typename Real, bool Roll, bool Wave>
__device__ __forceinline__ void sized_lane_path(const DevParams &P, const BoxParams &G, const int *__restrict__ cell_start,
                                                const double4 *__restrict__ pa, const double4 *__restrict__ vel,
                                                const double4 *__restrict__ omg, const ForceBufs &B, const HistView &H,
                                                DevClock *clk, int *pair_out, unsigned long long *pair_count,
                                                double delta, int n_lane, int lb, int nlb, PairTally &tally)
{
    for (int i = lb * kBlock + threadIdx.x; i < n_lane; i += nlb * kBlock) {
        const double4 Xi = pa[i];
        const double4 Vi = vel[i];
        const double4 Wi = omg[i];
        const int idi = (int)Wi.w;
        const int ci = size_class(P, Xi.w);
        const int R = ci + 1;
        const int cx = cell_coord(Xi.x, G.cw[0], G.nc[0]);
        const int cy = cell_coord(Xi.y, G.cw[1], G.nc[1]);
        const int cz = cell_coord(Xi.z, G.cw[2], G.nc[2]);
        double f[6] = {0, 0, 0, 0, 0, 0};
        int fill = 0;
        for (int dz = -R; dz <= R; ++dz)
            for (int dy = -R; dy <= R; ++dy)
                sized_row(G, cell_start, pa, i, Xi, ci, cx, cy, cz, dy, dz, delta, [&](int j, const double4 &Xj) {
                    int need, idj = 0;
                    PairOut o;
                    sized_pair<Real, Roll, Wave>(P, G, H, i, j, idi, Xi, Vi, Wi, Xj, delta, vel, omg, B, clk, pair_out,
                                           pair_count, tally, f, need, o, idj);
                    if (need) {
                        store_history<Roll>(H, P.M, i, fill, idi, idj, o, clk);
                        ++fill;
                    }
                });
        finish_row<Roll>(H, P.M, i, fill, idi);
        tally.fill = max(tally.fill, fill);
        stokes_terms<Wave>(P, G, Xi, Vi, Wi, f, tally.S);
        store_ft(B.own + 6LL * i, f);
        if (!finite6(f)) atomicOr(&clk->err, kErrNonFinite);
    }
}

// Sort a history row of n entries by partner id with the 64 lanes of a wavefront: every lane
// holds entries lane, lane + 64, ... (at most kWaveSortChunks each), ranks them against all n
// keys, then stores them at their ranks.  Longer rows are sorted by lane 0 alone.
constexpr int kWaveSortChunks = 4;

template <bool Roll>
__device__ __forceinline__ void wave_finish_row(const HistView &H, int M, int gi, int fill, int idi)
{
    const int lane = threadIdx.x & 63;
    const int n = fill < M ? fill : M;
    if (n > 64 * kWaveSortChunks) {
        if (lane == 0) finish_row<Roll>(H, M, gi, fill, idi);
        return;
    }
    int *krow = H.key_new + (long long)gi * M;
    double *xrow = H.xi_new + (long long)gi * M * 3;
    double *rrow = Roll ? H.xr_new + (long long)gi * M * 3 : nullptr;
    int key[kWaveSortChunks], rank[kWaveSortChunks];
    double x0[kWaveSortChunks], x1[kWaveSortChunks], x2[kWaveSortChunks];
    double y0[kWaveSortChunks], y1[kWaveSortChunks], y2[kWaveSortChunks];
#pragma unroll
    for (int m = 0; m < kWaveSortChunks; ++m) {
        const int e = lane + 64 * m;
        key[m] = e < n ? krow[e] : 0;
        rank[m] = 0;
        if (e < n) {
            x0[m] = xrow[3 * e];
            x1[m] = xrow[3 * e + 1];
            x2[m] = xrow[3 * e + 2];
            if constexpr (Roll) {
                y0[m] = rrow[3 * e];
                y1[m] = rrow[3 * e + 1];
                y2[m] = rrow[3 * e + 2];
            }
        }
    }
    for (int e = 0; e < n; ++e) {
        const int ke = krow[e] & kKeyMask;
#pragma unroll
        for (int m = 0; m < kWaveSortChunks; ++m) rank[m] += ke < (key[m] & kKeyMask) ? 1 : 0;
    }
    // every lane has read the whole row (the ranks depend on all of it) before any store
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int m = 0; m < kWaveSortChunks; ++m) {
        const int e = lane + 64 * m;
        if (e < n) {
            const int d = rank[m];
            krow[d] = key[m];
            xrow[3 * d] = x0[m];
            xrow[3 * d + 1] = x1[m];
            xrow[3 * d + 2] = x2[m];
            if constexpr (Roll) {
                rrow[3 * d] = y0[m];
                rrow[3 * d + 1] = y1[m];
                rrow[3 * d + 2] = y2[m];
            }
        }
    }
    if (lane == 0) {
        H.cnt_new[gi] = n;
        H.own_new[gi] = idi;
    }
}

// ----------------------------------------------------------------------------------
// Wavefront path: one wavefront per particle of the classes from wave_cls up (slots
// [n_lane, N)), workgroup wb of nwb; lanes stride over the (2R+1)^2 stencil rows, contacts
// take their history slots from a per-wavefront LDS counter, the wavefront sums its own side
// and sorts the row.
// ----------------------------------------------------------------------------------
template <typename Real, bool Roll, bool Wave>
__device__ __forceinline__ void sized_wave_path(const DevParams &P, const BoxParams &G, const int *__restrict__ cell_start,
                                                const double4 *__restrict__ pa, const double4 *__restrict__ vel,
                                                const double4 *__restrict__ omg, const ForceBufs &B, const HistView &H,
                                                DevClock *clk, int *pair_out, unsigned long long *pair_count,
                                                double delta, int n_lane, int wb, int nwb, int *wfill,
                                                PairTally &tally)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nwave = nwb * (kBlock / 64);
    for (int i = n_lane + wb * (kBlock / 64) + wid; i < P.N; i += nwave) {
        const double4 Xi = pa[i];
        const double4 Vi = vel[i];
        const double4 Wi = omg[i];
        const int idi = (int)Wi.w;
        const int ci = size_class(P, Xi.w);
        const int R = ci + 1, side = 2 * R + 1;
        const int cx = cell_coord(Xi.x, G.cw[0], G.nc[0]);
        const int cy = cell_coord(Xi.y, G.cw[1], G.nc[1]);
        const int cz = cell_coord(Xi.z, G.cw[2], G.nc[2]);
        if (lane == 0) wfill[wid] = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        double f[6] = {0, 0, 0, 0, 0, 0};
        for (int q = lane; q < side * side; q += 64) {
            const int dz = q / side - R, dy = q % side - R;
            sized_row(G, cell_start, pa, i, Xi, ci, cx, cy, cz, dy, dz, delta, [&](int j, const double4 &Xj) {
                int need, idj = 0;
                PairOut o;
                sized_pair<Real, Roll, Wave>(P, G, H, i, j, idi, Xi, Vi, Wi, Xj, delta, vel, omg, B, clk, pair_out,
                                       pair_count, tally, f, need, o, idj);
                if (need) store_history<Roll>(H, P.M, i, atomicAdd(&wfill[wid], 1), idi, idj, o, clk);
            });
        }
        // the row's entries, written by all lanes, are visible to the whole wavefront
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const int fill = wfill[wid];
#pragma unroll
        for (int k = 0; k < 6; ++k) f[k] = warp_sum(f[k]);
        wave_finish_row<Roll>(H, P.M, i, fill, idi);
        if (lane == 0) {
            tally.fill = max(tally.fill, fill);
            stokes_terms<Wave>(P, G, Xi, Vi, Wi, f, tally.S);
            store_ft(B.own + 6LL * i, f);
            if (!finite6(f)) atomicOr(&clk->err, kErrNonFinite);
        }
    }
}

// ----------------------------------------------------------------------------------
// k_pairs_sized: workgroups [0, g_wave) take the wavefront path (the long-running large
// particles start first), the others the lane path over XCD-contiguous slot blocks (see
// xcd_row; g_wave is a multiple of 8, so the XCD of a lane workgroup is unchanged).  Partial
// record = blockIdx.x, written only when Sum (a step whose stress is summed).
// ----------------------------------------------------------------------------------
template <typename Real, bool Roll, bool Wave, bool Sum>
__global__ void __launch_bounds__(kBlock, 2) k_pairs_sized(DevParams P, const BoxParams *__restrict__ boxes,
                                                        const int *__restrict__ cell_start,
                                                        const double4 *__restrict__ pa,
                                                        const double4 *__restrict__ vel,
                                                        const double4 *__restrict__ omg, ForceBufs B, HistView H,
                                                        DevClock *__restrict__ clk, double *__restrict__ partials,
                                                        int g_wave, int *__restrict__ pair_out,
                                                        unsigned long long *__restrict__ pair_count)
{
    __shared__ double red[kBlock / 64][12];
    __shared__ int wfill[kBlock / 64];
    const BoxParams G = boxes[0];
    const int ncb = G.nc[0] * G.nc[1] * G.nc[2];
    const int n_lane = P.wave_cls < P.ncls ? cell_start[P.wave_cls * ncb] : P.N;
    const double delta = le_offset(P, G, clk->step);
    if (blockIdx.x == 0 && threadIdx.x == 0) clk->deferred = 1;  // the atomic record is in use
    PairTally tally;
#pragma unroll
    for (int k = 0; k < 9; ++k) tally.S[k] = 0.0;
    tally.npair = tally.ncont = 0;
    tally.fill = 0;
    const int b = blockIdx.x;
    if (b < g_wave)
        sized_wave_path<Real, Roll, Wave>(P, G, cell_start, pa, vel, omg, B, H, clk, pair_out, pair_count, delta, n_lane, b,
                                    g_wave, wfill, tally);
    else
        sized_lane_path<Real, Roll, Wave>(P, G, cell_start, pa, vel, omg, B, H, clk, pair_out, pair_count, delta, n_lane,
                                    xcd_row(b - g_wave, (int)gridDim.x - g_wave), (int)gridDim.x - g_wave, tally);
    if constexpr (Sum) reduce_tally(tally, red, partials, P.pstride, b);
}

}  // namespace dss
