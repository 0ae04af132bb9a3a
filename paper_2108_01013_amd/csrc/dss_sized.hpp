// Size-class stencils for boxes of high size ratio (the remedy named in Section 2.2 of the
// paper: a cell spacing suited to the smallest particles, with the search stencil widened
// for the larger ones, as in Hoetzlein's and LAMMPS's multi-size searches).
//
// Lattice: spacing cw >= cell_scale x 2 c a_min.  Particle i of radius a_i belongs to size
// class k_i = floor(a_i cls_mul), cls_mul = 2 c (1 + 1e-9) / min(cw); its stencil radius is
// R_i = k_i + 1 cells, so R_i cw > 2 c a_i >= c (a_i + a_j) for every partner j with
// a_j <= a_i.  With the electro-chemical ranges the reach is 2 max(c, 1) a_i + rext, which
// bounds max(c (a_i + a_j), a_i + a_j + rext): the class is floor(a_i cls_mul + cls_add) with
// cls_add = rext (1 + 1e-9) / min(cw), on a lattice of spacing >= the smallest reach.  The counting sort is class-major (cell id = k n_cells + cell), so the slots of
// class k are one contiguous, spatially sorted block, and a wavefront of consecutive slots
// holds one class (uniform stencil work).
//
// Ownership: a pair is found once, by its larger member under the key (a, slot): i scans
// classes 0 .. k_i of every cell of its (2 R_i + 1)^3 stencil (2 R_i + 2 x-cells in a row
// reached across a sheared y face), and within its own class only partners of smaller key.
// The owner's side goes into its own record (with the Stokes terms), the partner side
// atomically into the atomic force record; the contact-history row of the pair is the
// owner's.  Classes from wave_cls up take one wavefront per particle (lanes split the stencil
// rows); the others one lane per particle; both in one launch.  Scans queue their listed
// pairs in LDS and the pair physics runs on the queue with every lane busy, instead of in
// the lane that found the pair (a wavefront would otherwise run the physics for one or two
// hit lanes at a time).
//
// Requirements checked on the host: one box, n_x >= 2 R_max + 2, n_y, n_z >= 2 R_max + 1
// (no cell is reached twice), partial records at most 4096.
#pragma once

#include "dss_kernels.hpp"

namespace dss {

// Stencil cursor of particle i (slot i, class ci): items (row, window piece, class) over the
// stencil rows q = q0, q0 + qstep, ... of the (2R+1)^2 rows (dz, dy), both pieces of each
// row's (wrapped) x window, classes 0 .. ci, and the slots of each item's cell range.  The
// range of the following item is requested when an item begins, so that its cell-start loads
// overlap the candidates of the current one.  Resumable: a scan that cannot queue a listed
// candidate stops on it and takes it up again in the next round.
struct StencilCursor {
    int q, part, k;     // current item: stencil row, window piece, class
    int j, je;          // its slot range; the next candidate is j
    int done;
    int nq, npart, nk;  // the following item, its range already requested
    int nj, nje;
    int ndone;
};

// The item after (q, part, k) for a lane striding qstep rows: classes, then pieces, then rows.
__device__ __forceinline__ void item_advance(int ci, int qstep, int &q, int &part, int &k, int &done)
{
    if (++k > ci) {
        k = 0;
        if (++part > 1) {
            part = 0;
            q += qstep;
            if (q >= (2 * ci + 3) * (2 * ci + 3)) done = 1;
        }
    }
}

// Slot range [j, je) of item (q, part, k).  A row reached across a sheared y face is the
// window of 2R + 2 x-cells around the displaced position (images shifted by +delta at the top
// face, so the window is centred on x - delta there, on x + delta at the bottom face).
__device__ __forceinline__ void item_range(const BoxParams &G, const int *__restrict__ cell_start, int ci, int cx,
                                           int cy, int cz, double delta, int q, int part, int k, int &j, int &je)
{
#pragma clang fp contract(off)
    const int nxc = G.nc[0], nyc = G.nc[1], nzc = G.nc[2];
    const int R = ci + 1, side = 2 * R + 1;
    const int dz = q / side - R, dy = q - (q / side) * side - R;
    int zz = cz + dz;
    zz = zz < 0 ? zz + nzc : (zz >= nzc ? zz - nzc : zz);
    int yy = cy + dy;
    const int cross = yy >= nyc ? 1 : (yy < 0 ? -1 : 0);
    yy = yy < 0 ? yy + nyc : (yy >= nyc ? yy - nyc : yy);
    int xlo, xhi;
    if (cross != 0) {
        const double sh = cross > 0 ? -delta : delta;
        const int k0 = (int)floor(((double)cx * G.cw[0] + sh) / G.cw[0]);
        xlo = k0 - R;
        xhi = k0 + R + 1;
    } else {
        xlo = cx - R;
        xhi = cx + R;
    }
    const int xl = ((xlo % nxc) + nxc) % nxc;
    const int span = xhi - xlo + 1;
    const int len0 = (xl + span <= nxc) ? span : nxc - xl;
    const int x0 = part == 0 ? xl : 0;
    const int len = part == 0 ? len0 : span - len0;
    if (len <= 0) {
        j = je = 0;
        return;
    }
    const int c0 = k * (nxc * nyc * nzc) + G.cell_off + (zz * nyc + yy) * nxc + x0;
    j = cell_start[c0];
    je = cell_start[c0 + len];
}

// Request the range of the following item (or mark the cursor's end).
__device__ __forceinline__ void cursor_prefetch(const BoxParams &G, const int *__restrict__ cell_start, int ci, int cx,
                                                int cy, int cz, double delta, int qstep, StencilCursor &C)
{
    C.nq = C.q;
    C.npart = C.part;
    C.nk = C.k;
    C.ndone = 0;
    C.nj = C.nje = 0;
    item_advance(ci, qstep, C.nq, C.npart, C.nk, C.ndone);
    if (!C.ndone) item_range(G, cell_start, ci, cx, cy, cz, delta, C.nq, C.npart, C.nk, C.nj, C.nje);
}

__device__ __forceinline__ void cursor_start(const BoxParams &G, const int *__restrict__ cell_start, int ci, int cx,
                                             int cy, int cz, double delta, int q0, int qstep, bool active,
                                             StencilCursor &C)
{
    const int side = 2 * ci + 3;
    C.q = q0;
    C.part = 0;
    C.k = 0;
    C.j = C.je = 0;
    C.done = (!active || q0 >= side * side) ? 1 : 0;
    C.nq = C.npart = C.nk = C.nj = C.nje = 0;
    C.ndone = 1;
    if (!C.done) {
        item_range(G, cell_start, ci, cx, cy, cz, delta, C.q, C.part, C.k, C.j, C.je);
        cursor_prefetch(G, cell_start, ci, cx, cy, cz, delta, qstep, C);
    }
}

// Scan of the listed candidates (pairs of smaller partner key within class ci): push(j) queues
// candidate j and returns false when the queue is full, which ends the scan on j.
template <typename Push>
__device__ __forceinline__ void cursor_scan(const DevParams &P, const BoxParams &G, const int *__restrict__ cell_start,
                                            const double4 *__restrict__ pa, int i, const double4 &Xi, int ci, int cx,
                                            int cy, int cz, double delta, int qstep, StencilCursor &C, Push &&push)
{
    while (!C.done) {
        if (C.j < C.je) {
            const int j = C.j;
            const double4 Xj = pa[j];
            if (C.k != ci || Xj.w < Xi.w || (Xj.w == Xi.w && j < i)) {
                double dx, dy, dz, r2;
                min_image(G, delta, Xi.x, Xi.y, Xi.z, Xj.x, Xj.y, Xj.z, dx, dy, dz);
                if (listed(P, dx, dy, dz, Xi.w, Xj.w, r2) && !push(j)) return;
            }
            C.j = j + 1;
        } else {
            // the following item, whose range was requested when this one began
            C.q = C.nq;
            C.part = C.npart;
            C.k = C.nk;
            C.j = C.nj;
            C.je = C.nje;
            C.done = C.ndone;
            if (!C.done) cursor_prefetch(G, cell_start, ci, cx, cy, cz, delta, qstep, C);
        }
    }
}

// Physics of a queued pair (i, j), partner side atomically; own side added to f.
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

// LDS of a workgroup: the lane path's own-side sums, history slot counters and pair queue, or
// the wavefront path's per-wavefront partner queues.
constexpr int kLaneQ = 4096;
constexpr int kWaveQ = 512;
struct LaneShared {
    double acc[kBlock * 6];
    int cnt[kBlock];
    int qj[kLaneQ];
    unsigned char qi[kLaneQ];
    int qn;
};
struct WaveShared {
    int qj[kBlock / 64][kWaveQ];
    int qn[kBlock / 64];
    int fill[kBlock / 64];
};
union SizedShared {
    LaneShared l;
    WaveShared w;
};

// ----------------------------------------------------------------------------------
// Lane path: one lane per particle of the classes below wave_cls (slots [0, n_lane), n_lane =
// first slot of class wave_cls); workgroup lb of nlb takes blocks of kBlock consecutive slots.
// Every lane scans its stencil and queues its listed candidates in LDS; when the queue is full
// or every scan has ended, all lanes evaluate the queued pairs (own side by LDS atomics,
// history slots from per-particle LDS counters), and the scans resume.
// ----------------------------------------------------------------------------------
template <typename Real, bool Roll, bool Wave>
__device__ __forceinline__ void sized_lane_path(const DevParams &P, const BoxParams &G, const int *__restrict__ cell_start,
                                                const double4 *__restrict__ pa, const double4 *__restrict__ vel,
                                                const double4 *__restrict__ omg, const ForceBufs &B, const HistView &H,
                                                DevClock *clk, int *pair_out, unsigned long long *pair_count,
                                                double delta, int n_lane, int lb, int nlb, int qcap, PairTally &tally,
                                                LaneShared &S)
{
    const int t = threadIdx.x;
    const int cap = qcap > 0 && qcap < kLaneQ ? qcap : kLaneQ;
    for (int base = lb * kBlock; base < n_lane; base += nlb * kBlock) {
        const int i = base + t;
        const bool act = i < n_lane;
        const double4 Xi = pa[act ? i : base];
        const int ci = size_class(P, Xi.w);
        const int cx = cell_coord(Xi.x, G.cw[0], G.nc[0]);
        const int cy = cell_coord(Xi.y, G.cw[1], G.nc[1]);
        const int cz = cell_coord(Xi.z, G.cw[2], G.nc[2]);
        StencilCursor C;
        cursor_start(G, cell_start, ci, cx, cy, cz, delta, 0, 1, act, C);
#pragma unroll
        for (int k = 0; k < 6; ++k) S.acc[6 * t + k] = 0.0;
        S.cnt[t] = 0;
        if (t == 0) S.qn = 0;
        __syncthreads();
        for (;;) {
            cursor_scan(P, G, cell_start, pa, i, Xi, ci, cx, cy, cz, delta, 1, C, [&](int j) -> bool {
                const int e = atomicAdd(&S.qn, 1);
                if (e >= cap) return false;
                S.qj[e] = j;
                S.qi[e] = (unsigned char)t;
                return true;
            });
            __syncthreads();
            const int nq = min(S.qn, cap);
            for (int e = t; e < nq; e += kBlock) {
                const int il = S.qi[e];
                const int gi = base + il;
                const int j = S.qj[e];
                const double4 Xa = pa[gi];
                const double4 Va = vel[gi];
                const double4 Wa = omg[gi];
                const int ida = (int)Wa.w;
                double f[6] = {0, 0, 0, 0, 0, 0};
                int need, idj = 0;
                PairOut o;
                sized_pair<Real, Roll, Wave>(P, G, H, gi, j, ida, Xa, Va, Wa, pa[j], delta, vel, omg, B, clk, pair_out,
                                             pair_count, tally, f, need, o, idj);
#pragma unroll
                for (int k = 0; k < 6; ++k) atomicAdd(&S.acc[6 * il + k], f[k]);
                if (need) store_history<Roll>(H, P.M, gi, atomicAdd(&S.cnt[il], 1), ida, idj, o, clk);
            }
            if (__syncthreads_and(C.done)) break;
            if (t == 0) S.qn = 0;
            __syncthreads();
        }
        if (act) {
            const double4 Vi = vel[i];
            const double4 Wi = omg[i];
            const int idi = (int)Wi.w;
            double f[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) f[k] = S.acc[6 * t + k];
            const int fill = S.cnt[t];
            finish_row<Roll>(H, P.M, i, fill, idi);
            tally.fill = max(tally.fill, fill);
            stokes_terms<Wave>(P, G, Xi, Vi, Wi, f, tally.S);
            store_ft(B.own + 6LL * i, f);
            if (!finite6(f)) atomicOr(&clk->err, kErrNonFinite);
        }
        __syncthreads();
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
// [n_lane, N)), workgroup wb of nwb.  Lanes stride over the (2R+1)^2 stencil rows and queue
// the listed candidates in the wavefront's LDS queue; when it is full or every lane's scan has
// ended, the 64 lanes evaluate the queued pairs (contacts take their history slots from a
// per-wavefront counter), and the scans resume.  The wavefront sums its own side and sorts
// the row.
// ----------------------------------------------------------------------------------
template <typename Real, bool Roll, bool Wave>
__device__ __forceinline__ void sized_wave_path(const DevParams &P, const BoxParams &G, const int *__restrict__ cell_start,
                                                const double4 *__restrict__ pa, const double4 *__restrict__ vel,
                                                const double4 *__restrict__ omg, const ForceBufs &B, const HistView &H,
                                                DevClock *clk, int *pair_out, unsigned long long *pair_count,
                                                double delta, int n_lane, int wb, int nwb, int qcap, WaveShared &S,
                                                PairTally &tally)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int cap = qcap > 0 && qcap < kWaveQ ? qcap : kWaveQ;
    const int nwave = nwb * (kBlock / 64);
    int *const qj = S.qj[wid];
    for (int i = n_lane + wb * (kBlock / 64) + wid; i < P.N; i += nwave) {
        const double4 Xi = pa[i];
        const double4 Vi = vel[i];
        const double4 Wi = omg[i];
        const int idi = (int)Wi.w;
        const int ci = size_class(P, Xi.w);
        const int cx = cell_coord(Xi.x, G.cw[0], G.nc[0]);
        const int cy = cell_coord(Xi.y, G.cw[1], G.nc[1]);
        const int cz = cell_coord(Xi.z, G.cw[2], G.nc[2]);
        if (lane == 0) {
            S.fill[wid] = 0;
            S.qn[wid] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        StencilCursor C;
        cursor_start(G, cell_start, ci, cx, cy, cz, delta, lane, 64, true, C);
        double f[6] = {0, 0, 0, 0, 0, 0};
        for (;;) {
            cursor_scan(P, G, cell_start, pa, i, Xi, ci, cx, cy, cz, delta, 64, C, [&](int j) -> bool {
                const int e = atomicAdd(&S.qn[wid], 1);
                if (e >= cap) return false;
                qj[e] = j;
                return true;
            });
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int nq = min(S.qn[wid], cap);
            for (int e = lane; e < nq; e += 64) {
                const int j = qj[e];
                int need, idj = 0;
                PairOut o;
                sized_pair<Real, Roll, Wave>(P, G, H, i, j, idi, Xi, Vi, Wi, pa[j], delta, vel, omg, B, clk, pair_out,
                                             pair_count, tally, f, need, o, idj);
                if (need) store_history<Roll>(H, P.M, i, atomicAdd(&S.fill[wid], 1), idi, idj, o, clk);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (__all(C.done)) break;
            if (lane == 0) S.qn[wid] = 0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        // the row's entries, written by all lanes, are visible to the whole wavefront
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const int fill = S.fill[wid];
#pragma unroll
        for (int k = 0; k < 6; ++k) f[k] = warp_sum(f[k]);
        wave_finish_row<Roll>(H, P.M, i, fill, idi);
        if (lane == 0) {
            tally.fill = max(tally.fill, fill);
            stokes_terms<Wave>(P, G, Xi, Vi, Wi, f, tally.S);
            store_ft(B.own + 6LL * i, f);
            if (!finite6(f)) atomicOr(&clk->err, kErrNonFinite);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
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
                                                        int g_wave, int qcap, int *__restrict__ pair_out,
                                                        unsigned long long *__restrict__ pair_count)
{
    __shared__ double red[kBlock / 64][12];
    __shared__ SizedShared U;
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
                                          g_wave, qcap, U.w, tally);
    else
        sized_lane_path<Real, Roll, Wave>(P, G, cell_start, pa, vel, omg, B, H, clk, pair_out, pair_count, delta, n_lane,
                                          xcd_row(b - g_wave, (int)gridDim.x - g_wave), (int)gridDim.x - g_wave, qcap,
                                          tally, U.l);
    if constexpr (Sum) reduce_tally(tally, red, partials, P.pstride, b);
}

}  // namespace dss
