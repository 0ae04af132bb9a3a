// On-device observables of Sec. 3 (the quantities behind the paper's figures of the
// rheology and microstructure):
//   - shear-wise diffusivity, eq. (diffY): D_y = <[y(t) - y(t0)]^2> / (2 (t - t0) a0^2 gdot),
//     with y unwrapped across the sheared y faces (the wrap in k_predict counts the crossings
//     of each particle);
//   - autocorrelation of the shear-wise velocity fluctuations, eq. (corrV):
//     C_v = <v'(t) v'(t0)> / <v'(t)^2>, v' = u_y (the ambient shear has no y component);
//   - local volume fraction along y by size group (Fig. localPhi): the volume of every sphere
//     inside each slab [k dy, (k+1) dy) of the periodic y axis, over the slab volume;
//   - clusters of contacting particles (Fig. histo): connected components of the graph of the
//     committed contacts (d_ij < 0), as a histogram of cluster sizes.
#pragma once

#include "dss_kernels.hpp"

namespace dss {

// Reference of the diffusivity and the velocity correlation: unwrapped y and v' by id.
__global__ void __launch_bounds__(kBlock) k_obs_ref(int N, double Ly, const double *__restrict__ x,
                                                     const double *__restrict__ u, const int *__restrict__ img,
                                                     double *__restrict__ y0, double *__restrict__ v0)
{
#pragma clang fp contract(off)
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    y0[id] = x[3 * id + 1] + (double)img[id] * Ly;
    v0[id] = u[3 * id + 1];
}

// Per-workgroup sums of [y_unwrapped(t) - y0]^2, v'(t) v'(t0), v'(t)^2 (3 x gridDim records).
__global__ void __launch_bounds__(kBlock) k_obs_sums(int N, double Ly, const double *__restrict__ x,
                                                      const double *__restrict__ u, const int *__restrict__ img,
                                                      const double *__restrict__ y0, const double *__restrict__ v0,
                                                      double *__restrict__ part)
{
#pragma clang fp contract(off)
    __shared__ double red[kBlock / 64][3];
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    if (id < N) {
        const double dy = (x[3 * id + 1] + (double)img[id] * Ly) - y0[id];
        const double v = u[3 * id + 1];
        s[0] = dy * dy;
        s[1] = v * v0[id];
        s[2] = v * v;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double t = warp_sum(s[k]);
        if (lane == 0) red[wid][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[w][threadIdx.x];
        part[3 * blockIdx.x + threadIdx.x] = t;
    }
}

// Volume of the sphere of radius a centred at 0 between heights z1 < z2 (a slab of the sphere):
// pi [a^2 z - z^3 / 3] over [max(z1, -a), min(z2, a)].
__device__ __forceinline__ double sphere_slab(double a, double z1, double z2)
{
    const double lo = fmax(z1, -a), hi = fmin(z2, a);
    if (!(hi > lo)) return 0.0;
    return kPi * ((a * a * hi - hi * hi * hi / 3.0) - (a * a * lo - lo * lo * lo / 3.0));
}

// Local volume fraction along y: per-workgroup partial profiles (group 0: a <= a_split,
// group 1: a > a_split), nb bins each, accumulated in LDS; part[blockIdx][2 nb].  The
// workgroups stride over the particles (one particle per lane when the grid covers N).
__global__ void __launch_bounds__(kBlock) k_phi_profile(int N, double Ly, int nb, double a_split,
                                                         const double4 *__restrict__ pa, double *__restrict__ part)
{
    extern __shared__ double hist[];  // 2 nb
    for (int k = threadIdx.x; k < 2 * nb; k += kBlock) hist[k] = 0.0;
    __syncthreads();
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const double4 X = pa[p];
        const double dy = Ly / (double)nb;
        const int g = X.w > a_split ? 1 : 0;
        // slabs touched by [y - a, y + a), unwrapped bin indices, periodic in y
        const int b0 = (int)floor((X.y - X.w) / dy), b1 = (int)floor((X.y + X.w) / dy);
        for (int b = b0; b <= b1; ++b) {
            const double v = sphere_slab(X.w, (double)b * dy - X.y, (double)(b + 1) * dy - X.y);
            const int bw = ((b % nb) + nb) % nb;
            atomicAdd(&hist[g * nb + bw], v);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * nb; k += kBlock) part[(long long)blockIdx.x * 2 * nb + k] = hist[k];
}

// Sum of the nw partial profiles of k_phi_profile in workgroup order (the order the host sums
// them in for dss_phi_profile): out[k] = sum_b part[b][k], k < m = 2 nb.
__global__ void __launch_bounds__(kBlock) k_phi_reduce(const double *__restrict__ part, int nw, int m,
                                                        double *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    double t = 0.0;
    for (int b = 0; b < nw; ++b) t += part[(long long)b * m + k];
    out[k] = t;
}

// Connected components of the contact graph by lock-free union-find over particle ids.
// parent[v] <= v at all times (a root is hooked under a smaller root only), so every find
// walks a strictly decreasing chain and ends.  The find splits the path it walks: each
// visited node is pointed at its grandparent, which is still an ancestor no larger than it,
// and only non-roots are written (hooks change roots only, by compare-and-swap), so the
// invariant holds under concurrent finds and hooks while chains stay short.
__device__ __forceinline__ int cc_find(int *parent, int v)
{
    int cur = __atomic_load_n(&parent[v], __ATOMIC_RELAXED);
    if (cur == v) return v;
    int prev = v;
    for (;;) {
        const int next = __atomic_load_n(&parent[cur], __ATOMIC_RELAXED);
        if (next == cur) return cur;
        __atomic_store_n(&parent[prev], next, __ATOMIC_RELAXED);
        prev = cur;
        cur = next;
    }
}

__global__ void __launch_bounds__(kBlock) k_cc_init(int N, int *__restrict__ parent, int *__restrict__ size)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    parent[v] = v;
    size[v] = 0;
}

// Every committed contact (row owner own[p], partner key) joins its two particles.
__global__ void __launch_bounds__(kBlock) k_cc_hook(int N, int M, const int *__restrict__ own,
                                                     const int *__restrict__ key, const int *__restrict__ cnt,
                                                     int *parent)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int a = own[p];
    const int n = cnt[p];
    for (int k = 0; k < n; ++k) {
        const int b = key[(long long)p * M + k] & kKeyMask;
        int ra = cc_find(parent, a), rb = cc_find(parent, b);
        while (ra != rb) {
            const int lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
            if (atomicCAS(&parent[hi], hi, lo) == hi) break;
            ra = cc_find(parent, lo);
            rb = cc_find(parent, hi);
        }
    }
}

// Cluster sizes: size[root] = particles under root.
__global__ void __launch_bounds__(kBlock) k_cc_count(int N, int *parent, int *__restrict__ size)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    atomicAdd(&size[cc_find(parent, v)], 1);
}

// Histogram of cluster sizes: hist[s - 1] += 1 for every root of size s (s > cap counts in
// hist[cap - 1]).
__global__ void __launch_bounds__(kBlock) k_cc_hist(int N, const int *parent, const int *__restrict__ size,
                                                     long long cap, unsigned long long *__restrict__ hist)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    if (parent[v] != v) return;
    const long long s = size[v];
    atomicAdd(&hist[(s < cap ? s : cap) - 1], 1ull);
}

}  // namespace dss
