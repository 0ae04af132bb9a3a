// dss_api.hip -- host side of libdss: handle, device memory, launch sequence, C ABI.
//
// One time step (dss_step) enqueues, on the handle's stream:
//   k_predict  (sorted order of the previous step)  kick/drift, Lees-Edwards wrap, cell id, rank
//   k_scan     exclusive scan of the cell counts -> cell_start, clock advance
//   k_scatter  reorder into the new sorted order, id -> slot map, clear force accumulators
//   k_pairs    half-shell search, pair physics, new history rows, per-workgroup stress partials
//   k_finish   stress and counters from the partials, stress sample (only on steps that take
//              a stress sample and on the last step of a dss_step call)
// The history rows written by k_pairs become the committed history of the step.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dss.h"
#include "dss_kernels.hpp"
#include "dss_adjoint.hpp"
#include "dss_sized.hpp"
#include "dss_observe.hpp"

using namespace dss;

// Device memory of the allocation-free entry point (dss_phi_profile_noalloc): a file-scope
// array, one copy per GPU, held until the process ends.  Host code never passes its name to a
// kernel or a copy (on the host the name is only a stand-in): the address of each device's
// copy is taken once per device, with that device current, when a handle is created there.
constexpr size_t kNoAllocDoubles = size_t(1) << 20;   // 8 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch (device current); 0 on success.
hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(ptr);
    return hipSuccess;
}

double *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Device buffers handed out in a fixed order and kept for the next round of the same
// requests: get() returns the next buffer of the list when it is large enough, else frees it
// and allocates anew; rewind() starts a round, so a repeated sequence of requests allocates
// nothing.
struct DevList {
    std::vector<std::pair<void *, size_t>> bufs;  // (buffer, bytes)
    size_t next = 0;
    DevList() = default;
    DevList(const DevList &) = delete;  // owns its buffers
    DevList &operator=(const DevList &) = delete;
    void rewind() { next = 0; }
    template <class T>
    hipError_t get(T **p, size_t n)
    {
        const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        if (next < bufs.size() && bufs[next].second >= bytes) {
            *p = static_cast<T *>(bufs[next++].first);
            return hipSuccess;
        }
        if (next == bufs.size()) bufs.push_back({nullptr, 0});
        if (bufs[next].first) (void)hipFree(bufs[next].first);
        bufs[next] = {nullptr, 0};
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return e;
        bufs[next++] = {q, bytes};
        *p = static_cast<T *>(q);
        return hipSuccess;
    }
    void release()
    {
        for (auto &b : bufs)
            if (b.first) (void)hipFree(b.first);
        bufs.clear();
        next = 0;
    }
    ~DevList() { release(); }
};

struct AdjointScratch;
}  // namespace

struct dss_handle {
    dss_params prm{};          // parameters of box 0 (the physical constants of every box)
    DevParams P{};
    int nbox = 1;
    std::vector<dss_params> bprm;     // per box (boxes differ only in L and shear_rate)
    std::vector<BoxParams> boxes;     // per box, host copy of the device table
    std::vector<int64_t> box_n;       // particles per box
    std::vector<double> box_sa3;      // sum of a^3 per box
    BoxParams *d_boxes = nullptr;
    int *d_row_box = nullptr;         // cell row -> box
    double *box_diag = nullptr;       // nbox x 3: listed pairs, contacts, largest history row
    int *tile_sum = nullptr;          // totals of the multi-workgroup scan
    int *cs_local = nullptr;          // tile-local cell starts of the parallel scan (up to 16 tiles)
    int ncell_total = 0, nrow_total = 0;
    int scan_tiles = 0;               // 0: one-workgroup scan (scan_c4), else workgroups of 16384 cells
    std::vector<double> box_amax;     // largest radius per box
    double a_min = 0.0;               // smallest radius of all boxes
    std::vector<double> rad_host;     // radii by id (size-class counts of the stencil path)
    int sized_grid[2] = {0, 0};       // lane and wavefront workgroups of k_pairs_sized
    int ec_grid = 0;                  // workgroups of k_pairs_ec (0: no far-pair pass)
    double max_mean_row = 0.0;        // mean particles per cell row of the densest box
    dss_tuning tune{1.0, 1.0, 1, 1, 0, 0, 0, 0};
    bool tune_pending = false;        // lattice to rebuild before the next time step
    // HIP graphs of one time step, keyed by (current buffers, committed history buffers,
    // half-step velocities, stress summation), and of runs of steps (the same key for the
    // first step, the run length and which of its steps sum the stress)
    hipGraphExec_t graph[16] = {};
    std::vector<std::pair<uint64_t, hipGraphExec_t>> run_graphs;
    bool graph_broken = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int n_cu = 256;            // compute units of the device (workgroup slots of k_pairs: 4 per CU)
    std::string err;

    int64_t N = 0;
    bool loaded = false;
    bool vel_is_half = false;  // vel holds the half-step velocity of the last forces
    int cur = 0;               // particle buffers holding the current state
    int hh = 0;                // history buffers holding the committed history
    int64_t step = 0;          // host mirror of the time index

    double4 *pa[2] = {nullptr, nullptr}, *vel[2] = {nullptr, nullptr}, *omg[2] = {nullptr, nullptr};
    double *ft_own = nullptr, *ft_nb = nullptr, *ft_x = nullptr;  // force records (ForceBufs)
    int *cell = nullptr, *rank = nullptr, *count = nullptr, *cell_start = nullptr;
    int *prev = nullptr;       // slot -> slot at the previous sort
    int *img = nullptr;        // y-face crossings by particle id (unwrapped shear-wise position)
    double *obs_y0 = nullptr, *obs_v0 = nullptr;  // observation reference (dss_observe_start)
    int64_t obs_step0 = -1;
    int *hkey[2] = {nullptr, nullptr}, *hcnt[2] = {nullptr, nullptr}, *hown[2] = {nullptr, nullptr};
    double *hxi[2] = {nullptr, nullptr};
    double *hxr[2] = {nullptr, nullptr};  // rolling stretches (only with rolling resistance)
    int *pairs = nullptr;
    unsigned long long *pair_count = nullptr;
    unsigned long long *hist_count = nullptr;  // counter of the history export (second word of pair_count)
    DevClock *clk = nullptr;
    DevRun *run = nullptr;
    double *sigma_last = nullptr;
    double *partials = nullptr;  // 12 doubles per k_pairs workgroup
    double *samples = nullptr;
    int64_t sample_cap_alloc = 0;
    int64_t last_samples = 0;
    int scan_c4 = 1;           // int4 chunks per lane of the cell-count scan
    size_t tile_lds = 0;       // dynamic LDS bytes of a k_pairs workgroup

    ForceBufs fb() const
    {
        ForceBufs b;
        b.own = ft_own;
        b.nb = ft_nb;
        b.x = ft_x;
        b.n = N;
        b.nnb = P.sized ? 0 : 4;
        return b;
    }
    DevRun run_host{};

    // kernel timing with events on the stream
    static constexpr int kKernels = 8;
    unsigned timing = 0;       // bit k: time kernel k
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<int, int>>> ev_marks;  // (kernel, (start event, stop event))
    double kernel_ms[kKernels] = {};
    int64_t kernel_launches[kKernels] = {};
    // the adjoint's device workspace (checkpoints, tape, reverse buffers), kept for the next
    // call of the same shapes; adj_key holds the shapes it was allocated for
    AdjointScratch *adj_ws = nullptr;
    int64_t adj_key[8] = {};
    // while set, k_predict also writes the state it reads (positions, evaluation velocities and
    // spins) by particle id: the adjoint's tape entry of the previous evaluation
    double *tape_x = nullptr, *tape_u = nullptr, *tape_w = nullptr;
    int *tape_zero = nullptr;  // while set, k_predict also clears these N counts
    DevList obs_ws;  // work buffers of the observables, kept between calls
};

namespace {

void release_adjoint_ws(dss_handle *h);

const char *kStatusText[] = {"ok", "invalid argument", "HIP error", "capacity exceeded", "cell lattice too small",
                             "non-finite force or torque", "call out of order"};

dss_status fail(dss_handle *h, dss_status s, const std::string &msg)
{
    if (h) h->err = msg;
    return s;
}

#define HIPTRY(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail(h, DSS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

template <class T>
hipError_t dalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

void destroy_graphs(dss_handle *h)
{
    for (auto &g : h->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (auto &g : h->run_graphs)
        if (g.second) (void)hipGraphExecDestroy(g.second);
    h->run_graphs.clear();
}

void free_lattice(dss_handle *h)
{
    auto F = [](void *p) {
        if (p) (void)hipFree(p);
    };
    destroy_graphs(h);
    F(h->count); F(h->cell_start); F(h->tile_sum); F(h->cs_local); F(h->partials); F(h->d_boxes); F(h->d_row_box);
    h->cs_local = nullptr;
    h->count = h->cell_start = h->tile_sum = h->d_row_box = nullptr;
    h->partials = nullptr;
    h->d_boxes = nullptr;
}

void free_all(dss_handle *h)
{
    auto F = [](void *p) {
        if (p) (void)hipFree(p);
    };
    release_adjoint_ws(h);
    h->obs_ws.release();
    free_lattice(h);
    for (int k = 0; k < 2; ++k) {
        F(h->pa[k]); F(h->vel[k]); F(h->omg[k]);
        F(h->hkey[k]); F(h->hcnt[k]); F(h->hown[k]); F(h->hxi[k]); F(h->hxr[k]);
        h->pa[k] = h->vel[k] = h->omg[k] = nullptr;
        h->hkey[k] = h->hcnt[k] = h->hown[k] = nullptr;
        h->hxi[k] = h->hxr[k] = nullptr;
    }
    F(h->ft_own); F(h->ft_nb); F(h->ft_x); F(h->prev); F(h->img); F(h->obs_y0); F(h->obs_v0);
    h->img = nullptr;
    h->obs_y0 = h->obs_v0 = nullptr;
    h->obs_step0 = -1;
    F(h->cell); F(h->rank);
    F(h->pairs); F(h->pair_count); F(h->clk); F(h->run); F(h->sigma_last); F(h->samples);
    F(h->box_diag);
    h->box_diag = nullptr;
    h->ft_own = h->ft_nb = h->ft_x = nullptr;
    h->prev = nullptr;
    h->cell = h->rank = h->pairs = nullptr;
    h->pair_count = nullptr;
    h->hist_count = nullptr;
    h->clk = nullptr;
    h->run = nullptr;
    h->sigma_last = h->samples = nullptr;
    h->sample_cap_alloc = 0;
    h->loaded = false;
}

// Capacity of the recorded pair list: 32 per particle, plus with the electro-chemical ranges
// the pairs of a uniform gas within the longest cutoff (N_b^2 / V_b x 4/3 pi r_c^3 per box,
// twice the expected count).
long long pair_record_capacity(const DevParams &P, const std::vector<BoxParams> &boxes,
                               const std::vector<double> &box_amax, const int64_t *n_per_box)
{
    double extra = 0.0, N = 0.0;
    for (size_t b = 0; b < boxes.size(); ++b) {
        N += (double)n_per_box[b];
        if (P.ec && P.rext > 0.0) {
            const double rc = 2.0 * box_amax[b] + P.rext;
            const double V = boxes[b].L[0] * boxes[b].L[1] * boxes[b].L[2];
            extra += (double)n_per_box[b] * (double)n_per_box[b] / V * (4.0 / 3.0) * kPi * rc * rc * rc;
        }
    }
    const double cap = 32.0 * N + 64.0 + std::min(extra, 0.5 * N * N);
    return (long long)std::min(cap, 2.0e9);
}

// Row capacity of the reduced history matrix: the shell of thickness 2 a_min around the
// largest particle, in units of the smallest particle's volume (Sec. 2.1).
int paper_capacity(double a_max, double a_min)
{
    double outer = a_max + 2.0 * a_min;
    double shell = outer * outer * outer - a_max * a_max * a_max;
    return (int)std::ceil(shell / (a_min * a_min * a_min));
}

// Per-box counters of the last summed evaluation (nbox x 3).
dss_status read_diag(dss_handle *h, std::vector<double> &d)
{
    d.assign(3 * (size_t)h->nbox, 0.0);
    HIPTRY(hipMemcpyAsync(d.data(), h->box_diag, d.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    return DSS_OK;
}

dss_status check_flags(dss_handle *h)
{
    DevClock c;
    HIPTRY(hipMemcpyAsync(&c, h->clk, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    if (c.err & kErrNonFinite) return fail(h, DSS_ERR_UNSTABLE, "non-finite force or torque");
    if (c.err & kErrRowOverflow) {
        std::vector<double> d;
        dss_status s = read_diag(h, d);
        if (s) return s;
        double mf = 0.0;
        for (int b = 0; b < h->nbox; ++b) mf = std::max(mf, d[3 * b + 2]);
        return fail(h, DSS_ERR_CAPACITY, "contact-history row overflow (max fill " + std::to_string((int)mf) +
                                             ", capacity " + std::to_string(h->P.M) + ")");
    }
    return DSS_OK;
}

// Start / stop events of one timed launch (events are reused across calls).  The kernel is
// launched with hipExtLaunchKernelGGL, which records them at the kernel's own start and end,
// so the measured time is the kernel's execution without the launch gaps.
struct TimedLaunch {
    dss_handle *h;
    int kernel;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int i0 = -1, i1 = -1;
    TimedLaunch(dss_handle *h_, int k) : h(h_), kernel(k)
    {
        if (!(h->timing & (1u << k))) return;
        i0 = take(0);
        i1 = take(1);
        if (i0 < 0 || i1 < 0) {
            i0 = i1 = -1;
            return;
        }
        e0 = h->ev_pool[i0];
        e1 = h->ev_pool[i1];
    }
    ~TimedLaunch()
    {
        if (i0 >= 0) h->ev_marks.push_back({kernel, {i0, i1}});
    }
    int take(int off)
    {
        const size_t used = 2 * h->ev_marks.size() + off;
        while (used >= h->ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            h->ev_pool.push_back(e);
        }
        return (int)used;
    }
};

dss_status collect_timing(dss_handle *h)
{
    if (h->ev_marks.empty()) return DSS_OK;
    HIPTRY(hipStreamSynchronize(h->stream));
    for (auto &m : h->ev_marks) {
        float ms = 0.f;
        HIPTRY(hipEventElapsedTime(&ms, h->ev_pool[m.second.first], h->ev_pool[m.second.second]));
        h->kernel_ms[m.first] += ms;
        h->kernel_launches[m.first] += 1;
    }
    h->ev_marks.clear();
    return DSS_OK;
}

dss_status require_loaded(dss_handle *h)
{
    if (!h) return DSS_ERR_ARG;
    if (!h->loaded) return fail(h, DSS_ERR_STATE, "no particles loaded (call dss_set_particles first)");
    return DSS_OK;
}

// Size classes of the stencil path: class of radius a = floor(a cls_mul + cls_add), ncls
// classes (cls_add = 0 without the electro-chemical ranges).
struct SizeClasses {
    int ncls = 1;
    double cls_mul = 0.0, cls_add = 0.0;
    int ec_ry = 0, ec_rz = 0;   // > 0: electro-chemical far pairs on their own pass (k_pairs_ec)
};

// Cell lattice of every box: spacing >= cell_scale times the box's largest pair cutoff
// 2 c a_max (with a 1e-9 margin), boxes numbered one after the other.  Returns false (and
// why) when a box has fewer than 4 x 3 x 3 cells or more than 4096 cell rows.
// Size-class stencils (one box): spacing >= cell_scale times the reach of the smallest
// particle (2 c a_min, or 2 max(c, 1) a_min + rext with the electro-chemical ranges), coarsened until the largest stencil (R_max = ncls cells) fits the box without
// reaching a cell twice: n_x >= 2 R_max + 2 (the window of a sheared row), n_y, n_z >=
// 2 R_max + 1.  Cells are numbered class-major: ncls x n_x n_y n_z sort keys.
// Electro-chemical ranges on one box without size classes: the lattice of the lubrication
// list when the far-pair pass fits it (sc.ec_ry, sc.ec_rz > 0), else that of the whole set.
bool lattice_of(std::vector<BoxParams> &boxes, const std::vector<double> &amax, double amin, double cf,
                double rext, double cell_scale, bool sized, int row_slots, SizeClasses &sc, std::string &why)
{
    sc = SizeClasses{};
    if (sized) {
        if (boxes.size() != 1) {
            why = "size-class stencils need a handle of one box";
            return false;
        }
        // reach of a particle of radius a: every partner of radius <= a lies within it.  The
        // lubrication cutoff c (a_i + a_j) gives 2 c a; with the electro-chemical ranges the
        // cutoff max(c (a_i + a_j), a_i + a_j + rext) is bounded by 2 max(c, 1) a + rext.
        const double cm = rext > 0.0 ? 2.0 * std::max(cf, 1.0) : 2.0 * cf;
        const double ca = rext > 0.0 ? rext : 0.0;
        BoxParams &G = boxes[0];
        const double rc = (cm * amin + ca) * (1.0 + 1e-9) * cell_scale;
        int n[3];
        for (int d = 0; d < 3; ++d) n[d] = std::max(1, (int)std::floor(G.L[d] / rc));
        for (;;) {
            if (n[0] < 4 || n[1] < 3 || n[2] < 3) {
                why = "box too small for size-class stencils (largest stencil does not fit)";
                return false;
            }
            const double cwmin = std::min(G.L[0] / n[0], std::min(G.L[1] / n[1], G.L[2] / n[2]));
            sc.cls_mul = cm * (1.0 + 1e-9) / cwmin;
            sc.cls_add = ca * (1.0 + 1e-9) / cwmin;
            sc.ncls = (int)std::floor(amax[0] * sc.cls_mul + sc.cls_add) + 1;
            if (n[0] >= 2 * sc.ncls + 2 && n[1] >= 2 * sc.ncls + 1 && n[2] >= 2 * sc.ncls + 1) break;
            for (int d = 0; d < 3; ++d) n[d] -= std::max(1, n[d] / 16);
        }
        for (int d = 0; d < 3; ++d) {
            G.nc[d] = n[d];
            G.cw[d] = G.L[d] / (double)n[d];
        }
        G.cell_off = 0;
        G.row_off = 0;
        G.nrec = 1;
        if ((int64_t)sc.ncls * n[0] * n[1] * n[2] > (int64_t)0x3fffffff) {
            why = "too many cells";
            return false;
        }
        return true;
    }
    // Electro-chemical ranges on one box: first the lattice of the lubrication list alone, the
    // pairs beyond it on the far-pair pass, whose reach of R_y, R_z cell rows must stay below
    // half the box (2 R + 1 distinct rows, and a box length beyond twice the reach along x);
    // else the lattice of the whole pair set.
    const bool try_split = rext > 0.0 && cf >= 1.0 && boxes.size() == 1;
    if (try_split) {
        std::vector<BoxParams> trial = boxes;
        if (lattice_of(trial, amax, amin, cf, 0.0, cell_scale, false, row_slots, sc, why)) {
            const BoxParams &G = trial[0];
            const double reach = (2.0 * amax[0] + rext) * (1.0 + 1e-9);
            const int ry = (int)std::ceil(reach / G.cw[1]), rz = (int)std::ceil(reach / G.cw[2]);
            if (G.nc[1] >= 2 * ry + 1 && G.nc[2] >= 2 * rz + 1 && G.L[0] >= 2.0 * reach + G.cw[0]) {
                boxes = trial;
                sc.ec_ry = ry;
                sc.ec_rz = rz;
                return true;
            }
        }
        sc = SizeClasses{};
    }
    int64_t ncell = 0;
    int nrow = 0;
    for (size_t b = 0; b < boxes.size(); ++b) {
        BoxParams &G = boxes[b];
        // largest pair cutoff of the box: c 2 a_max, or with the electro-chemical ranges
        // max(c 2 a_max, 2 a_max + rext)
        const double cut = rext > 0.0 ? std::max(cf * 2.0 * amax[b], 2.0 * amax[b] + rext) : cf * 2.0 * amax[b];
        const double rc = cut * (1.0 + 1e-9) * cell_scale;
        for (int d = 0; d < 3; ++d) G.nc[d] = std::max(1, (int)std::floor(G.L[d] / rc));
        // one box whose cell rows exceed the k_pairs workgroup slots by a little: coarser cells
        // along z (the vorticity direction, away from the sheared faces) until every row has a
        // slot, so the rows run in one round instead of a nearly empty second one.  The rows
        // are kept 1/64 below the slots: with every slot taken, a few workgroups have been seen
        // to wait for a slot of a finished row at launch
        if (boxes.size() == 1 && row_slots > 0) {
            const int rows = G.nc[1] * G.nc[2];
            const int fit = row_slots - row_slots / 64;
            if (rows > fit && rows * 100 <= row_slots * 115)
                while (G.nc[1] * G.nc[2] > fit && G.nc[2] > 3) --G.nc[2];
        }
        for (int d = 0; d < 3; ++d) G.cw[d] = G.L[d] / (double)G.nc[d];
        if (G.nc[0] < 4 || G.nc[1] < 3 || G.nc[2] < 3) {
            why = "cell lattice " + std::to_string(G.nc[0]) + "x" + std::to_string(G.nc[1]) + "x" +
                  std::to_string(G.nc[2]) + " of box " + std::to_string(b) + " is smaller than 4x3x3";
            return false;
        }
        const int rows = G.nc[1] * G.nc[2];
        if (rows > 4096) {
            why = "more than 4096 cell rows in box " + std::to_string(b);
            return false;
        }
        G.cell_off = (int)ncell;
        G.row_off = nrow;
        G.nrec = rows;
        ncell += (int64_t)G.nc[0] * rows;
        nrow += rows;
        if (ncell > (int64_t)0x3fffffff) {
            why = "too many cells";
            return false;
        }
    }
    return true;
}

// (Re)build everything that depends on the cell lattice: the box table, the cell-row ->
// box map, cell counts and starts, the scan layout, the per-row stress partials and the
// row-tile capacities of k_pairs.  The particles keep their slots; the next counting sort
// uses the new lattice.
dss_status setup_lattice(dss_handle *h)
{
    std::string why;
    SizeClasses sc;
    const bool sized = h->tune.sized != 0;
    if (!lattice_of(h->boxes, h->box_amax, h->a_min, h->prm.cutoff_factor, h->P.ec ? h->P.rext : 0.0,
                    h->tune.cell_scale, sized, h->tune.tiled ? 4 * h->n_cu : 0, sc, why))
        return fail(h, DSS_ERR_BOX, why);
    free_lattice(h);
    const int B = h->nbox;
    int64_t ncell = 0;
    int nrow = 0, max_rows_box = 0;
    double max_mean_row = 0.0;
    std::vector<int> row_box;
    for (int b = 0; b < B; ++b) {
        const BoxParams &G = h->boxes[b];
        const int rows = G.nc[1] * G.nc[2];
        row_box.insert(row_box.end(), rows, b);
        ncell += (int64_t)G.nc[0] * rows;
        nrow += rows;
        max_rows_box = std::max(max_rows_box, rows);
        max_mean_row = std::max(max_mean_row, (double)G.n_part / (double)rows);
    }
    {
        // size-class stencils: class-major sort keys, one lane per particle below wave_cls
        // (stencil radius 4 and up by default), one wavefront per particle above; the stress
        // partial records are the workgroups of the two kernels
        DevParams &P = h->P;
        P.sized = sized ? 1 : 0;
        P.ncls = sc.ncls;
        P.cls_mul = sc.cls_mul;
        P.cls_add = sc.cls_add;
        P.wave_cls = h->tune.wave_class > 0 ? h->tune.wave_class : 3;
        h->sized_grid[0] = h->sized_grid[1] = 0;
        // electro-chemical far pairs: one k_pairs_ec workgroup per kBlock / kEcLanes particles,
        // whose stress partials follow the cell rows' records of the box
        P.ec_split = sc.ec_ry > 0 ? 1 : 0;
        P.ec_ry = sc.ec_ry;
        P.ec_rz = sc.ec_rz;
        P.ec_amax = h->box_amax[0];
        h->ec_grid = 0;
        if (P.ec_split) {
            h->ec_grid = (int)((h->N * kEcLanes + kBlock - 1) / kBlock);
            h->boxes[0].nrec += h->ec_grid;
            max_rows_box = h->boxes[0].nrec;
        }
        if (sized) {
            ncell *= sc.ncls;
            int64_t n_big = 0;
            for (double a : h->rad_host)
                n_big += std::min((int)std::floor(a * sc.cls_mul + sc.cls_add), sc.ncls - 1) >= P.wave_cls ? 1 : 0;
            const int64_t n_lane = h->N - n_big;
            // wavefront workgroups in multiples of 8 (one per XCD), launched first
            const int g_wave =
                P.wave_cls < sc.ncls ? (int)std::min<int64_t>((std::max<int64_t>((n_big + 3) / 4, 1) + 7) / 8 * 8, 1024)
                                     : 0;
            const int g_lane = (int)std::min<int64_t>(std::max<int64_t>((n_lane + kBlock - 1) / kBlock, 1), 4096 - g_wave);
            h->sized_grid[0] = g_lane;
            h->sized_grid[1] = g_wave;
            h->boxes[0].nrec = g_lane + g_wave;
            max_rows_box = g_lane + g_wave;
        }
    }
    // cell-count scan: one workgroup up to 65535 cells, else workgroups of 16384 cells
    int64_t ncell_pad;
    if (ncell + 1 <= 4096 * 16) {
        h->scan_c4 = (int)((ncell + 1 + 4095) / 4096);
        h->scan_tiles = 0;
        ncell_pad = 4096 * (int64_t)h->scan_c4;
    } else {
        h->scan_c4 = 0;
        h->scan_tiles = (int)((ncell + 1 + 16383) / 16384);
        ncell_pad = 16384 * (int64_t)h->scan_tiles;
    }
    h->ncell_total = (int)ncell;
    h->nrow_total = nrow;
    h->max_mean_row = max_mean_row;
    // row-tile capacities of k_pairs from the mean occupancy of a cell row (own row and the
    // five rows of the half shell) of the densest box, times tile_scale; rows beyond them
    // take the per-particle path, which every row takes when tiling is off.  When capacities
    // with a margin of two standard deviations over the mean row occupancy fit four
    // workgroups per CU (40 KB of LDS each), they are taken: every cell row then has a slot
    // of its own on a box of up to 4 x n_CU rows.
    DevParams &P = h->P;
    {
        const double mean_row = max_mean_row * h->tune.tile_scale;
        auto up = [](double v, int m) { return ((int)std::ceil(v) + m - 1) / m * m; };
        int own_cap = up(1.5 * mean_row + 16.0, 32);
        int stage_cap = up(6.25 * mean_row + 32.0, 64);
        int qcap = up(8.0 * mean_row + 64.0, 64);
        // (dynamic and static LDS are each allocated in blocks of up to 1 KB)
        const size_t lds_four = 40 * 1024 - 1024;
        const int own4 = up(1.3 * mean_row + 8.0, 32);
        const int stage4 = up(5.0 * mean_row + 2.0 * std::sqrt(5.0 * mean_row), 16);
        const int q4 = up(4.5 * mean_row + 64.0, 64);
        if (tile_lds_bytes(own4, stage4, q4) <= lds_four) {
            own_cap = own4;
            stage_cap = stage4;
            qcap = q4;
        }
        const size_t lds_max = 150 * 1024;
        while (tile_lds_bytes(own_cap, stage_cap, qcap) > lds_max && own_cap > 32) {
            own_cap = std::max(32, own_cap * 3 / 4 / 32 * 32);
            stage_cap = std::max(64, stage_cap * 3 / 4 / 64 * 64);
            qcap = std::max(64, qcap * 3 / 4 / 64 * 64);
        }
        own_cap = std::min(own_cap, 4096);
        stage_cap = std::min(stage_cap, 16384 - 64);  // staged indices are 14-bit
        if (!h->tune.tiled) {
            own_cap = 32;
            stage_cap = 64;
            qcap = 64;
        }
        h->tile_lds = tile_lds_bytes(own_cap, stage_cap, qcap);
        P.own_cap = own_cap;
        P.tiled = h->tune.tiled ? 1 : 0;
        P.stage_cap = stage_cap;
        P.qcap = qcap;
        // margin on r^2 of the FP32 candidate pre-test: FP32 coordinates and image shifts of
        // magnitude up to 6 L round the components of r by at most 29, 10, 10 u L (u = 2^-24),
        // so r^2 near the cutoff r_c moves by at most 2 r_c 49 u L, and the FP32 cutoff r_c^2
        // by 6 u r_c^2; twice that bound over the largest box and cutoff
        double lmax = 0.0, rcmax = 0.0;
        for (int b = 0; b < B; ++b) {
            const BoxParams &G = h->boxes[b];
            lmax = std::max(lmax, std::max(G.L[0], std::max(G.L[1], G.L[2])));
            const double a2 = 2.0 * h->box_amax[b];
            rcmax = std::max(rcmax, (P.ec && !P.ec_split) ? std::max(h->prm.cutoff_factor * a2, a2 + P.rext)
                                                          : h->prm.cutoff_factor * a2);
        }
        const double u = std::ldexp(1.0, -24);
        P.pf_m2 = (float)(2.0 * (2.0 * rcmax * 49.0 * u * lmax + 6.0 * u * rcmax * rcmax));
    }
    for (const void *k :
         {(const void *)k_pairs<double, false, false, true>, (const void *)k_pairs<float, false, false, true>,
          (const void *)k_pairs<double, true, false, true>, (const void *)k_pairs<float, true, false, true>,
          (const void *)k_pairs<double, false, true, true>, (const void *)k_pairs<float, false, true, true>,
          (const void *)k_pairs<double, true, true, true>, (const void *)k_pairs<float, true, true, true>,
          (const void *)k_pairs<double, false, false, false>, (const void *)k_pairs<float, false, false, false>,
          (const void *)k_pairs<double, true, false, false>, (const void *)k_pairs<float, true, false, false>,
          (const void *)k_pairs<double, false, true, false>, (const void *)k_pairs<float, false, true, false>,
          (const void *)k_pairs<double, true, true, false>, (const void *)k_pairs<float, true, true, false>})
        HIPTRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->tile_lds));
    P.pstride = (std::max(nrow, max_rows_box) + 63) / 64 * 64;
    HIPTRY(dalloc(&h->count, ncell_pad));
    HIPTRY(dalloc(&h->cell_start, ncell_pad));
    HIPTRY(dalloc(&h->tile_sum, std::max(h->scan_tiles, 16)));
    HIPTRY(dalloc(&h->cs_local, ncell_pad));
    HIPTRY(dalloc(&h->partials, 12 * (size_t)P.pstride));
    HIPTRY(dalloc(&h->d_boxes, B));
    HIPTRY(dalloc(&h->d_row_box, nrow));
    HIPTRY(hipMemcpyAsync(h->d_boxes, h->boxes.data(), B * sizeof(BoxParams), hipMemcpyHostToDevice, h->stream));
    HIPTRY(hipMemcpyAsync(h->d_row_box, row_box.data(), nrow * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPTRY(hipMemsetAsync(h->partials, 0, 12 * (size_t)P.pstride * sizeof(double), h->stream));
    HIPTRY(hipMemsetAsync(h->count, 0, ncell_pad * sizeof(int), h->stream));
    return DSS_OK;
}

// One force evaluation.
//   EVAL_STEP:    a full time step: drift + kick, counting sort, pairs; history committed.
//   EVAL_SORT:    counting sort of the current positions, then pairs (initial evaluation).
//   EVAL_INPLACE: pairs at the current state and order (velocities completed to u^n).
//   EVAL_RESORT:  counting sort of the current positions (velocities completed to u^n), the
//                 committed history moved to the new slots, then pairs; no time advance.
enum EvalMode { EVAL_STEP = 0, EVAL_SORT = 1, EVAL_INPLACE = 2, EVAL_RESORT = 3 };

// The pair kernels of one evaluation: size-class stencils (lane and wavefront paths), or
// the row tiles (a row beyond their capacities on the per-particle path, by its own
// workgroup), after the electro-chemical far pairs when they have a pass of their own.
// Real: FP64 or mixed arithmetic; Roll: rolling resistance; Wave: the wavy ambient shear;
// Sum: the stress and counters are summed (k_finish follows), else the tile and stencil
// kernels skip them.
template <typename Real, bool Roll, bool Wave, bool Sum>
void launch_pair_kernels(dss_handle *h, int buf, const HistView &H)
{
    if (h->P.sized) {
        TimedLaunch t(h, 3);
        hipExtLaunchKernelGGL(k_pairs_sized<Real, Roll, Wave, Sum>, dim3(h->sized_grid[0] + h->sized_grid[1]), dim3(kBlock), 0,
                              h->stream, t.e0, t.e1, 0, h->P, h->d_boxes, h->cell_start, h->pa[buf], h->vel[buf],
                              h->omg[buf], h->fb(), H, h->clk, h->partials, h->sized_grid[1], h->tune.queue_cap,
                              h->pairs, h->pair_count);
        return;
    }
    if (h->P.ec_split) {
        // the far electro-chemical pairs first: plain stores into the atomic record, which the
        // deferred rows below add to
        TimedLaunch t(h, 7);
        const BoxParams &G = h->boxes[0];
        hipExtLaunchKernelGGL(k_pairs_ec<Sum>, dim3(h->ec_grid), dim3(kBlock), 0, h->stream, t.e0, t.e1, 0, h->P,
                              h->d_boxes, h->cell_start, h->pa[buf], h->omg[buf], h->ft_x, h->clk, h->partials,
                              G.row_off + G.nc[1] * G.nc[2], h->pairs, h->pair_count);
    }
    {
        TimedLaunch t(h, 3);
        RowArgs R;
        R.P = h->P;
        R.B = h->fb();
        R.H = H;
        R.boxes = h->d_boxes;
        R.row_box = h->d_row_box;
        R.cell_start = h->cell_start;
        R.pa = h->pa[buf];
        R.vel = h->vel[buf];
        R.omg = h->omg[buf];
        R.clk = h->clk;
        R.partials = h->partials;
        R.pair_out = h->pairs;
        R.pair_count = h->pair_count;
        hipExtLaunchKernelGGL(k_pairs<Real, Roll, Wave, Sum>, dim3(h->nrow_total), dim3(kPairBlock), h->tile_lds, h->stream, t.e0,
                              t.e1, 0, h->P, h->d_boxes, h->d_row_box, h->cell_start, h->pa[buf], h->vel[buf],
                              h->omg[buf], h->fb(), H, h->clk, h->partials, h->pairs, h->pair_count, R);
    }
}

dss_status launch_pairs(dss_handle *h, int buf, const int *prev, int sample, bool finish)
{
    HistView H;
    H.key_old = h->hkey[h->hh];
    H.xi_old = h->hxi[h->hh];
    H.cnt_old = h->hcnt[h->hh];
    H.prev = prev;
    H.key_new = h->hkey[1 - h->hh];
    H.xi_new = h->hxi[1 - h->hh];
    H.cnt_new = h->hcnt[1 - h->hh];
    H.own_new = h->hown[1 - h->hh];
    H.xr_old = h->hxr[h->hh];
    H.xr_new = h->hxr[1 - h->hh];
    const bool roll = h->P.kr > 0.0, wave = h->P.wave_amp != 0.0;
    const int v = (finish ? 8 : 0) | (h->prm.precision == DSS_MIXED ? 4 : 0) | (roll ? 2 : 0) | (wave ? 1 : 0);
    switch (v) {
    case 0: launch_pair_kernels<double, false, false, false>(h, buf, H); break;
    case 1: launch_pair_kernels<double, false, true, false>(h, buf, H); break;
    case 2: launch_pair_kernels<double, true, false, false>(h, buf, H); break;
    case 3: launch_pair_kernels<double, true, true, false>(h, buf, H); break;
    case 4: launch_pair_kernels<float, false, false, false>(h, buf, H); break;
    case 5: launch_pair_kernels<float, false, true, false>(h, buf, H); break;
    case 6: launch_pair_kernels<float, true, false, false>(h, buf, H); break;
    case 7: launch_pair_kernels<float, true, true, false>(h, buf, H); break;
    case 8: launch_pair_kernels<double, false, false, true>(h, buf, H); break;
    case 9: launch_pair_kernels<double, false, true, true>(h, buf, H); break;
    case 10: launch_pair_kernels<double, true, false, true>(h, buf, H); break;
    case 11: launch_pair_kernels<double, true, true, true>(h, buf, H); break;
    case 12: launch_pair_kernels<float, false, false, true>(h, buf, H); break;
    case 13: launch_pair_kernels<float, false, true, true>(h, buf, H); break;
    case 14: launch_pair_kernels<float, true, false, true>(h, buf, H); break;
    default: launch_pair_kernels<float, true, true, true>(h, buf, H); break;
    }
    if (!finish) return DSS_OK;
    TimedLaunch t(h, 4);
    hipExtLaunchKernelGGL(k_finish, dim3(12 * h->nbox), dim3(kBlock), 0, h->stream, t.e0, t.e1, 0, h->d_boxes,
                          h->partials, h->P.pstride, h->clk, h->run, sample);
    return DSS_OK;
}

// Host bookkeeping after an evaluation: the particles now live in the other buffers; a
// time step commits the new history rows and advances the clock.
void commit_eval(dss_handle *h, bool advance)
{
    h->cur = 1 - h->cur;
    h->vel_is_half = advance;
    if (advance) {
        h->hh = 1 - h->hh;
        h->step += 1;
    }
}

dss_status evaluate(dss_handle *h, EvalMode mode, bool finish = true)
{
    const int N = (int)h->N;
    const int grid = (N + kBlock - 1) / kBlock;
    const int c = h->cur, o = 1 - h->cur;
    const int advance = mode == EVAL_STEP ? 1 : 0;
    if (mode == EVAL_INPLACE) {
        if (h->vel_is_half) {
            TimedLaunch t(h, 0);
            hipExtLaunchKernelGGL(k_complete, dim3(grid), dim3(kBlock), 0, h->stream, t.e0, t.e1, 0, h->P, h->pa[c],
                                  h->vel[c], h->omg[c], h->fb());
        }
        HIPTRY(hipMemsetAsync(h->ft_x, 0, 6 * h->N * sizeof(double), h->stream));
        if (h->P.record_pairs) HIPTRY(hipMemsetAsync(h->pair_count, 0, sizeof(unsigned long long), h->stream));
        dss_status s = launch_pairs(h, c, nullptr, 0, true);
        if (s) return s;
        HIPTRY(hipGetLastError());
        h->vel_is_half = false;
        return DSS_OK;
    }
    {
        TimedLaunch t(h, 0);
        hipExtLaunchKernelGGL(k_predict, dim3(grid), dim3(kBlock), 0, h->stream, t.e0, t.e1, 0, h->P, h->d_boxes,
                              h->pa[c], h->vel[c], h->omg[c], h->fb(), h->vel_is_half ? 1 : 0, advance, h->clk,
                              h->cell, h->rank, h->count, h->img, h->boxes[0],
                              h->P.record_pairs ? h->pair_count : (unsigned long long *)nullptr, h->tape_x,
                              h->tape_u, h->tape_w, h->tape_zero);
    }
    if (h->scan_tiles > 0) {
        TimedLaunch t(h, 1);
        hipExtLaunchKernelGGL(k_scan<4>, dim3(h->scan_tiles), dim3(1024), 0, h->stream, t.e0, (hipEvent_t) nullptr,
                              0, h->count, h->cell_start, h->clk, advance, h->tile_sum);
        hipExtLaunchKernelGGL(k_scan_add, dim3(h->scan_tiles), dim3(1024), 0, h->stream, (hipEvent_t) nullptr, t.e1,
                              0, h->cell_start, h->tile_sum, 4 * 1024, h->clk, advance);
    } else {
        // one workgroup per tile of 4096 cells, in parallel; k_scatter adds the tile offsets
        TimedLaunch t(h, 1);
        if (h->scan_c4 < 1 || h->scan_c4 > 16) return fail(h, DSS_ERR_BOX, "cell lattice too large for the scan");
        hipExtLaunchKernelGGL(k_scan<1>, dim3(h->scan_c4), dim3(1024), 0, h->stream, t.e0, t.e1, 0, h->count,
                              h->cs_local, h->clk, advance, h->tile_sum);
    }
    {
        TimedLaunch t(h, 2);
        const bool tiles = h->scan_tiles == 0;
        hipExtLaunchKernelGGL(k_scatter, dim3(grid), dim3(kBlock), 0, h->stream, t.e0, t.e1, 0, N, h->cell, h->rank,
                              tiles ? h->cs_local : h->cell_start, h->tile_sum, tiles ? h->scan_c4 : 0,
                              h->ncell_total + 1, h->cell_start, h->clk, advance, h->pa[c], h->vel[c], h->omg[c],
                              h->pa[o], h->vel[o], h->omg[o], h->prev);
    }
    if (mode == EVAL_RESORT) {
        // the committed rows follow their particles; the pair kernels then find them in place
        const int hn = 1 - h->hh;
        hipLaunchKernelGGL(k_history_move, dim3(grid), dim3(kBlock), 0, h->stream, N, h->P.M, h->prev,
                           h->hkey[h->hh], h->hxi[h->hh], h->hxr[h->hh], h->hcnt[h->hh], h->hown[h->hh], h->hkey[hn],
                           h->hxi[hn], h->hxr[hn], h->hcnt[hn], h->hown[hn]);
        HIPTRY(hipGetLastError());
        h->hh = hn;
    }
    dss_status s = launch_pairs(h, o, mode == EVAL_RESORT ? nullptr : h->prev, advance, finish);
    if (s) return s;
    HIPTRY(hipGetLastError());
    commit_eval(h, advance != 0);
    return DSS_OK;
}

// One time step through a HIP graph: captured on first use of its key, replayed after.
// Graphs are used only without kernel timing and pair recording (the pair counter reset is
// a memset, which is not recorded into graphs).
dss_status graph_step(dss_handle *h, bool finish)
{
    const int key = h->cur | (h->hh << 1) | ((h->vel_is_half ? 1 : 0) << 2) | ((finish ? 1 : 0) << 3);
    if (!h->graph[key]) {
        hipGraph_t g = nullptr;
        const int cur = h->cur, hh = h->hh;
        const bool vih = h->vel_is_half;
        const int64_t step = h->step;
        HIPTRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        dss_status s = evaluate(h, EVAL_STEP, finish);
        hipError_t e = hipStreamEndCapture(h->stream, &g);
        // the capture recorded the launches without running them
        h->cur = cur;
        h->hh = hh;
        h->vel_is_half = vih;
        h->step = step;
        if (s) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return fail(h, DSS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&h->graph[key], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            h->graph[key] = nullptr;
            return fail(h, DSS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
    }
    HIPTRY(hipGraphLaunch(h->graph[key], h->stream));
    commit_eval(h, true);
    return DSS_OK;
}

// n consecutive time steps (n <= kRunSteps) through one HIP graph: bit k of `finish` sums the
// stress at step k.  One launch for the run, so the steps follow each other without the gap
// that separates two graph launches on the device.  run_graph finds or captures the graph of
// the run from the current buffers (capturing records the launches without running them, and
// leaves the handle's state as it was); graph_run launches it and advances the state.
constexpr int kRunSteps = 16;
constexpr size_t kMaxRunGraphs = 64;  // graphs of runs kept per handle
dss_status run_graph(dss_handle *h, int n, unsigned finish, hipGraphExec_t *out)
{
    const uint64_t key = (uint64_t)h->cur | ((uint64_t)h->hh << 1) | ((uint64_t)(h->vel_is_half ? 1 : 0) << 2) |
                         ((uint64_t)n << 3) | ((uint64_t)finish << 8);
    for (auto &g : h->run_graphs)
        if (g.first == key) {
            *out = g.second;
            return DSS_OK;
        }
    if (h->run_graphs.size() >= kMaxRunGraphs) {
        // calls of many different shapes: start the collection afresh
        for (auto &r : h->run_graphs)
            if (r.second) (void)hipGraphExecDestroy(r.second);
        h->run_graphs.clear();
    }
    const int cur = h->cur, hh = h->hh;
    const bool vih = h->vel_is_half;
    const int64_t step = h->step;
    hipGraph_t g = nullptr;
    HIPTRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    dss_status s = DSS_OK;
    for (int k = 0; k < n && !s; ++k) s = evaluate(h, EVAL_STEP, (finish >> k) & 1u);
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    h->cur = cur;
    h->hh = hh;
    h->vel_is_half = vih;
    h->step = step;
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return fail(h, DSS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(h, DSS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    h->run_graphs.push_back({key, ge});
    // its first launch should not pay for setting it up on the device
    HIPTRY(hipGraphUpload(ge, h->stream));
    *out = ge;
    return DSS_OK;
}

dss_status graph_run(dss_handle *h, int n, unsigned finish)
{
    hipGraphExec_t ge = nullptr;
    dss_status s = run_graph(h, n, finish, &ge);
    if (s) return s;
    HIPTRY(hipGraphLaunch(ge, h->stream));
    for (int k = 0; k < n; ++k) commit_eval(h, true);
    return DSS_OK;
}

// The runs of a dss_step call of n_steps steps sampling every stress_every: a run of steps
// starting at index k of the call (its length, and which of its steps sum the stress), or a
// single step when fewer than two remain.
struct StepRuns {
    int64_t n_steps, stress_every, step0, run;
    StepRuns(int64_t n, int64_t se, int64_t s0)
        : n_steps(n), stress_every(se), step0(s0), run(se >= 2 && se <= kRunSteps ? se : kRunSteps / 2) {}
    bool finish_at(int64_t k) const  // k: the step's index within the call
    {
        return k == n_steps - 1 || (stress_every > 0 && (step0 + k + 1) % stress_every == 0);
    }
    int length_at(int64_t k) const { return n_steps - k >= 2 ? (int)std::min<int64_t>(run, n_steps - k) : 1; }
    unsigned mask_at(int64_t k, int n) const
    {
        unsigned mask = 0;
        for (int j = 0; j < n; ++j) mask |= (finish_at(k + j) ? 1u : 0u) << j;
        return mask;
    }
};

}  // namespace

extern "C" {

const char *dss_status_string(dss_status s)
{
    int k = (int)s;
    if (k < 0 || k > 6) return "unknown status";
    return kStatusText[k];
}

const char *dss_last_error(const dss_handle *h) { return h ? h->err.c_str() : "null handle"; }

dss_status dss_set_timing(dss_handle *h, int enable)
{
    if (!h) return DSS_ERR_ARG;
    dss_status s = collect_timing(h);
    if (s) return s;
    h->timing = enable < 0 ? 0xffffffffu : (unsigned)enable;
    for (int k = 0; k < dss_handle::kKernels; ++k) {
        h->kernel_ms[k] = 0.0;
        h->kernel_launches[k] = 0;
    }
    return DSS_OK;
}

dss_status dss_get_timing(dss_handle *h, int kernel, double *total_ms, int64_t *launches)
{
    if (!h) return DSS_ERR_ARG;
    if (kernel < 0 || kernel >= dss_handle::kKernels) return fail(h, DSS_ERR_ARG, "kernel index out of range");
    dss_status s = collect_timing(h);
    if (s) return s;
    if (total_ms) *total_ms = h->kernel_ms[kernel];
    if (launches) *launches = h->kernel_launches[kernel];
    return DSS_OK;
}

static bool valid_params(const dss_params *p)
{
    return (p->L[0] > 0 && p->L[1] > 0 && p->L[2] > 0) && p->dt > 0 && p->cutoff_factor > 0 && p->rho > 0 &&
           p->a0 > 0 && p->reserved == 0 && p->capacity >= 0 && p->k_roll >= 0 && p->mu_roll >= 0 &&
           std::isfinite(p->k_roll) && std::isfinite(p->mu_roll) && std::isfinite(p->wave_amp) &&
           p->wave_n >= 0 && p->wave_n <= 1e6 && p->wave_n == std::floor(p->wave_n) &&
           (p->wave_amp == 0.0 || p->wave_n >= 1) &&
           (p->precision == DSS_FP64 || p->precision == DSS_MIXED) && p->eps_lub > 0 &&
           std::isfinite(p->shear_rate);
}

// Parameters of two boxes agree in everything but the box lengths and the shear rate.
static bool same_physics(const dss_params &a, const dss_params &b)
{
    dss_params x = a, y = b;
    for (int d = 0; d < 3; ++d) x.L[d] = y.L[d] = 0.0;
    x.shear_rate = y.shear_rate = 0.0;
    return std::memcmp(&x, &y, sizeof(dss_params)) == 0;
}

dss_status dss_create_batch(const dss_params *per_box, int32_t n_boxes, void *hip_stream, dss_handle **out)
{
    if (!per_box || !out || n_boxes < 1 || n_boxes > 65535) return DSS_ERR_ARG;
    *out = nullptr;
    for (int b = 0; b < n_boxes; ++b)
        if (!valid_params(&per_box[b]) || !same_physics(per_box[0], per_box[b])) return DSS_ERR_ARG;
    dss_handle *h = new dss_handle();
    h->prm = per_box[0];
    h->nbox = n_boxes;
    h->bprm.assign(per_box, per_box + n_boxes);
    if (hipGetDevice(&h->device) != hipSuccess || scratch_setup(h->device) != hipSuccess ||
        hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) {
        delete h;
        return DSS_ERR_HIP;
    }
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&h->stream) != hipSuccess) {
            delete h;
            return DSS_ERR_HIP;
        }
        h->own_stream = true;
    }
    *out = h;
    return DSS_OK;
}

dss_status dss_create(const dss_params *p, void *hip_stream, dss_handle **out)
{
    return dss_create_batch(p, 1, hip_stream, out);
}

void dss_destroy(dss_handle *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto e : h->ev_pool) (void)hipEventDestroy(e);
    free_all(h);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

dss_status dss_set_particles_batch(dss_handle *h, const int64_t *n_per_box, const double *x, const double *radius,
                                   const double *u, const double *omega, int on_device)
{
    if (!h) return DSS_ERR_ARG;
    if (!n_per_box || !x || !radius) return fail(h, DSS_ERR_ARG, "null n_per_box, x or radius");
    const int B = h->nbox;
    int64_t N = 0;
    for (int b = 0; b < B; ++b) {
        if (n_per_box[b] < 1) return fail(h, DSS_ERR_ARG, "every box needs at least one particle");
        N += n_per_box[b];
    }
    if (N > (int64_t)kKeyMask) return fail(h, DSS_ERR_ARG, "too many particles (ids must stay below 2^29)");
    const dss_params &p = h->prm;
    // host copies for validation and the lattice sizes
    std::vector<double> hx(3 * N), hr(N);
    if (on_device) {
        HIPTRY(hipMemcpy(hx.data(), x, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
        HIPTRY(hipMemcpy(hr.data(), radius, N * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::memcpy(hx.data(), x, 3 * N * sizeof(double));
        std::memcpy(hr.data(), radius, N * sizeof(double));
    }
    std::vector<BoxParams> boxes(B);
    std::vector<double> box_sa3(B, 0.0), box_amax(B, 0.0);
    std::vector<int> pbox(N);
    double a_min = INFINITY, a_max = 0.0;
    int64_t part = 0;
    for (int b = 0; b < B; ++b) {
        const dss_params &q = h->bprm[b];
        BoxParams &G = boxes[b];
        for (int64_t i = part; i < part + n_per_box[b]; ++i) {
            if (!(hr[i] > 0.0) || !std::isfinite(hr[i])) return fail(h, DSS_ERR_ARG, "radius must be finite and > 0");
            a_min = std::min(a_min, hr[i]);
            box_amax[b] = std::max(box_amax[b], hr[i]);
            box_sa3[b] += hr[i] * hr[i] * hr[i];
            for (int d = 0; d < 3; ++d)
                if (!(hx[3 * i + d] >= 0.0 && hx[3 * i + d] < q.L[d]))
                    return fail(h, DSS_ERR_ARG, "position outside [0, L) for particle " + std::to_string(i));
            pbox[i] = b;
        }
        a_max = std::max(a_max, box_amax[b]);
        for (int d = 0; d < 3; ++d) G.L[d] = q.L[d];
        G.gd = q.shear_rate;
        G.wk = 2.0 * kPi * q.wave_n / q.L[1];  // wave number of the wavy shear, eq. uinf
        G.part_off = (int)part;
        G.n_part = (int)n_per_box[b];
        part += n_per_box[b];
    }
    DevParams P{};
    P.eta0 = p.eta0; P.rho = p.rho; P.kn = p.kn; P.kt = p.kt; P.gn = p.gamma_n;
    P.inv_kt = p.kt > 0.0 ? 1.0 / p.kt : 0.0;
    P.mu = p.mu; P.fer = p.F_ER; P.lamd = p.lambda_D; P.a0 = p.a0; P.ham = p.hamaker; P.eps_vdw = p.eps_vdw;
    P.eps_lub = p.eps_lub; P.cf = p.cutoff_factor; P.dt = p.dt;
    P.k6 = 6.0 * kPi * p.eta0;
    P.k8 = 8.0 * kPi * p.eta0;
    P.inv_lamd = p.lambda_D > 0.0 ? 1.0 / p.lambda_D : 0.0;
    P.fer_a0 = p.F_ER / p.a0;
    P.nbox = B;
    P.N = (int)N;
    P.M = p.capacity > 0 ? p.capacity : paper_capacity(a_max, a_min);
    P.record_pairs = (p.flags & DSS_FLAG_RECORD_PAIRS) ? 1 : 0;
    // electro-chemical ranges (Fig. elch): repulsion below 20 lambda_D, attraction below 4 a0
    P.ec = (p.flags & DSS_FLAG_EC_RANGES) ? 1 : 0;
    P.rep_rng = (p.F_ER != 0.0 && p.lambda_D > 0.0) ? 20.0 * p.lambda_D : 0.0;
    P.att_rng = p.hamaker != 0.0 ? 4.0 * p.a0 : 0.0;
    P.rext = P.ec ? std::max(P.rep_rng, P.att_rng) : 0.0;
    P.kr = p.k_roll;
    P.inv_kr = p.k_roll > 0.0 ? 1.0 / p.k_roll : 0.0;
    P.mu_r = p.mu_roll;
    P.wave_amp = p.wave_amp;
    P.pair_cap = P.record_pairs ? pair_record_capacity(P, boxes, box_amax, n_per_box) : 0;
    // the lattice is checked before anything is freed or allocated
    {
        std::vector<BoxParams> trial = boxes;
        std::string why;
        SizeClasses sc;
        if (!lattice_of(trial, box_amax, a_min, p.cutoff_factor, P.ec ? P.rext : 0.0, h->tune.cell_scale,
                        h->tune.sized != 0, h->tune.tiled ? 4 * h->n_cu : 0, sc, why))
            return fail(h, DSS_ERR_BOX, why);
    }

    free_all(h);
    h->P = P;
    h->boxes = boxes;
    h->box_n.assign(n_per_box, n_per_box + B);
    h->box_sa3 = box_sa3;
    h->box_amax = box_amax;
    h->a_min = a_min;
    h->rad_host = hr;
    h->N = N;
    const size_t rows = (size_t)N * (size_t)P.M;
    for (int k = 0; k < 2; ++k) {
        HIPTRY(dalloc(&h->pa[k], N));
        HIPTRY(dalloc(&h->vel[k], N));
        HIPTRY(dalloc(&h->omg[k], N));
        HIPTRY(dalloc(&h->hkey[k], rows));
        HIPTRY(dalloc(&h->hxi[k], rows * 3));
        if (P.kr > 0.0) HIPTRY(dalloc(&h->hxr[k], rows * 3));
        HIPTRY(dalloc(&h->hcnt[k], N));
        HIPTRY(dalloc(&h->hown[k], N));
    }
    HIPTRY(dalloc(&h->ft_own, 6 * N));
    HIPTRY(dalloc(&h->ft_nb, 24 * N));
    HIPTRY(dalloc(&h->ft_x, 6 * N));
    HIPTRY(dalloc(&h->prev, N));
    HIPTRY(dalloc(&h->img, N));
    HIPTRY(hipMemsetAsync(h->img, 0, N * sizeof(int), h->stream));
    HIPTRY(dalloc(&h->cell, N));
    HIPTRY(dalloc(&h->rank, N));
    HIPTRY(dalloc(&h->pairs, P.record_pairs ? 2 * P.pair_cap : 2));
    HIPTRY(dalloc(&h->pair_count, 2));
    h->hist_count = h->pair_count + 1;
    HIPTRY(dalloc(&h->clk, 1));
    HIPTRY(dalloc(&h->run, 1));
    HIPTRY(dalloc(&h->sigma_last, 9 * (size_t)B));
    HIPTRY(dalloc(&h->box_diag, 3 * (size_t)B));
    dss_status ls = setup_lattice(h);
    if (ls) return ls;
    HIPTRY(hipMemsetAsync(h->pair_count, 0, sizeof(unsigned long long), h->stream));
    HIPTRY(hipMemsetAsync(h->clk, 0, sizeof(DevClock), h->stream));
    HIPTRY(hipMemsetAsync(h->sigma_last, 0, 9 * (size_t)B * sizeof(double), h->stream));
    HIPTRY(hipMemsetAsync(h->box_diag, 0, 3 * (size_t)B * sizeof(double), h->stream));
    for (int k = 0; k < 2; ++k) {
        HIPTRY(hipMemsetAsync(h->hcnt[k], 0, N * sizeof(int), h->stream));
        HIPTRY(hipMemsetAsync(h->hown[k], 0, N * sizeof(int), h->stream));
    }
    h->run_host = DevRun{};
    h->run_host.sigma_last = h->sigma_last;
    h->run_host.box_diag = h->box_diag;
    HIPTRY(hipMemcpyAsync(h->run, &h->run_host, sizeof(DevRun), hipMemcpyHostToDevice, h->stream));

    // stage the inputs on the device
    double *dx = nullptr, *dr = nullptr, *du = nullptr, *dw = nullptr;
    int *dpb = nullptr;
    HIPTRY(dalloc(&dx, 3 * N));
    HIPTRY(dalloc(&dr, N));
    HIPTRY(dalloc(&dpb, N));
    HIPTRY(hipMemcpyAsync(dx, hx.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPTRY(hipMemcpyAsync(dr, hr.data(), N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPTRY(hipMemcpyAsync(dpb, pbox.data(), N * sizeof(int), hipMemcpyHostToDevice, h->stream));
    if (u) {
        HIPTRY(dalloc(&du, 3 * N));
        HIPTRY(hipMemcpyAsync(du, u, 3 * N * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              h->stream));
    }
    if (omega) {
        HIPTRY(dalloc(&dw, 3 * N));
        HIPTRY(hipMemcpyAsync(dw, omega, 3 * N * sizeof(double),
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
    }
    h->cur = 0;
    h->hh = 0;
    h->step = 0;
    h->vel_is_half = false;
    h->tune_pending = false;
    const int grid = (int)((N + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_load, dim3(grid), dim3(kBlock), 0, h->stream, (int)N, dx, dr, du, dw, dpb, h->d_boxes,
                       h->pa[0], h->vel[0], h->omg[0], h->fb(), h->P.wave_amp);
    HIPTRY(hipGetLastError());
    h->loaded = true;
    dss_status s = evaluate(h, EVAL_SORT);
    HIPTRY(hipStreamSynchronize(h->stream));
    (void)hipFree(dx);
    (void)hipFree(dr);
    (void)hipFree(dpb);
    if (du) (void)hipFree(du);
    if (dw) (void)hipFree(dw);
    if (s != DSS_OK) return s;
    return check_flags(h);
}

dss_status dss_set_particles(dss_handle *h, int64_t N, const double *x, const double *radius, const double *u,
                             const double *omega, int on_device)
{
    if (!h) return DSS_ERR_ARG;
    if (h->nbox != 1) return fail(h, DSS_ERR_ARG, "a batch handle takes dss_set_particles_batch");
    if (N < 1 || N > (int64_t)kKeyMask || !x || !radius) return fail(h, DSS_ERR_ARG, "N < 1 or null x / radius");
    return dss_set_particles_batch(h, &N, x, radius, u, omega, on_device);
}

dss_status dss_set_tuning(dss_handle *h, const dss_tuning *t)
{
    if (!h || !t) return DSS_ERR_ARG;
    if (!(t->cell_scale >= 1.0 && t->cell_scale <= 4.0) || !(t->tile_scale >= 0.25 && t->tile_scale <= 4.0) ||
        (t->tiled != 0 && t->tiled != 1) || (t->graph != 0 && t->graph != 1) || (t->sized != 0 && t->sized != 1) ||
        t->wave_class < 0 || t->wave_class > 64 || t->queue_cap < 0 || t->adj_cap < 0 || t->adj_cap > 4096)
        return fail(h, DSS_ERR_ARG, "tuning out of range (cell_scale in [1, 4], tile_scale in [0.25, 4], "
                                    "wave_class in [0, 64], queue_cap >= 0, adj_cap in [0, 4096], flags 0/1)");
    if (t->sized && h->nbox != 1) return fail(h, DSS_ERR_ARG, "size-class stencils need a handle of one box");
    if (h->loaded) {
        // the lattice must still be legal for every box
        std::vector<BoxParams> trial = h->boxes;
        std::string why;
        SizeClasses sc;
        if (!lattice_of(trial, h->box_amax, h->a_min, h->prm.cutoff_factor, h->P.ec ? h->P.rext : 0.0,
                        t->cell_scale, t->sized != 0, t->tiled ? 4 * h->n_cu : 0, sc, why))
            return fail(h, DSS_ERR_BOX, why);
    }
    const bool lattice = t->cell_scale != h->tune.cell_scale || t->tile_scale != h->tune.tile_scale ||
                         t->tiled != h->tune.tiled || t->sized != h->tune.sized ||
                         t->wave_class != h->tune.wave_class;
    // the captured graphs hold the queue length as a kernel argument
    if (!t->graph || t->queue_cap != h->tune.queue_cap) destroy_graphs(h);
    h->tune = *t;
    if (h->loaded && lattice) h->tune_pending = true;
    return DSS_OK;
}

dss_status dss_get_tuning(dss_handle *h, dss_tuning *t)
{
    if (!h || !t) return DSS_ERR_ARG;
    *t = h->tune;
    return DSS_OK;
}

dss_status dss_set_step(dss_handle *h, int64_t n)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (n < 0) return fail(h, DSS_ERR_ARG, "negative time index");
    DevClock c;
    HIPTRY(hipMemcpyAsync(&c, h->clk, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    c.step = n;
    HIPTRY(hipMemcpyAsync(h->clk, &c, sizeof(c), hipMemcpyHostToDevice, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    h->step = n;
    return DSS_OK;
}

dss_status dss_build_neighbours(dss_handle *h)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (h->tune_pending) {
        // a new lattice takes effect at this counting sort
        s = setup_lattice(h);
        if (s) return s;
        h->tune_pending = false;
    }
    s = evaluate(h, EVAL_RESORT);
    if (s) return s;
    return check_flags(h);
}

dss_status dss_compute_forces(dss_handle *h)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    s = evaluate(h, EVAL_INPLACE);
    if (s) return s;
    return check_flags(h);
}

dss_status dss_step(dss_handle *h, int64_t n_steps, int64_t stress_every, int sync)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (n_steps < 0 || stress_every < 0) return fail(h, DSS_ERR_ARG, "negative n_steps or stress_every");
    // stress sampling schedule of this call
    int64_t first = 0, cap = 0;
    if (stress_every > 0) {
        first = ((h->step / stress_every) + 1) * stress_every;
        int64_t last = h->step + n_steps;
        cap = last >= first ? (last - first) / stress_every + 1 : 0;
    }
    if (cap > h->sample_cap_alloc) {
        if (h->samples) HIPTRY(hipFree(h->samples));
        h->samples = nullptr;
        HIPTRY(dalloc(&h->samples, 9 * (size_t)h->nbox * cap));
        h->sample_cap_alloc = cap;
    }
    h->run_host.sample_every = cap > 0 ? stress_every : 0;
    h->run_host.sample_first = first;
    h->run_host.sample_cap = cap;
    h->run_host.samples = h->samples;
    h->run_host.sigma_last = h->sigma_last;
    h->run_host.box_diag = h->box_diag;
    HIPTRY(hipMemcpyAsync(h->run, &h->run_host, sizeof(DevRun), hipMemcpyHostToDevice, h->stream));
    h->last_samples = cap;
    if (h->tune_pending && n_steps > 0) {
        // a new lattice takes effect at the counting sort of this step
        s = setup_lattice(h);
        if (s) return s;
        h->tune_pending = false;
    }
    const bool graphs = h->tune.graph && !h->graph_broken && h->timing == 0 && !h->P.record_pairs;
    // the stress and counters are summed only when a sample is due and after the last step;
    // with graphs, runs of steps as one launch: as long as the sampling period (2 .. 16) when
    // there is one, so that the runs of a call repeat, else kRunSteps / 2
    const StepRuns R(n_steps, stress_every, h->step);
    for (int64_t k = 0; k < n_steps;) {
        const int n = graphs ? R.length_at(k) : 1;
        if (n >= 2)
            s = graph_run(h, n, R.mask_at(k, n));
        else
            s = graphs ? graph_step(h, R.finish_at(k)) : evaluate(h, EVAL_STEP, R.finish_at(k));
        k += n;
        if (s) return s;
    }
    if (sync) return check_flags(h);
    return DSS_OK;
}

dss_status dss_prepare_steps(dss_handle *h, int64_t n_steps, int64_t stress_every)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (n_steps < 0 || stress_every < 0) return fail(h, DSS_ERR_ARG, "negative n_steps or stress_every");
    const bool graphs = h->tune.graph && !h->graph_broken && h->timing == 0 && !h->P.record_pairs;
    if (!graphs || h->tune_pending) return DSS_OK;  // direct launches, or a lattice change comes first
    // walk the call's runs as dss_step will, capturing the graphs it does not have yet; only
    // the handle's bookkeeping of the buffers advances, and it is put back
    const int cur = h->cur, hh = h->hh;
    const bool vih = h->vel_is_half;
    const int64_t step = h->step;
    const StepRuns R(n_steps, stress_every, h->step);
    for (int64_t k = 0; k < n_steps && !s;) {
        const int n = R.length_at(k);
        if (n >= 2) {
            hipGraphExec_t ge = nullptr;
            s = run_graph(h, n, R.mask_at(k, n), &ge);
        }
        for (int j = 0; j < n; ++j) commit_eval(h, true);
        k += n;
    }
    h->cur = cur;
    h->hh = hh;
    h->vel_is_half = vih;
    h->step = step;
    return s;
}

dss_status dss_read_stress_batch(dss_handle *h, double *sigma_last, double *sigma_mean, int64_t *n_samples)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    const int B = h->nbox;
    const int64_t ns = h->last_samples;
    std::vector<double> last(9 * (size_t)B);
    std::vector<double> smp(9 * (size_t)B * (size_t)std::max<int64_t>(ns, 1));
    HIPTRY(hipMemcpyAsync(last.data(), h->sigma_last, last.size() * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
    if (sigma_mean && ns > 0)
        HIPTRY(hipMemcpyAsync(smp.data(), h->samples, 9 * (size_t)B * ns * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    for (int b = 0; b < B; ++b) {
        const dss_params &p = h->bprm[b];
        const double V = p.L[0] * p.L[1] * p.L[2];
        // constant part: 2 eta0 E_inf + (1/V) sum_i 20/3 pi eta0 a_i^3 E_inf (eqs. stress, stresslet)
        double base[9] = {0};
        const double exy = 0.5 * p.shear_rate;
        const double c = 2.0 * p.eta0 * exy + (20.0 / 3.0) * kPi * p.eta0 * h->box_sa3[b] * exy / V;
        base[1] = c;
        base[3] = c;
        if (sigma_last)
            for (int k = 0; k < 9; ++k) sigma_last[9 * b + k] = base[k] + last[9 * b + k] / V;
        if (sigma_mean) {
            for (int k = 0; k < 9; ++k) {
                double acc = 0.0;
                for (int64_t q = 0; q < ns; ++q) acc += smp[(q * B + b) * 9 + k];
                sigma_mean[9 * b + k] = ns > 0 ? base[k] + acc / (double)ns / V : NAN;
            }
        }
    }
    if (n_samples) *n_samples = ns;
    return check_flags(h);
}

dss_status dss_read_stress(dss_handle *h, double *sigma_last, double *sigma_mean, int64_t *n_samples)
{
    if (!h) return DSS_ERR_ARG;
    if (h->nbox != 1) return fail(h, DSS_ERR_ARG, "a batch handle takes dss_read_stress_batch");
    return dss_read_stress_batch(h, sigma_last, sigma_mean, n_samples);
}

dss_status dss_get_state(dss_handle *h, double *x, double *u, double *omega, double *F, double *T, int on_device)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    const int64_t N = h->N;
    double *bufs[5] = {x, u, omega, F, T};
    double *dev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 5; ++k) {
        if (!bufs[k]) continue;
        if (on_device)
            dev[k] = bufs[k];
        else
            HIPTRY(dalloc(&dev[k], 3 * N));
    }
    const int grid = (int)((N + kBlock - 1) / kBlock);
    const int c = h->cur;
    hipLaunchKernelGGL(k_unsort, dim3(grid), dim3(kBlock), 0, h->stream, h->P, h->pa[c], h->vel[c], h->omg[c],
                       h->fb(), h->vel_is_half ? 1 : 0, 1, dev[0], dev[1], dev[2], dev[3], dev[4]);
    HIPTRY(hipGetLastError());
    for (int k = 0; k < 5; ++k)
        if (bufs[k] && !on_device)
            HIPTRY(hipMemcpyAsync(bufs[k], dev[k], 3 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    for (int k = 0; k < 5; ++k)
        if (bufs[k] && !on_device) (void)hipFree(dev[k]);
    return check_flags(h);
}

dss_status dss_get_eval_velocities(dss_handle *h, double *u, double *omega, int on_device)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    const int64_t N = h->N;
    double *bufs[2] = {u, omega};
    double *dev[2] = {nullptr, nullptr};
    for (int k = 0; k < 2; ++k) {
        if (!bufs[k]) continue;
        if (on_device)
            dev[k] = bufs[k];
        else
            HIPTRY(dalloc(&dev[k], 3 * N));
    }
    const int grid = (int)((N + kBlock - 1) / kBlock);
    const int c = h->cur;
    hipLaunchKernelGGL(k_unsort, dim3(grid), dim3(kBlock), 0, h->stream, h->P, h->pa[c], h->vel[c], h->omg[c],
                       h->fb(), h->vel_is_half ? 1 : 0, 0, (double *)nullptr, dev[0], dev[1], (double *)nullptr,
                       (double *)nullptr);
    HIPTRY(hipGetLastError());
    for (int k = 0; k < 2; ++k)
        if (bufs[k] && !on_device)
            HIPTRY(hipMemcpyAsync(bufs[k], dev[k], 3 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    for (int k = 0; k < 2; ++k)
        if (bufs[k] && !on_device) (void)hipFree(dev[k]);
    return DSS_OK;
}

dss_status dss_get_pairs(dss_handle *h, int64_t cap, int32_t *pairs, int64_t *n)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (!h->P.record_pairs) return fail(h, DSS_ERR_STATE, "pairs are recorded only with DSS_FLAG_RECORD_PAIRS");
    if (!n || cap < 0 || (cap > 0 && !pairs)) return fail(h, DSS_ERR_ARG, "null output");
    unsigned long long cnt = 0;
    HIPTRY(hipMemcpyAsync(&cnt, h->pair_count, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    *n = (int64_t)cnt;
    if ((int64_t)cnt > h->P.pair_cap) return fail(h, DSS_ERR_CAPACITY, "internal pair buffer overflow");
    if ((int64_t)cnt > cap) return fail(h, DSS_ERR_CAPACITY, "pair buffer too small");
    if (cnt) HIPTRY(hipMemcpy(pairs, h->pairs, 2 * cnt * sizeof(int32_t), hipMemcpyDeviceToHost));
    return DSS_OK;
}

dss_status dss_get_cells(dss_handle *h, int32_t *dims, int64_t cap_cells, int32_t *cell_start, int32_t *perm)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (dims)
        for (int d = 0; d < 3; ++d) dims[d] = h->boxes[0].nc[d];
    if (cell_start) {
        if (cap_cells < (int64_t)h->ncell_total + 1) return fail(h, DSS_ERR_CAPACITY, "cell_start buffer too small");
        HIPTRY(hipMemcpy(cell_start, h->cell_start, (h->ncell_total + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    if (perm) {
        std::vector<double4> w(h->N);
        HIPTRY(hipMemcpy(w.data(), h->omg[h->cur], h->N * sizeof(double4), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < h->N; ++i) perm[i] = (int32_t)w[i].w;
    }
    return DSS_OK;
}

// The committed contact history as (id_min, id_max, stretch) triples: the tangential
// stretches (rolling = false) or the rolling ones.
static dss_status export_history(dss_handle *h, int64_t cap, int32_t *pairs, double *xi, int64_t *n, bool rolling)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (!n) return fail(h, DSS_ERR_ARG, "null count");
    if (rolling && !h->hxr[h->hh]) return fail(h, DSS_ERR_STATE, "no rolling resistance (k_roll = 0)");
    int *dp = nullptr;
    double *dxv = nullptr;
    const int64_t room = std::max<int64_t>(cap, 1);
    HIPTRY(dalloc(&dp, 2 * room));
    HIPTRY(dalloc(&dxv, 3 * room));
    // its own counter: the listed-pair count of the last evaluation stays for dss_get_pairs
    HIPTRY(hipMemsetAsync(h->hist_count, 0, sizeof(unsigned long long), h->stream));
    const int grid = (int)((h->N + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_history_export, dim3(grid), dim3(kBlock), 0, h->stream, (int)h->N, h->P.M, h->hown[h->hh],
                       h->hkey[h->hh], rolling ? h->hxr[h->hh] : h->hxi[h->hh], h->hcnt[h->hh], (long long)cap, dp,
                       dxv, h->hist_count);
    HIPTRY(hipGetLastError());
    unsigned long long cnt = 0;
    HIPTRY(hipMemcpyAsync(&cnt, h->hist_count, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    *n = (int64_t)cnt;
    dss_status r = DSS_OK;
    if ((int64_t)cnt > cap) {
        r = fail(h, DSS_ERR_CAPACITY, "history buffer too small");
    } else if (cnt) {
        if (pairs) HIPTRY(hipMemcpy(pairs, dp, 2 * cnt * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (xi) HIPTRY(hipMemcpy(xi, dxv, 3 * cnt * sizeof(double), hipMemcpyDeviceToHost));
    }
    (void)hipFree(dp);
    (void)hipFree(dxv);
    return r;
}

dss_status dss_get_history(dss_handle *h, int64_t cap, int32_t *pairs, double *xi, int64_t *n)
{
    return export_history(h, cap, pairs, xi, n, false);
}

dss_status dss_get_rolling_history(dss_handle *h, int64_t cap, int32_t *pairs, double *xr, int64_t *n)
{
    return export_history(h, cap, pairs, xr, n, true);
}

dss_status dss_get_info(dss_handle *h, dss_info *info)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (!info) return fail(h, DSS_ERR_ARG, "null info");
    DevClock c;
    HIPTRY(hipMemcpyAsync(&c, h->clk, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    std::vector<double> d;
    s = read_diag(h, d);
    if (s) return s;
    info->n_particles = h->N;
    info->step = c.step;
    for (int k = 0; k < 3; ++k) info->cells[k] = h->boxes[0].nc[k];
    info->capacity = h->P.M;
    double np = 0.0, nc = 0.0, mf = 0.0;
    for (int b = 0; b < h->nbox; ++b) {
        np += d[3 * b];
        nc += d[3 * b + 1];
        mf = std::max(mf, d[3 * b + 2]);
    }
    info->n_pairs = (int64_t)np;
    info->n_contacts = (int64_t)nc;
    info->max_row_fill = (int32_t)mf;
    info->error_flags = (int32_t)c.err;
    double t = (double)c.step * h->prm.dt;
    info->le_offset = std::fmod(h->prm.shear_rate * h->prm.L[1] * t, h->prm.L[0]);
    return DSS_OK;
}

dss_status dss_get_box_info(dss_handle *h, int32_t box, dss_box_info *info)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (!info || box < 0 || box >= h->nbox) return fail(h, DSS_ERR_ARG, "null info or box out of range");
    DevClock c;
    HIPTRY(hipMemcpyAsync(&c, h->clk, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    std::vector<double> d;
    s = read_diag(h, d);
    if (s) return s;
    const BoxParams &G = h->boxes[box];
    info->n_particles = G.n_part;
    info->first_id = G.part_off;
    for (int k = 0; k < 3; ++k) {
        info->cells[k] = G.nc[k];
        info->L[k] = G.L[k];
    }
    info->first_cell = G.cell_off;
    info->n_pairs = (int64_t)d[3 * box];
    info->n_contacts = (int64_t)d[3 * box + 1];
    info->max_row_fill = (int32_t)d[3 * box + 2];
    info->size_classes = h->P.sized ? h->P.ncls : 1;
    info->shear_rate = G.gd;
    double t = (double)c.step * h->prm.dt;
    info->le_offset = std::fmod(G.gd * G.L[1] * t, G.L[0]);
    info->ec_far_rows[0] = h->P.ec_split ? h->P.ec_ry : 0;
    info->ec_far_rows[1] = h->P.ec_split ? h->P.ec_rz : 0;
    return DSS_OK;
}

}  // extern "C"

// ======================================================================================
// Adjoint: checkpointed reverse sweep over a run of n_steps time steps.
// ======================================================================================
namespace {

// Device copy of everything a time step, or an evaluation in place, reads from the
// previous one (including cell_start, which must match the sorted order of the records).
struct Snapshot {
    double4 *pa = nullptr, *vel = nullptr, *omg = nullptr;
    double *ft = nullptr;   // own 6N, nb 24N, x 6N
    int *cs = nullptr;      // cell_start, n_cells + 1
    int *hkey = nullptr, *hcnt = nullptr, *hown = nullptr;
    double *hxi = nullptr;
    double *hxr = nullptr;  // rolling stretches (only with rolling resistance)
    DevClock *clk = nullptr;
    double *sig = nullptr;  // sigma_last (9) and box_diag (3) of box 0
    int *img = nullptr;     // y-face crossing counts
    int cur = 0, hh = 0;
    int64_t step = 0;
    bool vel_is_half = false;
    void release()
    {
        void *ps[] = {pa, vel, omg, ft, cs, hkey, hcnt, hown, hxi, hxr, clk, sig, img};
        for (void *q : ps)
            if (q) (void)hipFree(q);
        *this = Snapshot{};
    }
};

dss_status snap_save(dss_handle *h, Snapshot &s)
{
    const int64_t N = h->N, M = h->P.M;
    if (!s.img) {  // allocated last: a snapshot without it is released and allocated whole
        s.release();
        HIPTRY(dalloc(&s.pa, N));
        HIPTRY(dalloc(&s.vel, N));
        HIPTRY(dalloc(&s.omg, N));
        HIPTRY(dalloc(&s.ft, 36 * N));
        HIPTRY(dalloc(&s.cs, (size_t)h->ncell_total + 1));
        HIPTRY(dalloc(&s.hkey, N * M));
        HIPTRY(dalloc(&s.hxi, 3 * N * M));
        if (h->hxr[h->hh]) HIPTRY(dalloc(&s.hxr, 3 * N * M));
        HIPTRY(dalloc(&s.hcnt, N));
        HIPTRY(dalloc(&s.hown, N));
        HIPTRY(dalloc(&s.clk, 1));
        HIPTRY(dalloc(&s.sig, 12));
        HIPTRY(dalloc(&s.img, N));
    }
    const hipMemcpyKind D = hipMemcpyDeviceToDevice;
    hipStream_t st = h->stream;
    HIPTRY(hipMemcpyAsync(s.pa, h->pa[h->cur], N * sizeof(double4), D, st));
    HIPTRY(hipMemcpyAsync(s.vel, h->vel[h->cur], N * sizeof(double4), D, st));
    HIPTRY(hipMemcpyAsync(s.omg, h->omg[h->cur], N * sizeof(double4), D, st));
    HIPTRY(hipMemcpyAsync(s.ft, h->ft_own, 6 * N * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(s.ft + 6 * N, h->ft_nb, 24 * N * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(s.ft + 30 * N, h->ft_x, 6 * N * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(s.cs, h->cell_start, ((size_t)h->ncell_total + 1) * sizeof(int), D, st));
    HIPTRY(hipMemcpyAsync(s.hkey, h->hkey[h->hh], N * M * sizeof(int), D, st));
    HIPTRY(hipMemcpyAsync(s.hxi, h->hxi[h->hh], 3 * N * M * sizeof(double), D, st));
    if (s.hxr) HIPTRY(hipMemcpyAsync(s.hxr, h->hxr[h->hh], 3 * N * M * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(s.hcnt, h->hcnt[h->hh], N * sizeof(int), D, st));
    HIPTRY(hipMemcpyAsync(s.hown, h->hown[h->hh], N * sizeof(int), D, st));
    HIPTRY(hipMemcpyAsync(s.clk, h->clk, sizeof(DevClock), D, st));
    HIPTRY(hipMemcpyAsync(s.sig, h->sigma_last, 9 * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(s.sig + 9, h->box_diag, 3 * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(s.img, h->img, N * sizeof(int), D, st));
    s.cur = h->cur;
    s.hh = h->hh;
    s.step = h->step;
    s.vel_is_half = h->vel_is_half;
    return DSS_OK;
}

dss_status snap_restore(dss_handle *h, const Snapshot &s)
{
    const int64_t N = h->N, M = h->P.M;
    const hipMemcpyKind D = hipMemcpyDeviceToDevice;
    hipStream_t st = h->stream;
    HIPTRY(hipMemcpyAsync(h->pa[s.cur], s.pa, N * sizeof(double4), D, st));
    HIPTRY(hipMemcpyAsync(h->vel[s.cur], s.vel, N * sizeof(double4), D, st));
    HIPTRY(hipMemcpyAsync(h->omg[s.cur], s.omg, N * sizeof(double4), D, st));
    HIPTRY(hipMemcpyAsync(h->ft_own, s.ft, 6 * N * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(h->ft_nb, s.ft + 6 * N, 24 * N * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(h->ft_x, s.ft + 30 * N, 6 * N * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(h->cell_start, s.cs, ((size_t)h->ncell_total + 1) * sizeof(int), D, st));
    HIPTRY(hipMemcpyAsync(h->hkey[s.hh], s.hkey, N * M * sizeof(int), D, st));
    HIPTRY(hipMemcpyAsync(h->hxi[s.hh], s.hxi, 3 * N * M * sizeof(double), D, st));
    if (s.hxr) HIPTRY(hipMemcpyAsync(h->hxr[s.hh], s.hxr, 3 * N * M * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(h->hcnt[s.hh], s.hcnt, N * sizeof(int), D, st));
    HIPTRY(hipMemcpyAsync(h->hown[s.hh], s.hown, N * sizeof(int), D, st));
    HIPTRY(hipMemcpyAsync(h->clk, s.clk, sizeof(DevClock), D, st));
    HIPTRY(hipMemcpyAsync(h->sigma_last, s.sig, 9 * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(h->box_diag, s.sig + 9, 3 * sizeof(double), D, st));
    HIPTRY(hipMemcpyAsync(h->img, s.img, N * sizeof(int), D, st));
    h->cur = s.cur;
    h->hh = s.hh;
    h->step = s.step;
    h->vel_is_half = s.vel_is_half;
    return DSS_OK;
}

// Stretch entries per contact in the canonical rows: the tangential stretch, and the rolling
// stretch after it when rolling resistance is on.
int stretch_width(const dss_handle *h) { return h->P.kr > 0.0 ? 6 : 3; }

// One recorded evaluation: state by id, listed pairs, committed history in canonical rows.
struct TapeEntry {
    double *x = nullptr, *u = nullptr, *w = nullptr;
    int *pairs = nullptr;
    int64_t npairs = 0;
    int *ckey = nullptr, *ccnt = nullptr;
    double *cxi = nullptr;  // per contact: xi, then xi^r with rolling resistance
    void release()
    {
        void *ps[] = {x, u, w, pairs, ckey, ccnt, cxi};
        for (void *q : ps)
            if (q) (void)hipFree(q);
        *this = TapeEntry{};
    }
};

dss_status tape_alloc(dss_handle *h, TapeEntry &t)
{
    const int64_t N = h->N, M = h->P.M;
    HIPTRY(dalloc(&t.x, 3 * N));
    HIPTRY(dalloc(&t.u, 3 * N));
    HIPTRY(dalloc(&t.w, 3 * N));
    HIPTRY(dalloc(&t.pairs, 2 * h->P.pair_cap));
    HIPTRY(dalloc(&t.ckey, N * M));
    HIPTRY(dalloc(&t.ccnt, N));
    HIPTRY(dalloc(&t.cxi, stretch_width(h) * N * M));
    return DSS_OK;
}

// Committed history -> canonical rows of a tape entry (their counts start at zero: cleared
// here, or already by the evaluation's k_predict when cleared = true).
dss_status tape_rows(dss_handle *h, TapeEntry &t, bool cleared = false)
{
    const int N = (int)h->N, M = h->P.M;
    const int grid = (N + kBlock - 1) / kBlock;
    if (!cleared) HIPTRY(hipMemsetAsync(t.ccnt, 0, N * sizeof(int), h->stream));
    const int sw = stretch_width(h);
    auto fill = sw == 6 ? k_canon_fill<6> : k_canon_fill<3>;
    auto sort = sw == 6 ? k_canon_sort<6> : k_canon_sort<3>;
    hipLaunchKernelGGL(fill, dim3(grid), dim3(kBlock), 0, h->stream, N, M, h->hown[h->hh], h->hkey[h->hh],
                       h->hxi[h->hh], h->hxr[h->hh], h->hcnt[h->hh], t.ckey, t.cxi, t.ccnt, h->clk);
    hipLaunchKernelGGL(sort, dim3(grid), dim3(kBlock), 0, h->stream, N, M, t.ckey, t.cxi, t.ccnt);
    HIPTRY(hipGetLastError());
    return DSS_OK;
}

// Point the pair recording of the next evaluation at a tape entry: the listed pairs go to
// its buffer and their count to its device slot (the host reads the counts of a whole
// segment at once).
void record_into(dss_handle *h, TapeEntry &t, unsigned long long *count_slot)
{
    h->pairs = t.pairs;
    h->pair_count = count_slot;
}

// State by id at the last evaluation -> tape entry.
dss_status tape_state(dss_handle *h, TapeEntry &t)
{
    const int N = (int)h->N;
    const int grid = (N + kBlock - 1) / kBlock;
    const int c = h->cur;
    hipLaunchKernelGGL(k_unsort, dim3(grid), dim3(kBlock), 0, h->stream, h->P, h->pa[c], h->vel[c], h->omg[c],
                       h->fb(), h->vel_is_half ? 1 : 0, 0, t.x, t.u, t.w, (double *)nullptr, (double *)nullptr);
    HIPTRY(hipGetLastError());
    return DSS_OK;
}

// Pair counts of tape entries lo .. hi from their device slots.
dss_status tape_counts(dss_handle *h, std::vector<TapeEntry> &tape, const unsigned long long *slots, int lo, int hi)
{
    std::vector<unsigned long long> c(hi - lo + 1);
    HIPTRY(hipMemcpyAsync(c.data(), slots + lo, c.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    for (int k = lo; k <= hi; ++k) {
        if ((int64_t)c[k - lo] > h->P.pair_cap) return fail(h, DSS_ERR_CAPACITY, "internal pair buffer overflow");
        tape[k].npairs = (int64_t)c[k - lo];
    }
    return DSS_OK;
}

// The adjoint's device workspace: checkpoints, tape entries and the reverse buffers (a
// DevList: a call with the shapes of the last one allocates nothing).
struct AdjointScratch {
    std::vector<Snapshot> ck;
    Snapshot fin;
    std::vector<TapeEntry> tape;
    DevList bufs;
    ~AdjointScratch()
    {
        for (auto &s : ck) s.release();
        fin.release();
        for (auto &t : tape) t.release();
    }
    template <class T>
    hipError_t get(T **p, size_t n)
    {
        return bufs.get(p, n);
    }
};

void release_adjoint_ws(dss_handle *h)
{
    delete h->adj_ws;
    h->adj_ws = nullptr;
}

// While the recompute records pairs straight into the tape entries, the handle's own pair
// buffer and count are set aside; they come back (with the recording flag) when the reverse
// sweep ends, also on an error return.
struct PairRecordGuard {
    dss_handle *h;
    int *pairs;
    unsigned long long *count;
    int rec;
    ~PairRecordGuard()
    {
        h->pairs = pairs;
        h->pair_count = count;
        h->P.record_pairs = rec;
        h->tape_x = h->tape_u = h->tape_w = nullptr;
        h->tape_zero = nullptr;
    }
};

}  // namespace

extern "C" dss_status dss_adjoint(dss_handle *h, int64_t n_steps, int64_t stress_every, int64_t ckpt_every,
                                  const double *weight, double *J, double *dJ_dparams, double *dJ_dx, double *dJ_du,
                                  double *dJ_dw, int on_device)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (h->nbox != 1) return fail(h, DSS_ERR_ARG, "the adjoint runs on single-box handles");
    if (h->P.wave_amp != 0.0) return fail(h, DSS_ERR_STATE, "the adjoint does not take the wavy shear");
    if (h->vel_is_half)
        return fail(h, DSS_ERR_STATE, "the adjoint starts from a state with forces at u^n: call it right after "
                                      "dss_set_particles or dss_compute_forces");
    if (n_steps < 1 || stress_every < 1 || ckpt_every < 1 || !weight)
        return fail(h, DSS_ERR_ARG, "n_steps, stress_every, ckpt_every must be >= 1 and weight non-null");
    const int64_t n0 = h->step, K = n_steps, C = ckpt_every;
    const int64_t first = ((n0 / stress_every) + 1) * stress_every;
    if (first > n0 + K) return fail(h, DSS_ERR_ARG, "no stress sample in the run (n_steps < stress_every)");
    const int64_t ns = (n0 + K - first) / stress_every + 1;
    const int N = (int)h->N, M = h->P.M;
    const int grid = (N + kBlock - 1) / kBlock;
    // pair recording for the tape (a larger buffer: the graphs, which hold the buffer and the
    // capacity, are captured again)
    const int rec0 = h->P.record_pairs;
    if (!rec0) {
        std::vector<int64_t> nb(h->boxes.size());
        for (size_t b = 0; b < h->boxes.size(); ++b) nb[b] = h->boxes[b].n_part;
        const int64_t cap = pair_record_capacity(h->P, h->boxes, h->box_amax, nb.data());
        if (h->P.pair_cap < cap) {
            destroy_graphs(h);
            if (h->pairs) HIPTRY(hipFree(h->pairs));
            h->pairs = nullptr;
            HIPTRY(dalloc(&h->pairs, 2 * cap));
            h->P.pair_cap = cap;
        }
    }
    const int64_t nck = (K + C - 1) / C;
    {
        // the workspace of the last call serves when its shapes are these
        const int64_t key[8] = {N, M, h->ncell_total, h->hxr[h->hh] ? 1 : 0, h->P.pair_cap, stretch_width(h), 0, 0};
        if (h->adj_ws && !std::equal(key, key + 8, h->adj_key)) release_adjoint_ws(h);
        if (!h->adj_ws) {
            h->adj_ws = new AdjointScratch;
            std::copy(key, key + 8, h->adj_key);
        }
    }
    AdjointScratch &W = *h->adj_ws;
    W.bufs.rewind();
    if ((int64_t)W.ck.size() < nck) W.ck.resize(nck);

    // ---------------- forward run with checkpoints and stress samples
    if (ns > h->sample_cap_alloc) {
        if (h->samples) HIPTRY(hipFree(h->samples));
        h->samples = nullptr;
        HIPTRY(dalloc(&h->samples, 9 * (size_t)h->nbox * ns));
        h->sample_cap_alloc = ns;
    }
    h->run_host.sample_every = stress_every;
    h->run_host.sample_first = first;
    h->run_host.sample_cap = ns;
    h->run_host.samples = h->samples;
    h->run_host.sigma_last = h->sigma_last;
    h->run_host.box_diag = h->box_diag;
    HIPTRY(hipMemcpyAsync(h->run, &h->run_host, sizeof(DevRun), hipMemcpyHostToDevice, h->stream));
    h->last_samples = ns;
    // the steps between checkpoints in graph runs, as dss_step takes them (the timing of the
    // reverse kernels does not stop them)
    const unsigned fwd_timed = h->timing & ~((1u << 5) | (1u << 6));
    const bool graphs = h->tune.graph && !h->graph_broken && fwd_timed == 0 && !h->P.record_pairs;
    const StepRuns R(K, stress_every, h->step);
    for (int64_t k = 0; k < K;) {
        if (k % C == 0) {
            s = snap_save(h, W.ck[k / C]);
            if (s) return s;
        }
        const int64_t seg_end = std::min<int64_t>(K, (k / C + 1) * C);  // the next checkpoint
        const int n = graphs && seg_end - k >= 2 ? (int)std::min<int64_t>(R.run, seg_end - k) : 1;
        if (n >= 2)
            s = graph_run(h, n, R.mask_at(k, n));
        else
            s = evaluate(h, EVAL_STEP, R.finish_at(k));
        k += n;
        if (s) return s;
    }
    double last[9], mean[9];
    int64_t nsr = 0;
    s = dss_read_stress_batch(h, last, mean, &nsr);
    if (s) return s;
    double Jv = 0.0;
    for (int k = 0; k < 9; ++k) Jv += weight[k] * mean[k];
    s = snap_save(h, W.fin);
    if (s) return s;

    // ---------------- reverse sweep
    const size_t n3 = 3 * (size_t)N;
    double *xb, *ub, *wb, *ax, *au, *aw, *Fb, *Tb, *Fb2, *Tb2, *theta, *rad, *Sb, *xibA, *xibB;
    int *bkey, *bcnt;
    unsigned long long *slots;
    HIPTRY(W.get(&slots, (size_t)C + 1));
    HIPTRY(W.get(&xb, n3)); HIPTRY(W.get(&ub, n3)); HIPTRY(W.get(&wb, n3));
    HIPTRY(W.get(&ax, n3)); HIPTRY(W.get(&au, n3)); HIPTRY(W.get(&aw, n3));
    HIPTRY(W.get(&Fb, n3)); HIPTRY(W.get(&Tb, n3)); HIPTRY(W.get(&Fb2, n3)); HIPTRY(W.get(&Tb2, n3));
    HIPTRY(W.get(&theta, 2)); HIPTRY(W.get(&rad, N)); HIPTRY(W.get(&Sb, 9));
    const int sw = stretch_width(h);
    HIPTRY(W.get(&xibA, sw * (size_t)N * M)); HIPTRY(W.get(&xibB, sw * (size_t)N * M));
    HIPTRY(W.get(&bkey, (size_t)N * M)); HIPTRY(W.get(&bcnt, N));
    // the recorded pairs by particle (per evaluation): lists of acap codes, their fill counts,
    // and the overflow list of the codes beyond a full list (at most every code)
    const int acap = h->tune.adj_cap > 0 ? h->tune.adj_cap : kAdjCap;
    const size_t ncode = 2 * (size_t)std::max<int64_t>(h->P.pair_cap, 1);
    int *apos = nullptr, *aadj = nullptr;
    unsigned *aovf_n = nullptr;
    int2 *aovf = nullptr;
    HIPTRY(W.get(&apos, (size_t)N)); HIPTRY(W.get(&aadj, (size_t)N * acap));
    HIPTRY(W.get(&aovf_n, 1)); HIPTRY(W.get(&aovf, ncode));
    double *agrad = nullptr;  // 18 cotangents per recorded pair
    HIPTRY(W.get(&agrad, 18 * (size_t)std::max<int64_t>(h->P.pair_cap, 1)));
    HIPTRY(hipMemsetAsync(apos, 0, (size_t)N * sizeof(int), h->stream));
    HIPTRY(hipMemsetAsync(aovf_n, 0, sizeof(unsigned), h->stream));
    double *zero_list[] = {xb, ub, wb, ax, au, aw, Fb, Tb, Fb2, Tb2};
    for (double *q : zero_list) HIPTRY(hipMemsetAsync(q, 0, n3 * sizeof(double), h->stream));
    HIPTRY(hipMemsetAsync(theta, 0, 2 * sizeof(double), h->stream));
    HIPTRY(hipMemsetAsync(xibA, 0, sw * (size_t)N * M * sizeof(double), h->stream));
    HIPTRY(hipMemsetAsync(bcnt, 0, N * sizeof(int), h->stream));
    {
        const double V = h->prm.L[0] * h->prm.L[1] * h->prm.L[2];
        double sb[9];
        for (int k = 0; k < 9; ++k) sb[k] = weight[k] / ((double)ns * V);
        HIPTRY(hipMemcpyAsync(Sb, sb, sizeof(sb), hipMemcpyHostToDevice, h->stream));
    }
    hipLaunchKernelGGL(k_rad_by_id, dim3(grid), dim3(kBlock), 0, h->stream, N, h->pa[h->cur], h->omg[h->cur], rad);
    if ((int64_t)W.tape.size() < C + 1) W.tape.resize(C + 1);
    for (int64_t k = 0; k <= C; ++k) {
        if (W.tape[k].cxi) continue;  // allocated last: the entry is whole
        W.tape[k].release();
        s = tape_alloc(h, W.tape[k]);
        if (s) return s;
    }
    DevParams Prec = h->P;
    Prec.record_pairs = 1;
    const BoxParams G = h->boxes[0];
    // the reverse of the pair terms of evaluation n from tape entry T1: the pair VJP (which also
    // lists each pair under its two ids), then the per-particle sums
    auto pairs_vjp = [&](const TapeEntry &T1, const VjpTape &tp, int64_t n, const double *xin, double *xout,
                         const double *sb) -> hipError_t {
        const int np = (int)T1.npairs;
        const int pg = std::max(1, (np + kBlock - 1) / kBlock);
        {
            TimedLaunch tl(h, 5);
            hipExtLaunchKernelGGL(k_pairs_vjp, dim3(pg), dim3(kBlock), 0, h->stream, tl.e0, tl.e1, 0, Prec, G,
                                  (long long)n, np, tp, xin, xout, Fb, Tb, sb, agrad, theta, acap, apos, aadj, aovf_n,
                                  aovf);
        }
        hipLaunchKernelGGL(k_pairs_vjp_sum, dim3(grid), dim3(kBlock), 0, h->stream, (int)N, acap, apos,
                           (const int *)aadj, (const unsigned *)aovf_n, (const int2 *)aovf, (const double *)agrad,
                           ax, au, aw);
        return hipGetLastError();
    };
    double *xib_in = xibA, *xib_out = xibB;
    PairRecordGuard guard{h, h->pairs, h->pair_count, rec0};
    h->P.record_pairs = 1;
    for (int64_t seg = nck - 1; seg >= 0; --seg) {
        const int64_t s0 = n0 + seg * C;
        const int64_t len = std::min<int64_t>(C, K - seg * C);
        s = snap_restore(h, W.ck[seg]);
        if (s) break;
        s = tape_rows(h, W.tape[0]);
        if (s) break;
        if (seg == 0) {
            // the evaluation at the initial state (its pairs; its state by id is written by the
            // next step's k_predict, which reads that state)
            record_into(h, W.tape[0], slots);
            s = evaluate(h, EVAL_INPLACE);
            if (s) break;
        }
        for (int64_t k = 1; k <= len; ++k) {
            record_into(h, W.tape[k], slots + k);
            // the state of evaluation k - 1 by id, written by this step's k_predict (the tape
            // entry 0 of a later segment is not read)
            const bool prev = seg == 0 || k >= 2;
            h->tape_x = prev ? W.tape[k - 1].x : nullptr;
            h->tape_u = prev ? W.tape[k - 1].u : nullptr;
            h->tape_w = prev ? W.tape[k - 1].w : nullptr;
            h->tape_zero = W.tape[k].ccnt;  // the counts of this step's canonical rows
            s = evaluate(h, EVAL_STEP, false);
            h->tape_x = h->tape_u = h->tape_w = nullptr;
            h->tape_zero = nullptr;
            if (s) break;
            s = tape_rows(h, W.tape[k], true);
            if (s) break;
        }
        if (s) break;
        s = tape_state(h, W.tape[len]);  // the segment's last evaluation
        if (s) break;
        s = tape_counts(h, W.tape, slots, seg == 0 ? 0 : 1, (int)len);
        if (s) break;
        if (seg < nck - 1) {
            // stretch adjoints at the segment boundary: rows of the later segment -> this one
            hipLaunchKernelGGL(sw == 6 ? k_canon_rekey<6> : k_canon_rekey<3>, dim3(grid), dim3(kBlock), 0, h->stream,
                               N, M, bkey, bcnt, xib_in, W.tape[len].ckey, W.tape[len].ccnt, xib_out);
            std::swap(xib_in, xib_out);
        }
        for (int64_t k = len; k >= 1; --k) {
            const int64_t n = s0 + k;
            const TapeEntry &T1 = W.tape[k], &T0 = W.tape[k - 1];
            // the stretch adjoints this step writes start at zero over the rows of T0 (after the
            // first step of the segment, the previous step's k_integrate_vjp cleared them)
            if (k == len)
                hipLaunchKernelGGL(sw == 6 ? k_canon_zero<6> : k_canon_zero<3>, dim3(grid), dim3(kBlock), 0, h->stream,
                                   N, M, T0.ccnt, xib_out);
            VjpTape tp{T1.pairs, T1.x, T1.u, T1.w, rad, T0.ckey, T0.ccnt, T0.cxi, T1.ckey, T1.ccnt, sw};
            const bool sampled = n >= first && (n - first) % stress_every == 0;
            HIPTRY(pairs_vjp(T1, tp, n, xib_in, xib_out, sampled ? Sb : (const double *)nullptr));
            const double c = (n - 1 == n0) ? 0.5 : 1.0;
            {
                TimedLaunch ti(h, 6);
                hipExtLaunchKernelGGL(k_integrate_vjp, dim3(grid), dim3(kBlock), 0, h->stream, ti.e0, ti.e1, 0, Prec,
                                      G.gd, N, c, 0, rad, Fb, Tb, ax, au, aw, xb, ub, wb, Fb2, Tb2, aovf_n,
                                      k >= 2 ? (const int *)W.tape[k - 2].ccnt : (const int *)nullptr, xib_in, M, sw);
            }
            std::swap(Fb, Fb2);
            std::swap(Tb, Tb2);
            std::swap(xib_in, xib_out);
        }
        HIPTRY(hipMemcpyAsync(bkey, W.tape[0].ckey, (size_t)N * M * sizeof(int), hipMemcpyDeviceToDevice, h->stream));
        HIPTRY(hipMemcpyAsync(bcnt, W.tape[0].ccnt, N * sizeof(int), hipMemcpyDeviceToDevice, h->stream));
        HIPTRY(hipGetLastError());
    }
    h->pairs = guard.pairs;
    h->pair_count = guard.count;
    h->P.record_pairs = rec0;
    if (s) return s;
    {
        // the evaluation at the initial state; the stretch of the initial history is held fixed
        const TapeEntry &T0 = W.tape[0];
        VjpTape tp{T0.pairs, T0.x, T0.u, T0.w, rad, T0.ckey, T0.ccnt, T0.cxi, nullptr, nullptr, sw};
        HIPTRY(pairs_vjp(T0, tp, n0, (const double *)nullptr, (double *)nullptr, (const double *)nullptr));
        hipLaunchKernelGGL(k_integrate_vjp, dim3(grid), dim3(kBlock), 0, h->stream, Prec, G.gd, N, 0.0, 1, rad, Fb, Tb,
                           ax, au, aw, xb, ub, wb, Fb2, Tb2, aovf_n, (const int *)nullptr, (double *)nullptr, M, sw);
        HIPTRY(hipGetLastError());
    }
    s = check_flags(h);
    if (s) return s;
    // outputs
    const hipMemcpyKind out = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (dJ_dx) HIPTRY(hipMemcpyAsync(dJ_dx, xb, n3 * sizeof(double), out, h->stream));
    if (dJ_du) HIPTRY(hipMemcpyAsync(dJ_du, ub, n3 * sizeof(double), out, h->stream));
    if (dJ_dw) HIPTRY(hipMemcpyAsync(dJ_dw, wb, n3 * sizeof(double), out, h->stream));
    double th[2];
    HIPTRY(hipMemcpyAsync(th, theta, sizeof(th), hipMemcpyDeviceToHost, h->stream));
    // leave the handle at the end of the run, as dss_step would
    s = snap_restore(h, W.fin);
    if (s) return s;
    HIPTRY(hipStreamSynchronize(h->stream));
    if (J) *J = Jv;
    if (dJ_dparams) {
        dJ_dparams[0] = th[0];
        dJ_dparams[1] = th[1];
    }
    return DSS_OK;
}

// Snapshot layout: header, then the current records, force records, cell_start, committed
// history, clock, last stress and counters, each as stored on the device.
namespace {
struct StateHeader {
    char magic[8];
    int32_t version, nbox;
    int64_t N, M, ncell, step;
    int32_t vel_is_half, reserved;
};
constexpr int32_t kStateVersion = 1;

struct StatePart {
    void *dev;
    size_t bytes;
};

std::vector<StatePart> state_parts(dss_handle *h, int cur, int hh)
{
    const size_t N = (size_t)h->N, M = (size_t)h->P.M, B = (size_t)h->nbox;
    return {{h->pa[cur], N * sizeof(double4)},
            {h->vel[cur], N * sizeof(double4)},
            {h->omg[cur], N * sizeof(double4)},
            {h->ft_own, 6 * N * sizeof(double)},
            {h->ft_nb, 24 * N * sizeof(double)},
            {h->ft_x, 6 * N * sizeof(double)},
            {h->cell_start, ((size_t)h->ncell_total + 1) * sizeof(int)},
            {h->hkey[hh], N * M * sizeof(int)},
            {h->hxi[hh], 3 * N * M * sizeof(double)},
            {h->hcnt[hh], N * sizeof(int)},
            {h->hown[hh], N * sizeof(int)},
            {h->hxr[hh], h->hxr[hh] ? N * M * 3 * sizeof(double) : 0},
            {h->img, N * sizeof(int)},
            {h->clk, sizeof(DevClock)},
            {h->sigma_last, 9 * B * sizeof(double)},
            {h->box_diag, 3 * B * sizeof(double)}};
}
}  // namespace

extern "C" {

dss_status dss_save_state(dss_handle *h, void *blob, size_t *bytes)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (!bytes) return fail(h, DSS_ERR_ARG, "null size");
    auto parts = state_parts(h, h->cur, h->hh);
    size_t need = sizeof(StateHeader);
    for (auto &q : parts) need += q.bytes;
    if (!blob) {
        *bytes = need;
        return DSS_OK;
    }
    if (*bytes < need) {
        *bytes = need;
        return fail(h, DSS_ERR_CAPACITY, "state buffer too small");
    }
    StateHeader hd{};
    std::memcpy(hd.magic, "DSSSTATE", 8);
    hd.version = kStateVersion;
    hd.nbox = h->nbox;
    hd.N = h->N;
    hd.M = h->P.M;
    hd.ncell = h->ncell_total;
    hd.step = h->step;
    hd.vel_is_half = h->vel_is_half ? 1 : 0;
    char *out = static_cast<char *>(blob);
    std::memcpy(out, &hd, sizeof(hd));
    size_t off = sizeof(hd);
    HIPTRY(hipStreamSynchronize(h->stream));
    for (auto &q : parts) {
        if (!q.bytes) continue;
        HIPTRY(hipMemcpy(out + off, q.dev, q.bytes, hipMemcpyDeviceToHost));
        off += q.bytes;
    }
    *bytes = need;
    return DSS_OK;
}

dss_status dss_load_state(dss_handle *h, const void *blob, size_t bytes)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (!blob || bytes < sizeof(StateHeader)) return fail(h, DSS_ERR_ARG, "null or short state");
    StateHeader hd;
    std::memcpy(&hd, blob, sizeof(hd));
    if (std::memcmp(hd.magic, "DSSSTATE", 8) != 0 || hd.version != kStateVersion)
        return fail(h, DSS_ERR_ARG, "not a state snapshot of this library version");
    if (hd.N != h->N || hd.M != h->P.M || hd.nbox != h->nbox || hd.ncell != h->ncell_total || h->tune_pending)
        return fail(h, DSS_ERR_STATE, "snapshot of another configuration (particle count, history capacity, boxes "
                                      "or cell lattice differ)");
    auto parts = state_parts(h, 0, 0);
    size_t need = sizeof(StateHeader);
    for (auto &q : parts) need += q.bytes;
    if (bytes != need) return fail(h, DSS_ERR_ARG, "state size does not match");
    const char *in = static_cast<const char *>(blob);
    size_t off = sizeof(hd);
    HIPTRY(hipStreamSynchronize(h->stream));
    for (auto &q : parts) {
        if (!q.bytes) continue;
        HIPTRY(hipMemcpy(q.dev, in + off, q.bytes, hipMemcpyHostToDevice));
        off += q.bytes;
    }
    h->cur = 0;
    h->hh = 0;
    h->step = hd.step;
    h->vel_is_half = hd.vel_is_half != 0;
    return DSS_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------------
// Observables (Sec. 3): shear-wise diffusivity and velocity autocorrelation from a
// reference time, local volume fraction along y, clusters of contacting particles.
// ----------------------------------------------------------------------------------
namespace {

// x and u^n by particle id into device buffers (3 N each).
dss_status state_by_id(dss_handle *h, double *x, double *u)
{
    const int grid = (int)((h->N + kBlock - 1) / kBlock);
    const int c = h->cur;
    hipLaunchKernelGGL(k_unsort, dim3(grid), dim3(kBlock), 0, h->stream, h->P, h->pa[c], h->vel[c], h->omg[c],
                       h->fb(), h->vel_is_half ? 1 : 0, 1, x, u, (double *)nullptr, (double *)nullptr,
                       (double *)nullptr);
    HIPTRY(hipGetLastError());
    return DSS_OK;
}

}  // namespace

extern "C" {

dss_status dss_observe_start(dss_handle *h)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (h->nbox != 1) return fail(h, DSS_ERR_ARG, "observables run on single-box handles");
    const int64_t N = h->N;
    if (!h->obs_y0) {
        HIPTRY(dalloc(&h->obs_y0, N));
        HIPTRY(dalloc(&h->obs_v0, N));
    }
    double *x = nullptr, *u = nullptr;
    h->obs_ws.rewind();
    HIPTRY(h->obs_ws.get(&x, 3 * N));
    HIPTRY(h->obs_ws.get(&u, 3 * N));
    s = state_by_id(h, x, u);
    if (!s) {
        const int grid = (int)((N + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_obs_ref, dim3(grid), dim3(kBlock), 0, h->stream, (int)N, h->boxes[0].L[1], x, u, h->img,
                           h->obs_y0, h->obs_v0);
        HIPTRY(hipGetLastError());
        HIPTRY(hipStreamSynchronize(h->stream));
        h->obs_step0 = h->step;
    }
    return s;
}

dss_status dss_observe(dss_handle *h, double out[4])
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (!out) return fail(h, DSS_ERR_ARG, "null output");
    if (h->obs_step0 < 0) return fail(h, DSS_ERR_STATE, "no reference: call dss_observe_start first");
    const int64_t N = h->N;
    const int grid = (int)((N + kBlock - 1) / kBlock);
    double *x = nullptr, *u = nullptr, *part = nullptr;
    h->obs_ws.rewind();
    HIPTRY(h->obs_ws.get(&x, 3 * N));
    HIPTRY(h->obs_ws.get(&u, 3 * N));
    HIPTRY(h->obs_ws.get(&part, 3 * (size_t)grid));
    s = state_by_id(h, x, u);
    std::vector<double> hp(3 * (size_t)grid);
    if (!s) {
        hipLaunchKernelGGL(k_obs_sums, dim3(grid), dim3(kBlock), 0, h->stream, (int)N, h->boxes[0].L[1], x, u, h->img,
                           h->obs_y0, h->obs_v0, part);
        HIPTRY(hipGetLastError());
        HIPTRY(hipMemcpy(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost));
    }
    if (s) return s;
    double sum[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < grid; ++b)
        for (int k = 0; k < 3; ++k) sum[k] += hp[3 * (size_t)b + k];
    const double elapsed = (double)(h->step - h->obs_step0) * h->prm.dt;
    const double msd = sum[0] / (double)N;
    const double gd = h->boxes[0].gd != 0.0 ? h->boxes[0].gd : 1.0;
    out[0] = elapsed > 0.0 ? msd / (2.0 * elapsed * h->prm.a0 * h->prm.a0 * gd) : 0.0;
    out[1] = sum[2] > 0.0 ? sum[1] / sum[2] : 0.0;
    out[2] = msd;
    out[3] = elapsed;
    return DSS_OK;
}

dss_status dss_phi_profile(dss_handle *h, int32_t nbins, double a_split, double *phi)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (h->nbox != 1) return fail(h, DSS_ERR_ARG, "observables run on single-box handles");
    if (nbins < 1 || nbins > 2048 || !phi) return fail(h, DSS_ERR_ARG, "nbins in [1, 2048] and phi non-null");
    const int64_t N = h->N;
    const int grid = (int)((N + kBlock - 1) / kBlock);
    double *part = nullptr;
    h->obs_ws.rewind();
    HIPTRY(h->obs_ws.get(&part, 2 * (size_t)nbins * grid));
    const BoxParams &G = h->boxes[0];
    hipLaunchKernelGGL(k_phi_profile, dim3(grid), dim3(kBlock), 2 * (size_t)nbins * sizeof(double), h->stream, (int)N,
                       G.L[1], (int)nbins, a_split, h->pa[h->cur], part);
    HIPTRY(hipGetLastError());
    std::vector<double> hp(2 * (size_t)nbins * grid);
    HIPTRY(hipMemcpy(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost));
    const double slab = G.L[0] * G.L[2] * (G.L[1] / (double)nbins);
    for (int k = 0; k < 2 * nbins; ++k) {
        double t = 0.0;
        for (int b = 0; b < grid; ++b) t += hp[(size_t)b * 2 * nbins + k];
        phi[k] = t / slab;
    }
    return DSS_OK;
}

dss_status dss_phi_profile_noalloc(dss_handle *h, int32_t nbins, double a_split, double *phi)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (h->nbox != 1) return fail(h, DSS_ERR_ARG, "observables run on single-box handles");
    if (nbins < 1 || nbins > 2048 || !phi) return fail(h, DSS_ERR_ARG, "nbins in [1, 2048] and phi non-null");
    double *ptr = scratch_of(h->device);
    if (!ptr) return fail(h, DSS_ERR_STATE, "no scratch address for this device");
    const int m = 2 * nbins;
    // partial profiles of at most (capacity - m) / m workgroups, then their sums, all in the scratch
    const int64_t cover = (h->N + kBlock - 1) / kBlock;
    const int64_t room = ((int64_t)kNoAllocDoubles - m) / m;
    const int grid = (int)std::max<int64_t>(1, std::min(cover, room));
    double *part = ptr, *sum = ptr + (size_t)grid * m;
    const BoxParams &G = h->boxes[0];
    hipLaunchKernelGGL(k_phi_profile, dim3(grid), dim3(kBlock), (size_t)m * sizeof(double), h->stream, (int)h->N,
                       G.L[1], (int)nbins, a_split, h->pa[h->cur], part);
    hipLaunchKernelGGL(k_phi_reduce, dim3((m + kBlock - 1) / kBlock), dim3(kBlock), 0, h->stream, part, grid, m, sum);
    HIPTRY(hipGetLastError());
    HIPTRY(hipMemcpyAsync(phi, sum, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    const double slab = G.L[0] * G.L[2] * (G.L[1] / (double)nbins);
    for (int k = 0; k < m; ++k) phi[k] = phi[k] / slab;
    return DSS_OK;
}

dss_status dss_contact_clusters(dss_handle *h, int64_t cap, int64_t *hist, int64_t *n_clusters, int64_t *largest)
{
    dss_status s = require_loaded(h);
    if (s) return s;
    if (cap < 1 || !hist) return fail(h, DSS_ERR_ARG, "cap >= 1 and hist non-null");
    const int64_t N = h->N;
    const int grid = (int)((N + kBlock - 1) / kBlock);
    int *parent = nullptr, *size = nullptr;
    unsigned long long *dh = nullptr;
    h->obs_ws.rewind();
    HIPTRY(h->obs_ws.get(&parent, N));
    HIPTRY(h->obs_ws.get(&size, N));
    HIPTRY(h->obs_ws.get(&dh, cap));
    HIPTRY(hipMemsetAsync(dh, 0, cap * sizeof(unsigned long long), h->stream));
    hipLaunchKernelGGL(k_cc_init, dim3(grid), dim3(kBlock), 0, h->stream, (int)N, parent, size);
    hipLaunchKernelGGL(k_cc_hook, dim3(grid), dim3(kBlock), 0, h->stream, (int)N, h->P.M, h->hown[h->hh],
                       h->hkey[h->hh], h->hcnt[h->hh], parent);
    hipLaunchKernelGGL(k_cc_count, dim3(grid), dim3(kBlock), 0, h->stream, (int)N, parent, size);
    hipLaunchKernelGGL(k_cc_hist, dim3(grid), dim3(kBlock), 0, h->stream, (int)N, parent, size, (long long)cap, dh);
    HIPTRY(hipGetLastError());
    std::vector<unsigned long long> hh(cap);
    HIPTRY(hipMemcpy(hh.data(), dh, cap * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    int64_t nc = 0, big = 0;
    for (int64_t k = 0; k < cap; ++k) {
        hist[k] = (int64_t)hh[k];
        nc += hist[k];
        if (hist[k]) big = k + 1;
    }
    if (n_clusters) *n_clusters = nc;
    if (largest) *largest = big;
    return DSS_OK;
}

}  // extern "C"
