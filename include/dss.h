/*
 * dss.h -- C ABI of the MI355X dense-suspension step library (libdss).
 *
 * Method: Monti, Rathee, Shen & Rosti, "A fast and efficient tool to study the
 * rheology of dense suspensions" (arXiv 2108.01013).  One time step advances N
 * polydisperse spheres under Lees-Edwards simple shear:
 *   - modified velocity-Verlet kick/drift (Sec. 2.1, numerical algorithm) and the
 *     Lees-Edwards wrap (eq. le);
 *   - counting sort of the particles into a cell lattice and the symmetric
 *     half-shell neighbour search (Sec. 2.1, Figs. alg and alg2);
 *   - pair forces: lubrication (eq. hydro, Appendix A), spring-dashpot contact with
 *     tangential history and Coulomb cap (eqs. contact0, csi), repulsion (eq. rep),
 *     attraction (eq. att), plus per-particle Stokes drag (eq. rst);
 *   - contact history in a reduced N x M matrix whose rows are sorted by partner
 *     index (Sec. 2.1, memory paragraph);
 *   - bulk stress tensor (eqs. stress, stresslet).
 *
 * Conventions (all entry points):
 *   - Every call returns a dss_status; DSS_OK = 0.  After an error,
 *     dss_last_error(h) returns a message owned by the handle.
 *   - Arrays of 3-vectors are N x 3, row-major, FP64, indexed by particle id
 *     0..N-1 = the order given to dss_set_particles.
 *   - "on_device" = 1: the pointer is device memory of the handle's GPU; 0: host
 *     memory.  The library never keeps a caller's pointer after a call returns;
 *     the caller keeps ownership of every buffer it passes.
 *   - All work is enqueued on the stream given to dss_create (NULL = a stream the
 *     handle creates).  Calls that return data to the caller synchronise that
 *     stream.  A handle is not thread-safe: use one handle per host thread/stream.
 *   - Device-side error flags (history-row overflow, non-finite forces) are checked
 *     whenever a call synchronises and reported as DSS_ERR_CAPACITY /
 *     DSS_ERR_UNSTABLE.
 */
#ifndef DSS_H
#define DSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dss_handle dss_handle;

typedef enum {
    DSS_OK = 0,
    DSS_ERR_ARG = 1,      /* invalid argument (null pointer, N < 1, non-positive size, bad position) */
    DSS_ERR_HIP = 2,      /* a HIP runtime call failed */
    DSS_ERR_CAPACITY = 3, /* a contact-history row or a caller buffer was too small */
    DSS_ERR_BOX = 4,      /* cell lattice too small: needs >= 4 cells along x and >= 3 along y, z */
    DSS_ERR_UNSTABLE = 5, /* non-finite force or torque */
    DSS_ERR_STATE = 6     /* call out of order (e.g. step before set_particles) */
} dss_status;

typedef enum { DSS_FP64 = 0, DSS_MIXED = 1 } dss_precision;

/* Bits of dss_params.flags */
#define DSS_FLAG_RECORD_PAIRS 1 /* keep the listed pairs of the last force evaluation (dss_get_pairs) */
/* Electro-chemical forces over their own ranges (Fig. elch): repulsion, eq. rep, while the
 * surface distance d_ij < 20 lambda_D, attraction, eq. att, while d_ij < 4 a0; lubrication
 * stays on |r| < cutoff_factor (a_i + a_j).  The pair set (and the cell lattice) then covers
 * |r| < max(cutoff_factor (a_i + a_j), a_i + a_j + the longest active range).  Without the
 * flag both forces are truncated at the lubrication list.  With size-class stencils a
 * particle's reach becomes 2 max(cutoff_factor, 1) a + the longest range.  On a handle of one
 * box without size classes (cutoff_factor >= 1) the lattice stays that of the lubrication
 * list when the longest reach 2 a_max + the longest range spans fewer than half the cell rows
 * along y and z and half of L_x: the pairs beyond the list then take a pass of their own
 * (central forces only), and the pair set is the same.  With the adjoint the three ranges
 * are held fixed like the pair set. */
#define DSS_FLAG_EC_RANGES 2

/* Physical and numerical parameters (units are the caller's; the defaults used by the
 * tests are eta0 = a_min = gdot = 1).  Ambient flow: simple shear U_inf = (gdot y, 0, 0),
 * Omega_inf = (0, 0, -gdot/2), E_inf_xy = E_inf_yx = gdot/2 (Sec. 2). */
typedef struct {
    double L[3];          /* box lengths; the box is [0, L_x) x [0, L_y) x [0, L_z) */
    double shear_rate;    /* gdot */
    double eta0;          /* fluid viscosity */
    double rho;           /* particle density: m = rho 4/3 pi a^3, I = 2/5 m a^2 */
    double kn, kt;        /* normal / tangential spring constants, eq. contact0 */
    double gamma_n;       /* normal dashpot, eq. contact0 */
    double mu;            /* Coulomb friction coefficient, eq. csi */
    double F_ER;          /* repulsion strength, eq. rep */
    double lambda_D;      /* Debye length, eq. rep */
    double a0;            /* reference radius of eq. rep */
    double hamaker;       /* Hamaker constant A, eq. att (0 = no attraction) */
    double eps_vdw;       /* attraction regularisation as a fraction of the harmonic radius */
    double eps_lub;       /* lubrication regularisation epsilon (Appendix A) */
    double cutoff_factor; /* a pair is listed iff |r| < cutoff_factor (a_i + a_j) */
    double dt;            /* time step */
    int32_t precision;    /* dss_precision */
    int32_t capacity;     /* history row capacity; 0 = the paper's estimate M(a_max, a_min) */
    int32_t flags;        /* DSS_FLAG_* */
    int32_t reserved;     /* must be 0 */
    double k_roll;        /* rolling spring stiffness k_r of Appendix roll (0 = no rolling resistance) */
    double mu_roll;       /* Coulomb coefficient of the rolling spring: |xi^r| <= mu_roll |F_nor| / k_r */
    double wave_amp;      /* amplitude W of the wavy shear of eq. uinf, U_inf = (gdot y + W sin(k y), 0, 0),
                           * k = 2 pi wave_n / L_y, with the Faxen terms of eqs. rst and stresslet
                           * (0 = simple shear; not with the adjoint) */
    double wave_n;        /* whole periods n of the wave along L_y (>= 1 when wave_amp != 0) */
} dss_params;

/* Diagnostics of the most recent force evaluation. */
typedef struct {
    int64_t n_particles;
    int64_t step;          /* time index n of the current state, t = n dt */
    int32_t cells[3];      /* lattice dimensions */
    int32_t capacity;      /* history row capacity M */
    int64_t n_pairs;       /* listed pairs */
    int64_t n_contacts;    /* pairs with d_ij < 0 */
    int32_t max_row_fill;  /* largest history row */
    int32_t error_flags;   /* raw device flags: 1 row overflow, 2 non-finite, 4 pair buffer overflow */
    double le_offset;      /* Lees-Edwards offset delta of the current state */
} dss_info;

/* Diagnostics of one box of a batch handle (dss_create_batch). */
typedef struct {
    int64_t n_particles;
    int64_t first_id;      /* the box's particles have ids first_id .. first_id + n_particles - 1 */
    int32_t cells[3];      /* lattice dimensions of the box */
    int32_t first_cell;    /* index of the box's first cell in the cell_start of dss_get_cells */
    int64_t n_pairs;       /* listed pairs of the last summed evaluation */
    int64_t n_contacts;
    int32_t max_row_fill;
    int32_t size_classes;  /* size classes of the cell numbering (1 unless size-class stencils) */
    double L[3];
    double shear_rate;
    double le_offset;      /* Lees-Edwards offset of the current state */
    int32_t ec_far_rows[2]; /* with DSS_FLAG_EC_RANGES on a lattice of the lubrication list: reach
                             * (cell rows along y, z) of the pass over the pairs beyond it; 0, 0
                             * when the lattice covers the whole pair set */
} dss_box_info;

/* Create a handle.  p is copied.  hip_stream: a hipStream_t of the current device, or
 * NULL.  Fails with DSS_ERR_ARG for non-positive L, dt, cutoff_factor, rho or a0, or
 * reserved != 0. */
dss_status dss_create(const dss_params *p, void *hip_stream, dss_handle **out);

/* Batched flow-curve sweep: one handle advances n_boxes independent boxes together (one
 * counting sort over the concatenated cell lattices, one pair launch over the cell rows of
 * every box, one stress tensor per box).  per_box: n_boxes parameter sets that may differ
 * only in L and shear_rate (each box has its own Lees-Edwards offset, eq. le); every other
 * field must equal per_box[0], else DSS_ERR_ARG.  A handle from dss_create is the
 * n_boxes = 1 case.  Particles are loaded with dss_set_particles_batch and the stress is
 * read with dss_read_stress_batch; every other entry point works on the whole batch with
 * particle ids running over the boxes in order (box b holds the ids first_id .. of
 * dss_get_box_info). */
dss_status dss_create_batch(const dss_params *per_box, int32_t n_boxes, void *hip_stream, dss_handle **out);

/* Load N particles (copy-in) and evaluate the initial forces at t = 0:
 * x: N x 3 positions inside the box; radius: N radii > 0; u, omega: N x 3 initial
 * velocities, or NULL for the ambient flow U_inf(x), Omega_inf.  The contact history
 * starts empty and the time index at 0.  Allocates all device memory of the handle
 * (sized for N and the row capacity M).  Fails with DSS_ERR_ARG for a position outside
 * [0, L) or a radius <= 0, DSS_ERR_BOX if the lattice has fewer than 4 x 3 x 3 cells. */
dss_status dss_set_particles(dss_handle *h, int64_t N, const double *x, const double *radius, const double *u,
                             const double *omega, int on_device);

/* dss_set_particles for a batch handle: n_per_box[b] >= 1 particles per box, stored box
 * after box in x, radius, u, omega (same layouts as dss_set_particles, N = the sum).
 * Positions of box b must lie in its own [0, L_b).  Each box gets its own lattice
 * (spacing >= 2 cutoff_factor times its largest radius); the history row capacity M is
 * taken over all particles.  Fails with DSS_ERR_BOX when a box has fewer than 4 x 3 x 3
 * cells or more than 4096 cell rows (n_y n_z). */
dss_status dss_set_particles_batch(dss_handle *h, const int64_t *n_per_box, const double *x, const double *radius,
                                   const double *u, const double *omega, int on_device);

/* Launch tuning of a handle.  None of these changes results: the pair set, forces and
 * stress do not depend on them (the summation order of the force atomics aside).
 *   cell_scale: lattice spacing = cell_scale x the box's largest pair cutoff (>= 1, <= 4;
 *               1 = the smallest legal cells); larger cells mean fewer, fuller cell rows;
 *               with size-class stencils, cell_scale x the reach of the smallest particle;
 *   tile_scale: scale (0.25 .. 4) of the k_pairs row-tile capacities, which are sized from
 *               the mean occupancy of a cell row; rows beyond them take the per-particle path;
 *   tiled:      1 = stage cell rows in LDS; 0 = every row takes the per-particle path;
 *   graph:      1 = dss_step replays HIP graphs of one time step (captured on first use;
 *               not while kernel timing is on or pairs are recorded);
 *   sized:      1 = size-class stencils for boxes of high size ratio (Section 2.2: cells
 *               fitted to the smallest particles, the stencil widened for larger ones): a
 *               particle of radius a searches a stencil of radius R(a) = floor(reach(a) / cw)
 *               + 1 cells, reach(a) = 2 c a (with DSS_FLAG_EC_RANGES 2 max(c, 1) a + the
 *               longest range), each pair is found by its larger member, the sort is class-major
 *               (dss_get_cells returns size_classes x n_cells + 1 starts); one box only
 *               (DSS_ERR_ARG on a batch handle); tile_scale and tiled are then unused;
 *   wave_class: with sized, size classes from this one up (stencil radius wave_class + 1
 *               and more) take one wavefront per particle; 0 = 3;
 *   queue_cap:  with sized, the length of the LDS queues of listed pairs (a workgroup's on
 *               the lane path, up to 4096; a wavefront's, up to 512), so that a scan stops
 *               and resumes after every queue_cap pairs; 0 = the full length, any other
 *               value only for checking the stop-and-resume path (it costs time);
 *   adj_cap:    the capacity of the per-particle lists of recorded pairs in the reverse
 *               sweep of dss_adjoint (0 = 32, at most 4096); the pairs of a particle beyond
 *               it are added from an overflow list with atomics, so a small value only
 *               checks that path.
 * Defaults: {1, 1, 1, 1, 0, 0, 0, 0}. */
typedef struct {
    double cell_scale;
    double tile_scale;
    int32_t tiled;
    int32_t graph;
    int32_t sized;
    int32_t wave_class;
    int32_t queue_cap;
    int32_t adj_cap;
} dss_tuning;

/* Set the launch tuning.  Before dss_set_particles it applies to the first lattice; after,
 * a new lattice takes effect at the counting sort of the next dss_step (dss_compute_forces
 * before that step still uses the current one).  Fails with DSS_ERR_ARG for values out of
 * range and DSS_ERR_BOX when a loaded box would get fewer than 4 x 3 x 3 cells. */
dss_status dss_set_tuning(dss_handle *h, const dss_tuning *t);
dss_status dss_get_tuning(dss_handle *h, dss_tuning *t);

/* Set the time index n of the current state (t = n dt; the Lees-Edwards offset follows
 * eq. le).  Forces are not re-evaluated: call dss_compute_forces afterwards.  For restarts
 * and for tests of the sheared boundary at arbitrary offsets.  Fails with DSS_ERR_ARG for
 * n < 0. */
dss_status dss_set_step(dss_handle *h, int64_t n);

/* Neighbour build of Sec. 2.1 (Figs. alg, alg2) at the current positions, without time
 * advance: cell id of every particle, counting sort into the cell lattice (histogram, exclusive
 * scan, scatter into cell-major order), the committed contact history moved with its
 * particles to their new sorted slots, then the half-shell pair search and the forces at the
 * current state (as dss_compute_forces).  A lattice set by dss_set_tuning takes effect here.
 * The cell lattice and order are read back with dss_get_cells.  Errors: DSS_ERR_STATE before
 * dss_set_particles, DSS_ERR_BOX for a pending lattice that is too small, DSS_ERR_CAPACITY /
 * DSS_ERR_UNSTABLE from the device flags (synchronises). */
dss_status dss_build_neighbours(dss_handle *h);

/* Forces, torques and stress of eqs. (hydro), (contact0), (csi), (rep), (att), (rst) and
 * (stress), (stresslet) at the current state (positions, velocities u^n, the current contact
 * history) over the pairs of the half-shell search of Sec. 2.1 in the current sorted order,
 * without advancing time or the history.  Synchronises; errors as dss_build_neighbours. */
dss_status dss_compute_forces(dss_handle *h);

/* Advance n_steps time steps of the modified velocity-Verlet scheme of Sec. 2.1 (numerical
 * algorithm): half kick and drift, the Lees-Edwards wrap of eq. (le), the counting sort and
 * half-shell search, the pair and particle forces of eqs. (hydro)-(att), the contact history
 * of the memory paragraph (rows sorted by partner id, entries of separated pairs dropped) and
 * the finishing kick.  If stress_every > 0, the stress tensor is sampled at
 * every step whose time index is a multiple of stress_every; the samples of this call
 * are returned by dss_read_stress.  The stress and the pair and contact counters are
 * summed only on those steps and on the last step of the call (the other steps skip the
 * stresslet; their forces, torques and history are the same).  Does not synchronise
 * unless sync != 0 (then device error flags are checked). */
dss_status dss_step(dss_handle *h, int64_t n_steps, int64_t stress_every, int sync);

/* Capture, without running anything, the HIP graphs that dss_step(h, n_steps, stress_every, .)
 * from the current state will replay (runs of consecutive steps: as many as the sampling period
 * when it is 2 .. 16, else 8, each run one graph launch; a last single step is captured when it
 * runs), so that the call itself spends no time capturing.  Leaves the state as it is.  Does
 * nothing when graphs are off (tuning, kernel timing, pair recording) or a lattice change is
 * pending; errors as dss_step.  Not part of the method: a host-side preparation for callers
 * that time or schedule the steps. */
dss_status dss_prepare_steps(dss_handle *h, int64_t n_steps, int64_t stress_every);

/* Stress of the last force evaluation (sigma_last, 9 values, row-major Sigma_ab) and the
 * mean over the samples of the last dss_step call (sigma_mean, nullable); n_samples
 * receives the sample count (nullable).  Sigma = 2 eta0 E_inf + (1/V)(sum_i S^S_i +
 * sum_pairs (S^L + S^C + S^E)), eq. stress, each pair once. */
dss_status dss_read_stress(dss_handle *h, double *sigma_last, double *sigma_mean, int64_t *n_samples);

/* dss_read_stress for a batch handle: sigma_last and sigma_mean hold n_boxes x 9 values
 * (box-major), each box's stress with its own volume and shear rate. */
dss_status dss_read_stress_batch(dss_handle *h, double *sigma_last, double *sigma_mean, int64_t *n_samples);

/* State at the current time index n, by particle id: x^n, u^n, omega^n, F^n, T^n (each
 * N x 3, nullable).  F, T are the totals of the last force evaluation. */
dss_status dss_get_state(dss_handle *h, double *x, double *u, double *omega, double *F, double *T, int on_device);

/* The velocities the last forces were evaluated with (u^{n-1/2}... i.e. the half-step
 * velocities u^{n+1/2} of the step that produced the state; after dss_compute_forces or
 * dss_set_particles they equal u^n, omega^n). */
dss_status dss_get_eval_velocities(dss_handle *h, double *u, double *omega, int on_device);

/* Listed pairs of the last force evaluation, (id_min, id_max), unordered; requires
 * DSS_FLAG_RECORD_PAIRS.  *n receives the count; fails with DSS_ERR_CAPACITY if cap < *n. */
dss_status dss_get_pairs(dss_handle *h, int64_t cap, int32_t *pairs, int64_t *n);

/* Cell lattice of the last counting sort: dims[3] (of box 0), cell_start (n_cells + 1
 * entries over the cells of every box, box after box) and perm (N entries: particle id at
 * each sorted position); host pointers. */
dss_status dss_get_cells(dss_handle *h, int32_t *dims, int64_t cap_cells, int32_t *cell_start, int32_t *perm);

/* Contact history after the last step: pairs (id_min, id_max) and xi (3 per pair, the
 * tangential stretch oriented from id_min to id_max), unordered; host pointers. */
dss_status dss_get_history(dss_handle *h, int64_t cap, int32_t *pairs, double *xi, int64_t *n);

/* Rolling stretches of the same contacts (Appendix roll: the spring on the rolling velocity
 * u_r = a_ij (n x w_i - n x w_j), a_ij = 2 a_i a_j / (a_i + a_j); it has no orientation):
 * pairs (id_min, id_max) and xr (3 per pair), unordered, host pointers.  Fails with
 * DSS_ERR_STATE when k_roll = 0, DSS_ERR_CAPACITY when cap < *n (*n is the count). */
dss_status dss_get_rolling_history(dss_handle *h, int64_t cap, int32_t *pairs, double *xr, int64_t *n);

/* Diagnostics of the most recent force evaluation (synchronises).  For a batch handle the
 * counts are summed over the boxes (max_row_fill: the largest), cells and le_offset are
 * those of box 0. */
dss_status dss_get_info(dss_handle *h, dss_info *info);

/* Diagnostics of box `box` (0 <= box < n_boxes) after the last summed evaluation. */
dss_status dss_get_box_info(dss_handle *h, int32_t box, dss_box_info *info);

/* Gradient of a stress objective by the discrete adjoint of the time step (reverse mode,
 * hand-written kernels).  Runs n_steps time steps from the current state, sampling the
 * stress every stress_every steps as dss_step does, and returns
 *   J = sum_ab weight[ab] mean_samples(Sigma_ab)      (weight: 9 values, row-major)
 * with its gradient with respect to the friction coefficient mu and the repulsion strength
 * F_ER (dJ_dparams[0], [1]) and to the state at the call, by particle id (dJ_dx, dJ_du,
 * dJ_dw: N x 3 each, nullable; host or device per on_device).  The derivative is that of
 * the recorded run with its pair set, contact states and Coulomb-cap states held fixed
 * (the step is smooth between these events); the contact history at the call is held
 * fixed.  State is checkpointed every ckpt_every steps and each segment is recomputed
 * forward before its reverse sweep (memory: one state and history copy per checkpoint plus
 * a segment of ckpt_every recorded steps).  This device workspace stays with the handle
 * and serves the next call of the same particle count, lattice and recording capacity
 * without allocating; dss_set_particles and dss_destroy free it.  On return the handle stands at the end of the
 * run, as after dss_step(h, n_steps, stress_every, 1).  Requires a single-box handle whose
 * forces were evaluated at u^n (right after dss_set_particles or dss_compute_forces: else
 * DSS_ERR_STATE) and at least one stress sample in the run (else DSS_ERR_ARG).  Takes the
 * electro-chemical ranges (which pair is inside which range is held fixed) and rolling
 * resistance (Appendix roll: the rolling stretch is carried and differentiated like the
 * tangential one, its Coulomb limit taken as in the run); the wavy shear is refused
 * (DSS_ERR_STATE). */
dss_status dss_adjoint(dss_handle *h, int64_t n_steps, int64_t stress_every, int64_t ckpt_every, const double *weight,
                       double *J, double *dJ_dparams, double *dJ_dx, double *dJ_du, double *dJ_dw, int on_device);

/* Snapshot of the whole time-stepping state into host memory: particle records (sorted
 * order), force records of the last evaluation, cell_start, committed contact history,
 * time index, last stress and counters.  blob = NULL: *bytes receives the size needed.
 * Otherwise *bytes is the capacity of blob (DSS_ERR_CAPACITY, with *bytes set to the size,
 * if too small) and receives the size written.  Synchronises the handle's stream. */
dss_status dss_save_state(dss_handle *h, void *blob, size_t *bytes);

/* Restore a snapshot of dss_save_state into a loaded handle of the same configuration (same
 * particle count, history capacity, boxes and cell lattice: the same handle, or one created
 * with the same parameters and loaded with the same particles).  Continuing from it repeats
 * the run from the snapshot's time index (up to the summation order of force atomics).
 * DSS_ERR_ARG for a malformed blob, DSS_ERR_STATE for another configuration. */
dss_status dss_load_state(dss_handle *h, const void *blob, size_t bytes);

/* Kernel timing with HIP events recorded on the handle's stream around the launches of
 * the kernels selected by enable (bit k: kernel k; -1: all; 0: off); every call starts a
 * new accumulation.  dss_get_timing synchronises and returns, for kernel k (0 predict or
 * velocity completion, 1 scan, 2 scatter, 3 pairs, 4 finish, 5 pair adjoint, 6 integrator
 * adjoint, 7 electro-chemical pairs beyond the lubrication list; with size-class stencils 3
 * is their one pair kernel), the summed duration in ms and the number of timed launches. */
dss_status dss_set_timing(dss_handle *h, int enable);
dss_status dss_get_timing(dss_handle *h, int kernel, double *total_ms, int64_t *launches);

/* Observables of Sec. 3 (single-box handles; DSS_ERR_ARG on a batch).
 * dss_observe_start: the current state becomes the reference time t0 (synchronises).
 * dss_observe: out = {D_y, C_v, <[y(t) - y(t0)]^2>, t - t0} at the current state, with
 *   D_y = <[y(t) - y(t0)]^2> / (2 (t - t0) a0^2 gdot), eq. (diffY) (gdot taken as 1 when 0;
 *   D_y = 0 at t = t0), y unwrapped across the sheared y faces, and
 *   C_v = <v'(t) v'(t0)> / <v'(t)^2>, eq. (corrV), v' = u_y; averages over all particles.
 *   DSS_ERR_STATE before dss_observe_start. */
dss_status dss_observe_start(dss_handle *h);
dss_status dss_observe(dss_handle *h, double out[4]);

/* Local volume fraction along y (Fig. localPhi): phi[g nbins + k] = volume of the spheres of
 * group g (0: radius <= a_split, 1: radius > a_split) inside the slab [k, k+1) L_y / nbins of
 * the periodic y axis, over the slab volume; 1 <= nbins <= 2048, phi host (2 nbins). */
dss_status dss_phi_profile(dss_handle *h, int32_t nbins, double a_split, double *phi);

/* dss_phi_profile for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same profile, with no hipMalloc,
 * hipFree or allocating library call.  Its partial profiles and their sums live in a device
 * array of the library, 8 MiB per GPU, taken when the first handle is created on that GPU and
 * held until the process ends; every call on one GPU shares it and leaves its last contents.
 * Calls on the same GPU that overlap in time (two host threads, or two streams) race on it and
 * must be serialised by the caller.  Particles are taken in workgroups of 256 over at most
 * (2^20 - 2 nbins) / (2 nbins) workgroups, so any N fits; nbins beyond 2048 is DSS_ERR_ARG.
 * phi: host, 2 nbins values as in dss_phi_profile (equal up to the order of the sums). */
dss_status dss_phi_profile_noalloc(dss_handle *h, int32_t nbins, double a_split, double *phi);

/* Clusters of contacting particles (Fig. histo): connected components of the graph of the
 * committed contacts (d_ij < 0 at the last step).  hist[s - 1] = number of clusters of s
 * particles for s < cap, hist[cap - 1] those of cap or more (isolated particles are clusters
 * of 1); *n_clusters their total, *largest the largest s with hist[s - 1] > 0 (nullable);
 * host pointers. */
dss_status dss_contact_clusters(dss_handle *h, int64_t cap, int64_t *hist, int64_t *n_clusters, int64_t *largest);

const char *dss_last_error(const dss_handle *h);
const char *dss_status_string(dss_status s);
void dss_destroy(dss_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* DSS_H */
