/*
 * libmd -- short-range pair-force molecular dynamics on one MI355X (gfx950).
 *
 * The engine implements the force step compared in Rovigatti, Sulc, Reguly and
 * Romano, "A comparison between parallelization approaches in molecular
 * dynamics simulations on GPUs", in both of its decompositions and the
 * Newton's-third-law variant the paper weighs against them:
 *
 *   MD_MODE_VERTEX  one thread per particle walks that particle's Verlet list
 *                   and sums every pair itself; each pair is evaluated twice
 *                   and no memory is written concurrently (Methods section,
 *                   "vertex-based" approach; Fig. 1 left).
 *   MD_MODE_EDGE    one thread per potentially non-zero interaction (one entry
 *                   of the half list, sum_i n_i / 2 threads) evaluates the pair
 *                   once and adds +F to one particle and -F to the other with
 *                   atomic operations, skipped when the pair force is exactly
 *                   zero (Methods section, "edge-based" approach; Fig. 1 right).
 *   MD_MODE_NEWTON  the vertex approach with Newton's third law (Discussion
 *                   section, Fig. S2): the threads of particle i walk its half
 *                   list (j > i), evaluate each pair once, keep -F (and tau_i)
 *                   for i and add +F (and tau_j) to j atomically -- into one
 *                   of m replicated force (and torque) arrays that a closing
 *                   pass sums (md_params.newton_m = m >= 1, as in the paper),
 *                   or, with newton_m = 0, for LJ into a per-workgroup LDS
 *                   accumulator over the tile's neighbour region that is
 *                   added to the forces once per workgroup, for patchy
 *                   particles straight into the force and torque arrays.
 *   MD_MODE_EDGE_DET the edge approach made deterministic as the Methods
 *                   section describes as its alternative to atomics: one
 *                   thread per half-list entry stores the pair's result per
 *                   edge, and one thread per particle then sums the stored
 *                   results of its edges in the fixed order of its list
 *                   (needs md_params.edge_store = 1).  Bitwise reproducible.
 *
 * Both read Verlet lists of radius r_v = r_c + r_s built with a cell algorithm
 * (Methods section), and are followed by an FP64 velocity-Verlet update
 * (Methods section: positions and momenta are integrated in double precision;
 * forces may be computed in single precision).  The potentials are the
 * Lennard-Jones fluid (Eq. 1) and patchy particles (Eqs. 2-4: the paper's
 * two-patch model, or a four-patch variant; md_patch_model); md_thermostat
 * adds the NVT momentum refresh the Methods section runs with.
 *
 * Conventions for every entry point:
 *   - Every function returns md_status; nothing aborts or throws across the ABI.
 *     Argument errors are detected on the host before any HIP call.
 *   - Device buffers are owned by the caller (see md_create); libmd owns only the
 *     handle and a few bytes of host state (for md_step, 64 pinned bytes).
 *     libmd never calls hipMalloc.
 *   - Work is enqueued on the caller's HIP stream.  Functions marked "async"
 *     return before the GPU finishes; functions marked "syncs" wait for the
 *     stream and report sticky device-side errors (list overflow, non-finite
 *     forces) that earlier async calls raised.
 *   - Host arrays are AoS in the caller's original particle order: x[3*i+c],
 *     q[4*i+k] with q = (w, x, y, z) a unit Hamilton quaternion.
 *   - Units: lengths in sigma, energies in eps, masses in m; the box is cubic
 *     and periodic with side `box`, positions in [0, box).
 *   - A handle is not thread-safe; distinct handles on distinct streams are.
 */
#ifndef LIBMD_H
#define LIBMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_system md_system; /* opaque handle */

typedef enum {
    MD_OK = 0,
    MD_ERR_INVALID_ARG = -1,       /* bad parameter or NULL pointer            */
    MD_ERR_BUFFER_TOO_SMALL = -2,  /* caller buffer smaller than md_query_sizes */
    MD_ERR_HIP = -3,               /* a HIP runtime call failed                 */
    MD_ERR_NEIGHBOR_OVERFLOW = -4, /* a Verlet list exceeded max_neighbors      */
    MD_ERR_BOX_TOO_SMALL = -5,     /* box <= 2 r_v: minimum image not unique    */
    MD_ERR_NONFINITE = -6,         /* a force or position became NaN/Inf        */
    MD_ERR_STATE = -7              /* call out of order (e.g. no state set)     */
} md_status;

typedef enum { MD_POT_LJ = 0, MD_POT_PATCHY = 1 } md_potential;

/* Patch geometry and pair potential of MD_POT_PATCHY (md_params.patch_model).
 * d = x_j - x_i, u the unit patch directions, d_ab = d + patch_delta (u_j^b - u_i^a),
 * s_ab = |d_ab|; every term vanishes beyond rcut, patch terms also for
 * s_ab >= patch_rcut when patch_rcut > 0. */
typedef enum {
    /* four tetrahedral patches; WCA core of (eps, sigma) plus, for facing
     * patches (u_i^a . d > 0 and u_j^b . d < 0),
     * -eps_p exp(-s_ab^2 / w^2) cos^2(theta_i^a) cos^2(theta_j^b) */
    MD_PATCH_TETRA = 0,
    /* the paper's model (Eqs. 2-4 with M = 2): two patches at the poles
     * +-R(q) e_z; core (sigma/r)^200 plus -eps_p exp(-(s_ab / w)^10 / 2) per
     * patch pair (w = patch_w) */
    MD_PATCH_POLAR2 = 1
} md_patch_model;
typedef enum { MD_MODE_VERTEX = 0, MD_MODE_EDGE = 1, MD_MODE_NEWTON = 2, MD_MODE_EDGE_DET = 3 } md_mode;

/* Arithmetic of the pair forces.  Positions, velocities and the integrator are
 * FP64 in every variant (Methods section, mixed precision). */
typedef enum {
    MD_PREC_FP64 = 0,        /* pair maths and accumulation in FP64                */
    MD_PREC_FP32_F64ACC = 1, /* pair maths in FP32 from an FP64 separation, sums FP64 */
    MD_PREC_FP32_KAHAN = 2   /* pair maths in FP32, compensated FP32 sums           */
} md_precision;

typedef struct {
    int32_t n;             /* number of particles, >= 2                              */
    int32_t pot;           /* md_potential                                           */
    int32_t prec;          /* md_precision                                           */
    int32_t max_neighbors; /* Verlet-list capacity per particle (full list), >= 1    */
    double box;            /* cubic box side L; must exceed 2 (rcut + skin)          */
    double eps, sigma;     /* LJ (Eq. 1) or WCA core strength and diameter           */
    double rcut;           /* interaction cut-off r_c                                */
    double skin;           /* Verlet skin r_s >= 0; lists hold pairs with r < r_c+r_s */
    double mass;           /* particle mass > 0                                      */
    double dt;             /* time step > 0                                          */
    /* patchy particles (MD_POT_PATCHY) only */
    double eps_p;          /* patch-patch strength                                   */
    double patch_w;        /* width w of the patch attraction                        */
    double patch_delta;    /* distance of a patch from the particle centre           */
    double patch_rcut;     /* patch-patch cut-off; <= 0 means none                    */
    double inertia;        /* isotropic moment of inertia > 0                        */
    /* MD_MODE_NEWTON only */
    int32_t newton_m;      /* replicated force (and torque) arrays, 1 .. 64; 0: none  */
                           /* (LJ: LDS accumulation, patchy: atomics into F and tau)  */
    int32_t edge_store;    /* 1: workspace for MD_MODE_EDGE_DET (32 B (LJ) or 96 B    */
                           /* (patchy) per half-list entry, 4 B per full-list slot);  */
                           /* 0: none.  Half-list capacity below 2^31 entries          */
    int32_t cell_order;    /* slot order of the cells (md_cell_order); the default 0  */
                           /* stages tile regions in LDS, the others gather from      */
                           /* global memory (locality study of the paper's Methods)   */
    int32_t patch_model;   /* md_patch_model (MD_POT_PATCHY); 0 for MD_POT_LJ         */
} md_params;

/* Order of the cells, and so of the particle slots after every list build.
 * MD_CELLS_ROW_MAJOR stages each tile's neighbour region in LDS (the
 * default); the others use global gathers, the setting the paper's Hilbert
 * sort is about (Methods section: sorting particles along a space-filling
 * curve for memory locality). */
typedef enum {
    MD_CELLS_ROW_MAJOR = 0,         /* x fastest, then y, then z; LDS-staged tiles       */
    MD_CELLS_ROW_MAJOR_GATHER = 1,  /* the same order, every tile gathers from HBM       */
    MD_CELLS_MORTON = 2,            /* Z order: interleaved bits of (x, y, z)            */
    MD_CELLS_HILBERT = 3            /* 3-D Hilbert curve (Skilling's transposition)      */
} md_cell_order;

typedef struct {
    uint64_t state_bytes;     /* persistent particle state                       */
    uint64_t workspace_bytes; /* cell lists, Verlet lists, scratch               */
    uint64_t alignment;       /* required alignment of both buffers (bytes)      */
} md_sizes;

typedef struct {
    int64_t steps;          /* MD steps taken by md_step                           */
    int64_t rebuilds;       /* Verlet-list builds, including the initial one       */
    int64_t pairs;          /* half-list entries |E| at the last build             */
    int32_t max_list_len;   /* longest full list at the last build                 */
    int32_t n_cells;        /* cells per box side                                  */
    int32_t tiles_total;    /* tiles of the vertex pass                            */
    int32_t tiles_staged;   /* tiles whose neighbour region was staged in LDS      */
    int64_t nonzero_pairs;  /* half-list entries whose pair result (force, or for
                               patchy either torque) is non-zero at the current
                               positions, in the configured precision: the pairs
                               whose atomics the edge pass does not skip (Methods
                               section); 0 without built lists                   */
} md_stats_t;

/* Sizes of the two device buffers a system needs (pure host, no HIP call).
 * Returns MD_ERR_INVALID_ARG / MD_ERR_BOX_TOO_SMALL for bad parameters. */
md_status md_query_sizes(const md_params* p, md_sizes* out);

/* Pure host, no HIP call: rank[(z * nc + y) * nc + x] = position of cell
 * (x, y, z) of an nc^3 grid in the given order (a permutation of 0 .. nc^3-1;
 * curves over the enclosing power-of-two cube, ranked).  `rank` holds nc^3
 * ints, caller-owned.  MD_ERR_INVALID_ARG for nc < 1, nc > 1024 or an
 * unknown order. */
md_status md_cell_order_ranks(int32_t nc, int32_t order, int32_t* rank);

/* Create a system on the current HIP device.  d_state and d_workspace are
 * device buffers of at least the sizes md_query_sizes reports, aligned to
 * `alignment`; they are borrowed and must outlive the handle.  hip_stream is a
 * hipStream_t (NULL = default stream) on which all work of the handle runs.
 * Validation as md_query_sizes, plus MD_ERR_BUFFER_TOO_SMALL. */
md_status md_create(const md_params* p, void* d_state, uint64_t state_bytes,
                    void* d_workspace, uint64_t workspace_bytes, void* hip_stream,
                    md_system** out);

/* Upload particle state (host AoS, original order).  x and v are n*3 doubles;
 * q (n*4) and angmom (n*3) are required for MD_POT_PATCHY and ignored for LJ.
 * Positions are wrapped into [0, box).  Invalidates lists and forces.  Syncs. */
md_status md_set_state(md_system* s, const double* x, const double* v,
                       const double* q, const double* angmom);

/* Cell-list counting sort (Methods section: cell filling, one particle per
 * thread): bins particles into cells of side >= r_v, sorts them by cell (and
 * by original id inside a cell) and reorders the particle arrays into that
 * order.  Async. */
md_status md_build_cells(md_system* s);

/* Verlet-list build (Methods section: one particle per thread over the
 * neighbouring cells): full lists of all j with r_ij < r_v for the vertex
 * kernel, the half list (pairs counted once) for the edge kernel, and the
 * reference positions for the rebuild test.  Requires md_build_cells first.
 * Overflow of max_neighbors is reported by the next syncing call.  Async. */
md_status md_build_neighbors(md_system* s);

/* Pair forces (and torques for patchy) at the current positions with the
 * given decomposition.  Requires built lists.  Async. */
md_status md_forces(md_system* s, int32_t mode);

/* nsteps velocity-Verlet steps (rotational velocity Verlet for patchy) with
 * forces from `mode`.  Per step: half kick, drift, wrap; if any particle moved
 * more than skin/2 since the last build the cells and lists are rebuilt;
 * forces; half kick.  Computes forces first if they are not valid.  The
 * vertex LJ mode runs a step as one launch (forces, both half kicks, drift)
 * and enqueues these in small batches: a launch whose predecessor's drift
 * asks for a rebuild does nothing, the host learns of it from a pinned word
 * the launches write (allocated with hipHostMalloc on the first such call)
 * and enqueues the rebuild before resuming.  The other modes run the rebuild
 * test on the device every step.  Syncs at the end and reports device
 * errors. */
md_status md_step(md_system* s, int32_t nsteps, int32_t mode);

/* The NVT thermostat of the Methods section, in the reading of the Brownian
 * scheme it cites: every particle's momenta are redrawn, with probability
 * prob, from the Maxwell-Boltzmann distribution at `temperature` (v_c normal
 * with variance T / m; for patchy particles also L_c, variance I T).  Call it
 * between md_step calls, every so many steps.  Random numbers: Philox4x64-10
 * (Salmon et al., SC 2011) with key (seed, 0) and counter (i, counter, b, 0),
 * i the particle's index in the caller's order, b = 0, 1 the block;
 * u(r) = ((r >> 11) + 1/2) 2^-53.  Particle i is drawn when u(A0) < prob;
 * Box-Muller pairs sqrt(-2 ln u(a)) (cos 2 pi u(b), sin 2 pi u(b)) from
 * (A1, A2), (A3, B0), (B1, B2) give v_x, v_y, v_z, then L_x, L_y, L_z.  The
 * same (seed, counter) gives the same draws; use a new counter per call.
 * Positions and forces are unchanged.  Errors: temperature < 0 or not finite,
 * prob outside [0, 1] (MD_ERR_INVALID_ARG); no state, or md_build_cells not
 * yet followed by md_build_neighbors (MD_ERR_STATE).  Async. */
md_status md_thermostat(md_system* s, double temperature, double prob, uint64_t seed,
                        uint64_t counter);

/* Kinetic energy (translational + rotational), potential energy
 * sum_{i<j} V_ij and virial sum_{i<j} r_ij . F_j, reduced in FP64 in a fixed
 * order (deterministic for a given particle order).  Any output may be NULL.
 * Syncs. */
md_status md_energy(md_system* s, double* e_kin, double* e_pot, double* virial);

/* Per-particle potential energies e_i = 1/2 sum_j V_ij (n doubles, original
 * order), evaluated with the configured precision.  Syncs. */
md_status md_particle_energies(md_system* s, double* e);

/* Download state in original order; any pointer may be NULL.  x, v, f, angmom,
 * torque are n*3 doubles, q is n*4.  Syncs. */
md_status md_get_state(md_system* s, double* x, double* v, double* f, double* q,
                       double* angmom, double* torque);

/* Half list of the last build in original ids, each pair as (min id, max id).
 * Writes min(cap, |E|) pairs (2 int32 each) and stores |E| in *n_pairs.
 * Syncs. */
md_status md_get_pairs(md_system* s, int32_t* pairs, int64_t cap, int64_t* n_pairs);

/* Counters; syncs.  With built lists it also counts nonzero_pairs: fills the
 * half list if needed and evaluates every half-list pair once (a pass of the
 * cost of an edge force pass, without its atomics). */
md_status md_stats(md_system* s, md_stats_t* out);

/* Per-phase GPU time of md_step, from HIP events recorded on the system's
 * stream around each phase of every step while profiling is enabled:
 * integrate (half kick + drift + rebuild test), rebuild (cell sort and list
 * build kernels, which return at once when no rebuild is due), force (the
 * force kernels: for the LJ vertex pass the one kernel that also does the
 * closing half kick and the next step's half kick and drift; for the edge
 * and Newton passes the on-demand half-list fill, which returns at once
 * between builds, and the force kernel) and kick (the separate closing half
 * kick kernel of the passes that do not fuse it; zero otherwise).  Times are
 * summed over the steps taken since profiling was enabled. */
typedef struct {
    int64_t steps;
    double integrate_ms, rebuild_ms, force_ms, kick_ms;
} md_profile_t;

/* Enables (on != 0) or disables event timing of md_step and clears the sums.
 * Creates its events lazily; costs one event record per phase and step. */
md_status md_profile_enable(md_system* s, int32_t on);

/* Reads the sums (syncs). */
md_status md_profile_read(md_system* s, md_profile_t* out);

/* Destroy the handle (does not free the caller's buffers).  A system still
 * admitted to a batch is retired first. */
void md_destroy(md_system* s);

/* ---------------------------------------------------------------------------
 * Batched serving.  Many independent systems (different n, potential,
 * density and precision) advance together: every kernel of one step runs once
 * for the whole batch, each block serving one block's worth of one system, so
 * small systems share the GPU instead of each paying the launch latency of a
 * full step.  The paper times single systems only (Results section); the
 * batch runs the same per-system arithmetic -- a system's vertex-mode and
 * deterministic-edge-mode trajectories are bitwise the ones md_step gives it
 * alone, and an edge-mode one differs only by the order of its atomic
 * additions.  The deterministic edge mode needs systems made with
 * edge_store = 1 (md_batch_admit returns MD_ERR_INVALID_ARG otherwise).
 *
 * The batch keeps a device table of per-slot descriptors and, per block class
 * of the step, a map from grid block to (slot, block of that system).  Maps
 * are sized once from max_systems and max_particles, so admission and
 * retirement only rewrite the table and maps between launches.  The kernels
 * that hold a tile's neighbour region in LDS run in three LDS-size buckets,
 * each launched with its own LDS, so that systems with large regions do not
 * lower the occupancy of the others.  A launch runs steps_per_launch steps
 * (fewer when no system needs that many) as one hipGraph; grids are the
 * blocks in use rounded up to a power of two.  A graph is captured once per
 * step count; when admissions and retirements change the grids, its kernel
 * nodes are re-gridded in place, without a new capture.
 * ------------------------------------------------------------------------- */
typedef struct md_batch md_batch; /* opaque handle */

typedef struct {
    int32_t max_systems;      /* slots, 1 .. 65536                                    */
    int32_t mode;             /* md_mode of every step: vertex, edge or edge_det     */
    int32_t steps_per_launch; /* steps in one launch, 1 .. 4096                        */
    int32_t use_graph;        /* 1: launch captured hipGraphs; 0: launch kernels      */
    int64_t max_particles;    /* bound on the sum of n over admitted systems          */
    uint64_t pool_bytes;      /* bound on the sum of the systems' state + workspace
                                 bytes (md_query_sizes): the HBM footprint budget     */
} md_batch_params;

/* Device workspace bytes of a batch (pure host, no HIP call). */
md_status md_batch_query_sizes(const md_batch_params* p, uint64_t* workspace_bytes);

/* Create an empty batch.  d_workspace (aligned to 256 bytes, at least
 * md_batch_query_sizes bytes) is borrowed and must outlive the handle; all
 * work runs on hip_stream.  MD_ERR_INVALID_ARG for bad parameters,
 * MD_ERR_BUFFER_TOO_SMALL for a short or misaligned workspace. */
md_status md_batch_create(const md_batch_params* p, void* d_workspace, uint64_t workspace_bytes,
                          void* hip_stream, md_batch** out);

/* Admit a system for nsteps (>= 0) further steps and return its slot.  The
 * system must have built lists (md_build_neighbors); its forces are computed
 * with the batch's mode if not valid, and its own stream is drained.  While
 * admitted, every single-system call on it returns MD_ERR_STATE.  Returns
 * MD_ERR_BUFFER_TOO_SMALL, with nothing changed, when no slot is free or the
 * system would exceed pool_bytes, max_particles or a block-class capacity;
 * MD_ERR_STATE when it is in a batch already or has no lists.  Syncs the
 * batch stream. */
md_status md_batch_admit(md_batch* b, md_system* s, int64_t nsteps, int32_t* slot);

/* One launch: every admitted system with steps left advances by
 * min(steps left, k) steps, where k is steps_per_launch, or the smallest power
 * of two covering the largest need when that is fewer.  *steps_run (may be
 * NULL) receives k, 0 if no system had steps left.  Async. */
md_status md_batch_step(md_batch* b, int32_t* steps_run);

/* Steps the slot's system has left (host bookkeeping, no sync); -1 for a free
 * slot. */
md_status md_batch_steps_left(const md_batch* b, int32_t slot, int64_t* left);

/* Remove the slot's system from the batch (also to cancel it early) and free
 * the slot.  Syncs; returns the system's own device status (list overflow,
 * non-finite forces) and leaves it usable by the single-system calls. */
md_status md_batch_retire(md_batch* b, int32_t slot);

/* md_thermostat for the system in `slot` while it is admitted: the same
 * momentum refresh (same draws for the same seed and counter), enqueued on the
 * batch stream after the steps launched so far and before the next
 * md_batch_step.  Errors: a free slot, temperature < 0 or not finite, prob
 * outside [0, 1] (MD_ERR_INVALID_ARG).  Async. */
md_status md_batch_thermostat(md_batch* b, int32_t slot, double temperature, double prob,
                              uint64_t seed, uint64_t counter);

/* Waits for the batch stream. */
md_status md_batch_sync(md_batch* b);

typedef struct {
    int32_t active;          /* admitted systems                                     */
    int32_t lds_cap;         /* region capacity (slots) of the largest LDS bucket in use */
    int64_t particles;       /* sum of n over admitted systems                       */
    uint64_t bytes;          /* sum of their footprints                              */
    int64_t launches;        /* md_batch_step launches so far                        */
    int64_t captures;        /* graphs captured so far                               */
    int64_t regrids;         /* captured graphs re-gridded in place (no recapture)   */
} md_batch_info_t;

md_status md_batch_info(const md_batch* b, md_batch_info_t* out);

/* Retires every admitted system and destroys the handle (not the caller's
 * workspace). */
void md_batch_destroy(md_batch* b);

/* Description of the last error on this batch ("" if none). */
const char* md_batch_last_error(const md_batch* b);

/* ---- Without device allocation ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * md_forces_static computes what md_create + md_set_state + md_build_cells +
 * md_build_neighbors + md_forces compute (the same kernels), for coordinates
 * already on the device and with no workspace argument: the particle
 * records, cell lists and Verlet lists live in a static device array of the
 * library, MD_STATIC_SCRATCH_BYTES per GPU, which each GPU the library runs
 * on holds from the first call there until the process ends.  Nothing is
 * allocated (no hipMalloc, no host-side buffers); the call only enqueues
 * kernels on hip_stream (NULL = default stream) and returns.
 *
 *   d_x       device, n*3 doubles, positions in the caller's order (wrapped
 *             into [0, box) as md_set_state wraps them); read only
 *   d_q       device, n*4 doubles, quaternions (w, x, y, z), normalised on
 *             load; required for MD_POT_PATCHY, ignored for LJ
 *   d_f       device, n*3 doubles: forces in the caller's order (written)
 *   d_torque  device, n*3 doubles: torques (MD_POT_PATCHY; ignored for LJ)
 *   mode      any md_mode md_forces takes (MD_MODE_EDGE_DET needs edge_store)
 *   d_status  device int32 or NULL: receives MD_OK, MD_ERR_NEIGHBOR_OVERFLOW
 *             or MD_ERR_NONFINITE (non-finite or zero-norm input, or a
 *             non-finite force) once the call's kernels have run
 *
 * Host-detected errors, returned before anything is enqueued:
 * MD_ERR_INVALID_ARG / MD_ERR_BOX_TOO_SMALL as md_query_sizes, a missing
 * pointer, an unknown mode, a cell order other than the two row-major ones;
 * MD_ERR_BUFFER_TOO_SMALL if the system needs more than
 * MD_STATIC_SCRATCH_BYTES: it needs state_bytes + workspace_bytes of
 * md_query_sizes (an LJ fluid at rho = 0.8 with max_neighbors 208 about
 * 2.0 kB per particle, so up to about 33 000 particles).  MD_ERR_HIP if a
 * launch fails.
 *
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents: calls that overlap on a GPU (other streams, other host
 * threads) race and must be serialised by the caller.  Async. */
#define MD_STATIC_SCRATCH_BYTES (64ull << 20)

md_status md_forces_static(const md_params* p, const double* d_x, const double* d_q,
                           double* d_f, double* d_torque, int32_t mode, int32_t* d_status,
                           void* hip_stream);

/* Static description of a status code. */
const char* md_status_str(int32_t status);

/* Description of the last error on this handle ("" if none). */
const char* md_last_error(const md_system* s);

#ifdef __cplusplus
}
#endif
#endif /* LIBMD_H */
