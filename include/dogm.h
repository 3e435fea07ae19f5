/*
 * dogm.h - C ABI of the MI355X (gfx950) implementation of the per-cycle particle recursion of
 * the Dempster-Shafer PHD/MIB dynamic occupancy grid filter (Nuss et al., "A Random Finite Set
 * Approach for Dynamic Occupancy Grid Maps with Real-Time Application", arXiv 1605.02406,
 * Sec. VI and the parallel form of Sec. VII, Algorithms 1-7).
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory.   The library never allocates device memory.  One grid lives entirely inside one
 *           caller-owned device buffer (the "arena", size from dogm_arena_bytes).  The arena
 *           must stay allocated and must not be touched by the caller while the grid exists,
 *           except through the arrays that dogm_view exposes.  The grid handle itself is a
 *           small host object owned by the library (freed by dogm_destroy).
 * Streams.  Every call only enqueues kernels on the grid's HIP stream and returns without
 *           synchronising; results are visible to work ordered after it on that stream.  No
 *           call reads device memory back to the host, so a cycle can be captured in a HIP
 *           graph.  Calls on one grid must not overlap from several host threads.
 * Errors.   Every call returns an int: DOGM_OK (0) or a negative code below.  A failed call
 *           enqueues nothing (argument and state checks) or reports the launch error of HIP
 *           (DOGM_EHIP, text from dogm_last_error).  Numeric anomalies found on the device
 *           set bits of the device status word (DOGM_ST_*), readable through dogm_view.
 * Order.    init -> per cycle: predict, assign, update, [moments], resample (or step).  A call
 *           out of this order returns DOGM_ESTATE and enqueues nothing.
 * Layout.   Cells are row-major, cell = iy*nx + ix, origin at the grid corner; x spans
 *           [0, nx*cell_size), y spans [0, ny*cell_size).  Particles are structure-of-arrays
 *           FP32 (x, y, vx, vy, w).  Key C (= nx*ny) marks a particle outside the grid.
 */
#ifndef DOGM_H
#define DOGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A hipStream_t, passed as an opaque pointer (NULL = the null stream). */
typedef void* dogm_stream_t;

typedef struct dogm_grid dogm_grid;

enum {
    DOGM_OK = 0,
    DOGM_EINVAL = -1,  /* bad pointer, parameter or size                            */
    DOGM_ESIZE = -2,   /* arena too small                                          */
    DOGM_EHIP = -3,    /* a HIP call or kernel launch failed                       */
    DOGM_ESTATE = -4,  /* call out of order                                        */
    DOGM_ENOTIMPL = -5 /* switched off in this version of the library             */
};

/* Device status word bits. */
enum {
    DOGM_ST_CONFLICT = 1u,  /* Dempster total conflict (1-K < 1e-12): prediction kept  */
    DOGM_ST_NOCARRIER = 2u, /* a cell with new-born mass received no new-born slot     */
    DOGM_ST_NONFINITE = 4u, /* a non-finite mass or weight was met                     */
    DOGM_ST_INTERNAL = 8u   /* an internal consistency check failed (library bug)      */
};

/* Filter parameters (Table I and the process model of eq. (process)). */
typedef struct dogm_params {
    int32_t nx, ny;        /* cells along x and y, 1 <= nx, ny; nx*ny < 2^24 (see below)   */
    float cell_size;       /* cell edge r [m], > 0                                          */
    float dt;              /* time step T [s]                                               */
    float p_s;             /* persistence probability p_S, eq. (particle_persistence)       */
    float p_b;             /* birth probability p_B, eq. (predicted_ex_born)                */
    float sigma_pos;       /* process-noise SD on position per step [m]                     */
    float sigma_vel;       /* process-noise SD on velocity per step [m/s]                   */
    float sigma_birth_vel; /* SD of new-born velocity sigma_B,v [m/s] (Table I)             */
    float alpha_free;      /* free-mass discount alpha(T) in [0,1], eq. (DS_freespace_pred) */
    int64_t n_pers;        /* persistent particles nu, 1 <= nu < 2^27 (see below)           */
    int64_t n_born;        /* new-born slots nu_b, 0 <= nu_b < 2^30                         */
    uint64_t seed;         /* Philox4x32-10 key                                            */
    uint32_t grid_id;      /* fourth Philox counter word: separates grids with one seed     */
    uint32_t model;        /* DOGM_MODEL_DS (0) or DOGM_MODEL_PHD_MIB (1), see below        */
    uint32_t precision;    /* DOGM_PRECISION_FP32 (0) or DOGM_PRECISION_FP64 (1), see below */
    /* Launch plan (results do not depend on it; a tuner picks it by timing, see below). */
    uint32_t sort_passes;  /* radix passes of Alg. 2's sort: 0 = the fewest whose digits have
                              at most 11 bits; else that many (at least the fewest, at most 3) */
    uint32_t scan_parts;   /* prefix of the per-tile partial sums (new-born masses, joint
                              weights): 0 = scanned once by a kernel of its own for grids with
                              more than 4096 of them, else added up by every consumer block;
                              1 = always scanned; 2 = scanned only when a grid of the same
                              launch asks for it                                            */
    uint32_t resample;     /* Alg. 7's outputs: 0 = automatic (1 above 2^22 persistent
                              particles, else 2); 1 = every tile's outputs shared evenly by its
                              threads; 2 = each source's draws written by the lane that owns it
                              (one kernel per launch: 1 if any grid of the launch asks for it) */
} dogm_params;

/* The launch plan changes how the work is cut into launches and tiles, never a result: the sort
 * is stable, so every digit plan gives the same permutation, and the prefix sums are exact
 * integer sums whichever kernel forms them.  Grids with different plans may share a batch. */

/* Precision modes.  DOGM_PRECISION_FP32: the particle state and the per-cell masses and moments
 * are stored in FP32; per-cell sums, the normalisation of Alg. 4 and the cell update are
 * evaluated in FP64, and the integer decisions (slot offsets of Alg. 5, the resampling CDF of
 * Alg. 7) on masses rounded to multiples of 2^-40 and summed exactly in 64-bit integers.
 * DOGM_PRECISION_FP64: every real-valued array (each "FP32" array of dogm_views below, except
 * the caller's measurement) holds FP64 and every step computes in FP64 (Box-Muller and the cell
 * decision included), with the same exact integer decisions; the arena grows accordingly. */
enum { DOGM_PRECISION_FP32 = 0, DOGM_PRECISION_FP64 = 1 };

/* Size limits.  Masses are summed in 64-bit fixed point (units of 2^-40; every cell holds at
 * most mass 1), which cannot overflow for nx*ny < 2^24.  The systematic draws of Alg. 7 are
 * evaluated in FP64 (spacing W/nu rounded once, then (j + U) times it); for nu < 2^27 the
 * last draw stays below the joint weight W however large W is, so every draw finds a
 * particle.  dogm_arena_bytes and dogm_init_grid return DOGM_EINVAL beyond either limit. */

/* The per-cell step of the filter.
 *  DOGM_MODEL_DS: the Dempster-Shafer approximation of Sec. VI (eqs. (DS_particle_sum_pred) to
 *    (DS_resulting_masses1/2)); measurements are the BBA m_occ, m_free; new-born mass only in
 *    cells with m_z(O) > 0.
 *  DOGM_MODEL_PHD_MIB: the particle PHD/MIB filter of Sec. V without that approximation, with
 *    p_A = 0: per cell r_p = min(sum w, 1), r_b = p_B (1 - r_p) (every cell), r = r_p + r_b,
 *    and every weight is scaled by f = p_TP / (p_FP (1 - r) + p_TP r) after a measurement
 *    (eqs. (updateParticleWeightsUnnormalized), (applyNormalization),
 *    (normalizationCalculation)) or by f = (1 - p_TP) / ((1 - p_TP) r + (1 - p_FP) (1 - r))
 *    without one (eq. (updateParticleWeightsEmpty)); rho_p = f r_p, rho_b = f r_b.  The cell
 *    outputs keep the layout of the first model: m_pO = r_p, m_pF = 1 - r, m_O = pign = f r,
 *    m_F = 1 - f r.  Measurements are p_tp, p_fp and det; alpha_free is not used. */
enum { DOGM_MODEL_DS = 0, DOGM_MODEL_PHD_MIB = 1 };

/* One measurement grid (Sec. VI.C): device pointers to C floats each, read only during the
 * dogm_update / dogm_step call's kernels.  m_occ, m_free: the observed BBA m_z(O), m_z(F)
 * with m_occ + m_free <= 1 (required).  p_assoc: association probability p_A per cell, or
 * NULL for p_A = 0 everywhere; when given, mu_vx, mu_vy, var_v (measured velocity and its
 * variance, > 0) define the spatial likelihood g(z|x) = N(v; mu, var I) and the associated
 * new-born velocity pdf, and must be non-NULL.
 * Velocity evidence is switched off in this version: a non-NULL p_assoc makes dogm_update,
 * dogm_step, dogm_step_noalloc and dogm_step_batch return DOGM_ENOTIMPL before anything is enqueued (the text
 * from dogm_status_string / dogm_last_error says so).
 * For a grid of DOGM_MODEL_PHD_MIB (Sec. V.C observation process) p_tp, p_fp and det are
 * required instead of m_occ, m_free (which are not read) and p_assoc must be NULL: p_tp, p_fp
 * are the true and false positive probabilities of the cell in [0, 1] (equal where the cell is
 * not observed, which then keeps its prediction), det is 1 where a measurement occurred and 0
 * elsewhere.  DOGM_EINVAL otherwise. */
typedef struct dogm_meas {
    const float* m_occ;
    const float* m_free;
    const float* p_assoc;
    const float* mu_vx;
    const float* mu_vy;
    const float* var_v;
    const float* p_tp;
    const float* p_fp;
    const float* det;
} dogm_meas;

/* Device pointers to every array of a grid (all inside the arena).  The arrays typed float
 * below hold double when the grid's precision is DOGM_PRECISION_FP64 (cast the pointer). */
typedef struct dogm_views {
    /* persistent particles at the start of a cycle / after resampling (nu each) */
    float *x, *y, *vx, *vy, *w;
    uint32_t* key;        /* cell key written by predict, in the order of x..w (nu)          */
    /* particles sorted by cell (after assign; update rewrites w) (nu each) */
    float *sx, *sy, *svx, *svy, *sw;
    uint32_t* skey;       /* sorted keys (nu)                                               */
    uint32_t* perm;       /* sorted position -> index in x..w (nu)                          */
    /* cells (C each unless noted) */
    uint32_t *cell_start, *cell_end; /* particle range [start, end) of each cell in sorted
                                         order (after assign); empty cells: start == end */
    double* sum_w;        /* sum of predicted persistent weights (FP64; 0 for empty cells) */
    float *m_pO, *m_pF;   /* predicted BBA                                                  */
    float *m_O, *m_F;     /* posterior BBA; m_F is also the state carried to the next cycle  */
    float *rho_b, *rho_p; /* new-born / persistent part of m_O                              */
    float* pign;          /* pignistic occupancy probability                                */
    double *mu_A, *mu_UA; /* normalisation components of the persistent update               */
    uint32_t* born_off;   /* new-born slot range [born_off[c], born_off[c+1]) (C+1)          */
    float *mean_x, *mean_y, *var_x, *var_y, *cov_xy; /* velocity moments                     */
    uint8_t* mom_flag;    /* 1 where the moments are defined (rho_p > 0 and particles)       */
    /* new-born particles of the last update (nu_b each) */
    float *bx, *by, *bvx, *bvy, *bw;
    uint32_t* bkey;
    uint8_t* bassoc;      /* 1 for associated new-born particles                            */
    /* device scalars */
    uint32_t* status;     /* DOGM_ST_* bits, sticky                                          */
    uint32_t* cycle;      /* cycle counter used by the random streams                        */
    uint64_t* W_fixed;    /* joint posterior weight of the last resampling, units 2^-40      */
    uint64_t* S_fixed;    /* total new-born mass of the last update, units 2^-40            */
    int64_t n_pers, n_born, n_cells;
} dogm_views;

/* Bytes of device memory one grid with these parameters needs.  DOGM_EINVAL on bad params. */
int dogm_arena_bytes(const dogm_params* params, size_t* bytes);

/* Creates a grid inside `arena` (device memory, >= dogm_arena_bytes bytes, 256-byte aligned)
 * and enqueues its initial state on `stream`: nu particles uniform over the grid, velocity
 * N(0, sigma_B^2 I), weight 0; m_F = 0; status 0; cycle counter 1.  (The paper leaves the
 * initial state open.)  *out receives the handle.  DOGM_EINVAL / DOGM_ESIZE / DOGM_EHIP. */
int dogm_init_grid(const dogm_params* params, void* arena, size_t arena_bytes,
                   dogm_stream_t stream, dogm_grid** out);

/* Frees the host handle (the arena stays the caller's).  Waits for nothing. */
int dogm_destroy(dogm_grid* grid);

/* Changes the stream later calls enqueue on. */
int dogm_set_stream(dogm_grid* grid, dogm_stream_t stream);

/* Sets the cycle counter (device and host copy, enqueued on the grid's stream) and makes
 * predict the next valid call.  For tests and for replaying a cycle from saved state. */
int dogm_set_cycle(dogm_grid* grid, uint32_t cycle);

/* Host copy of the cycle counter. */
int dogm_get_cycle(const dogm_grid* grid, uint32_t* cycle);

/* Device pointers of every array (valid for the lifetime of the grid). */
int dogm_view(const dogm_grid* grid, dogm_views* views);

/* Alg. 1, eqs. (process) and (particle_persistence): in place on x..w, per particle
 * x' = x + T vx + sigma_pos n1, y' = y + T vy + sigma_pos n2, vx' = vx + sigma_vel n3,
 * vy' = vy + sigma_vel n4, w' = p_S w, with standard normals from Philox counter
 * (index, cycle, 1, grid_id); writes the cell key (C and w' = 0 outside the grid). */
int dogm_predict(dogm_grid* grid);

/* Alg. 2: stable sort of the particles by cell key into sx..sw / skey / perm, and the
 * particle range of every cell (cell_start, cell_end; empty cells have start == end).  The same
 * pass over the sorted particles also forms the per-cell sums the update reads (sum of weights
 * and, for Alg. 6, of the weighted velocities), which do not depend on the measurement. */
int dogm_assign(dogm_grid* grid);

/* Alg. 3, 4 and 5 in the paper's order:
 *  - per cell: m_p(O) = min(sum w, 1), m_p(F) = min(alpha m_F, 1 - m_p(O)),
 *    (m_O, m_F) = m_p (+) m_z (Dempster), rho_b / rho_p split of eq. (DS_resulting_masses1/2)
 *    (new-born mass only where m_z(O) > 0);
 *  - persistent weights: w <- p_A mu_A g w + (1 - p_A) mu_UA w, eq. (DSnormalization);
 *  - new-born particles: nu_b slots allocated in proportion to rho_b, split into associated /
 *    unassociated sets, uniform position in the cell, velocity from p(x|z) or N(0, sigma_B^2),
 *    weights of eqs. (weights_associated), (weights_unassociated).
 * Without velocity evidence (p_assoc NULL) the updated weights are mu_UA w, so the update
 * also writes the velocity moments of Alg. 6.
 * `meas` is a host struct of device pointers (see dogm_meas).  DOGM_EINVAL if m_occ/m_free is
 * NULL or p_assoc is given without mu_vx/mu_vy/var_v. */
int dogm_update(dogm_grid* grid, const dogm_meas* meas);

/* Alg. 6, eqs. (mean_x), (var_x), (covar_xy): velocity mean, variance and covariance of the
 * updated persistent particles of every cell, normalised by rho_p; zeros and mom_flag 0
 * where rho_p <= 0 or the cell holds no particle.  Launches work only for a grid whose last
 * update had velocity evidence (otherwise the update already wrote the moments); the call is
 * still required in the order of a cycle.  It reads no measurement array: the buffers passed
 * to the last dogm_update may be released once that call's work has completed. */
int dogm_moments(dogm_grid* grid);

/* Alg. 7, eq. (resampledParticleWeights): systematic resampling of nu particles from the joint
 * set [sorted persistent | new-born] into x..w, every weight W/nu with W the joint weight;
 * draws u_j = (j + U) W / nu with U from Philox counter (0, cycle, 3, grid_id).  With W = 0
 * the sorted persistent set is kept.  Advances the device cycle counter (cycle + 1). */
int dogm_resample(dogm_grid* grid);

/* predict, assign, update, moments, resample in order (one full cycle). */
int dogm_step(dogm_grid* grid, const dogm_meas* meas);

/* For callers that cannot allocate device memory or take an allocating code path (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the cycle of
 * dogm_step, bit-identical to it, with the per-cycle scratch (digit histograms and their
 * totals, partial sums of new-born masses and joint weights, first-slot marks, tile starts)
 * and a private copy of the grid descriptor in a static device array of 16 MiB instead of the
 * grid's arena.  The inputs and outputs stay the caller's: the grid's arena and `meas`.  The
 * call allocates nothing (no hipMalloc or hipFree, no allocating library routine).  Each
 * device holds one such array until the process ends, found at dogm_init_grid (or at the
 * first call on a device) with that device current, and shared by every call on that device:
 * calls that overlap in time on one device race and must be ordered by the caller (one
 * stream, or events).  Nothing in the array needs clearing: every part is rewritten within
 * the cycle before it is read.  DOGM_ESIZE, before anything is enqueued, if the grid's scratch
 * exceeds the array (about 2 bytes per persistent particle plus 4 per new-born slot: e.g.
 * nu = 2^22 with nu_b = 2^19 fits, nu = 2^23 does not); otherwise as dogm_step. */
int dogm_step_noalloc(dogm_grid* grid, const dogm_meas* meas);

/* One full cycle of n independent grids, each kernel launched once for all of them (grids of
 * different sizes share every launch).  All grids must have completed the same phase (ready
 * for predict); all work is enqueued on `stream`.  meas[i] belongs to grids[i].  The result of
 * every grid is bit-identical to dogm_step on that grid alone. */
int dogm_step_batch(dogm_grid* const* grids, const dogm_meas* meas, int n,
                    dogm_stream_t stream);

/* The synthetic sensor ahead of the recursion.  The filter takes one measurement grid per
 * cycle as its input (Sec. VII); these two calls generate it on the device from a scene, so a
 * closed loop of scene, sensor and filter needs no host work per cycle.  Both only enqueue on
 * `stream`; every pointer is device memory owned by the caller; cells are row-major.
 *
 * dogm_sensor_truth: occ[c] = 1 where the centre ((ix + 1/2) r, (iy + 1/2) r) of cell c lies in
 * one of the n_rects axis-aligned rectangles rects[4i .. 4i+3] = (x0, y0, x1, y1) (bounds
 * included; boxes and walls) or where static_occ[c] != 0 (optional, e.g. clutter), else 0.
 * DOGM_EINVAL for a bad size, a NULL occ or rects with n_rects > 0, or cell_size <= 0. */
int dogm_sensor_truth(const double* rects, int32_t n_rects, const uint8_t* static_occ,
                      int32_t nx, int32_t ny, double cell_size, uint8_t* occ,
                      dogm_stream_t stream);

/* dogm_sensor_scan: the cells a sensor at the grid centre (nx/2, ny/2 in cell units) observes,
 * and the evidence masses of one cycle.  One Amanatides-Woo traversal (FP64) per perimeter
 * cell towards that cell's centre marks seen[c] = 1 in every cell it passes up to and
 * including the first cell with occ != 0 (or the perimeter cell); every other cell gets 0.
 * The i-th cell boundary crossed along an axis lies at ray parameter t_0 + i d (d = 1 / |the
 * direction's component|, one rounded product and one rounded sum), and a step crosses an x
 * boundary only when its parameter is strictly below the next y boundary's.  In
 * each observed cell one Bernoulli draw (Philox4x32-10, key `seed`, counter (c, cycle, 4, 0),
 * uniform as in the filter) detects with probability p_d if occupied and p_cl if free; a
 * detection gives (m_occ, m_free) = (2 P - 1, 0) with P = p_d / (p_d + p_cl), an observed cell
 * without one (0, 1 - 2 Q) with Q = (1 - p_d) / ((1 - p_d) + (1 - p_cl)) (the masses whose
 * pignistic transform is the Bayesian occupancy with prior 1/2), an unobserved cell (0, 0).
 * m_occ and m_free may both be NULL (ray cast only).  DOGM_EINVAL for a bad size or pointer,
 * probabilities outside [0, 1] or p_d < p_cl (negative evidence). */
int dogm_sensor_scan(const uint8_t* occ, int32_t nx, int32_t ny, double p_d, double p_cl,
                     uint64_t seed, uint32_t cycle, uint8_t* seen, float* m_occ, float* m_free,
                     dogm_stream_t stream);

/* Per-kernel timing on the device clock.  While a trace is active, every launch of the kernel
 * named `kernel` (every kernel if NULL) that the calling thread enqueues through this library
 * is bracketed by two of the caller's HIP events (hipEvent_t, created with timing enabled),
 * recorded on that launch's stream: events[2i] before and events[2i+1] after the i-th traced
 * launch, for the first `capacity` launches; names[i] (if names is not NULL) receives the
 * kernel's name, static storage.  The events, the arrays and the `kernel` string are the
 * caller's and must stay valid until dogm_trace_end, which returns the number of traced
 * launches in *count.  A trace is per thread; DOGM_EINVAL on a negative capacity or NULL
 * events with capacity > 0, DOGM_ESTATE from dogm_trace_end without an active trace,
 * DOGM_EHIP from dogm_trace_end if recording one of the events failed (the count is still
 * written; the trace ends either way). */
int dogm_trace_begin(void* const* events, const char** names, int capacity, const char* kernel);
int dogm_trace_end(int* count);

/* Text of a status code, or of the last DOGM_EHIP error of the calling thread. */
const char* dogm_status_string(int code);
const char* dogm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DOGM_H */
