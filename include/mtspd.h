/*
 * mtspd -- multi-time-step coupling of bond-based peridynamics (PD) and finite
 * elements (FE) in the Arlequin framework, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Zhong, Han, Du, Guo, "Multi-time-step coupling of peridynamics and
 * classical continuum mechanics for dynamic brittle fracture", arXiv 2403.03605.
 * The PD subdomain is advanced m times per FE step (Sec. 2.5, Algorithm 1):
 * neighbour lists (Sec. 2.1), pairwise force (Eq. 2), stretch (Eq. 3),
 * irreversible bond breaking (Eq. 4), damage (Eq. 5), velocity Verlet
 * (Newmark gamma = 1/2, beta = 0, Eq. 38).  Around it: the explicit
 * lumped-mass FE step (Eq. 24-34) and the velocity-continuity multipliers of
 * the free/link split (Eq. 47-50).
 *
 * Conventions of this interface
 *  - Plain C types only.  Host pointers are named `host_*`, device pointers
 *    `dev_*`.  The library never keeps a caller pointer after a call returns.
 *  - Every call returns an mts_status; on failure mts_last_error() (per host
 *    thread) describes it.  No C++ exception or abort crosses the interface.
 *  - Node order of every per-node array is the order of `pd_pos` as given.
 *    Vectors are node-major: value (node i, component c) at [i * dim + c].
 *  - All work is enqueued on the HIP stream given at create; calls that return
 *    host data synchronise that stream.
 *  - One solver must not be used from two host threads at once.
 */
#ifndef MTSPD_H
#define MTSPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mts_status {
  MTS_OK = 0,
  MTS_EINVAL = 1,    /* invalid argument or problem description */
  MTS_ENOMEM = 2,    /* device or host allocation failed */
  MTS_EDEVICE = 3,   /* a HIP call failed */
  MTS_EUNSTABLE = 4, /* non-finite state detected at a macro-step boundary (sticky) */
  MTS_EAGAIN = 5,    /* pool: request does not fit now; resubmit later */
  MTS_ETOOBIG = 6,   /* pool: request can never fit the budget */
  MTS_ESTATE = 7     /* call not valid in the current state */
} mts_status;

enum { MTS_COUPLED = 0, MTS_PURE_PD = 1 };            /* mts_problem.mode */
enum { MTS_FP64 = 0, MTS_MIXED = 1 };                 /* mts_problem.precision */
enum { MTS_W_CUBIC = 0, MTS_W_LINEAR = 1, MTS_W_CONSTANT = 2 }; /* weight_kind, Sec. 3.2 */
enum { MTS_K_PMB = 0, MTS_K_EXP = 1 };                /* micromodulus kernel */

/* Problem description (deep-copied by mts_create).
 * Geometry: PD nodes at `pd_pos` with nodal volume dx^dim (x thickness in 2D),
 * horizon delta = horizon_factor * dx.  The body is the box [dom_lo, dom_hi];
 * the FE mesh is fe_n[] square (cube) elements of side fe_h starting at dom_lo.
 * The PD box [pd_lo, pd_hi] overlaps the FE mesh over a band of width `overlap`
 * along its faces that lie inside the body (Arlequin weights, Eq. 17-18).
 * Cracks (2D): horizontal segments y = cracks[c][0], cracks[c][1] <= x <= cracks[c][2].
 * Loads: traction on the faces y = dom_lo[1] and y = dom_hi[1] (outward,
 * magnitude `traction`, Pa), prescribed x-velocity `vel_bc` on the face
 * x = dom_lo[0].  In MTS_PURE_PD mode the PD box is the body and the traction
 * becomes a body force traction/delta on nodes within delta of its y faces.
 * s_crit <= 0 derives the critical stretch from G0. */
typedef struct mts_problem {
  int32_t dim;          /* 2 (plane stress, nu = 1/3) or 3 (nu = 1/4) */
  int32_t mode;         /* MTS_COUPLED or MTS_PURE_PD */
  int32_t precision;    /* MTS_FP64 or MTS_MIXED */
  int32_t breaking;     /* 1: critical-stretch breaking on */
  int32_t weight_kind;  /* MTS_W_* */
  int32_t kernel;       /* MTS_K_* */
  int32_t m;            /* step ratio dt_FE / dt_PD, >= 1 */
  int32_t n_cracks;     /* 0..8 */
  int32_t fe_n[3];      /* elements per axis (ignored in MTS_PURE_PD) */
  int64_t n_pd;         /* number of PD nodes */
  const double *host_pd_pos; /* n_pd * dim reference positions */
  double dx, horizon_factor;
  double pd_lo[3], pd_hi[3], dom_lo[3], dom_hi[3];
  double fe_h, overlap;
  double cracks[8][3];
  double E, rho, G0, thickness, s_crit, l_over_delta;
  double traction, vel_bc;
  double dt_pd;         /* PD step (s) > 0; the FE step is m * dt_pd */
  double fe_beta;       /* Newmark beta of the FE step (gamma = 1/2): 0 explicit (lumped mass),
                           1/4 average acceleration, implicit: each FE step solves
                           (M + beta dt_FE^2 K) a = f by conjugate gradients, which lifts the
                           FE stability bound on dt_FE (Eq. 38; coupled mode, one solver, not
                           the pool) */
  double traction_x;    /* uniform traction (Pa, +x) on the FE face x = dom_hi[0], weighted by
                           alpha like the y-face traction (Eq. 34 P^FE): the end load of the
                           beam of Sec. 3.2 (coupled mode, one solver, not the pool) */
  int32_t clamp_x0;     /* 1: every displacement component of the FE nodes on the face
                           x = dom_lo[0] is held at zero (the fixed end of that beam); needs
                           vel_bc = 0 (coupled mode, one solver, not the pool) */
  double pd_beta;       /* Newmark beta of the PD step (gamma = 1/2): 0 explicit (velocity Verlet),
                           1/4 average acceleration, implicit: each step solves
                           (M + beta dt^2 K) a = P + f(u*) by conjugate gradients with the current
                           bond states, and the critical-stretch test runs on the solved
                           displacement (Eq. 38; pure-PD mode, FP64, one solver, not the pool;
                           dt_pd may exceed the explicit bound) */
} mts_problem;

typedef struct mts_info {
  double delta, volume, c0, s_crit, dt_pd, dt_fe;
  int64_t n_pd, nnz, n_fe_nodes, n_fe_elems, n_constraints, n_region;
  int64_t pd_steps, macro_steps, n_rebuilds, n_colors;
  int64_t device_bytes;  /* device memory the solver holds */
  int32_t dim, precision;
  double dt_bound_pd;    /* PD stability bound of the step (create rejects dt_pd above it) */
  int64_t inverse_bytes; /* bytes of the packed inverse of H that each multiplier solve
                            (Eq. 49) reads: the kept 64 x 64 lower tiles of every component
                            block, 32 KiB each in FP64 or 16 KiB for tiles whose entries are
                            all at most 2^-29 of the component's largest (stored in FP32);
                            0 in pure-PD mode */
  double slot_bytes;     /* bytes of slot record the bond pass reads per bond slot: 12 (FP64
                            coefficient and neighbour offset), 8 (mixed), 6 (mixed with
                            neighbour records staged in LDS: two slots per 12-byte record) */
  int64_t n_rebuild_columns; /* unit-load columns (constraint nodes) recomputed by the rebuilds
                                after setup: a rebuild recomputes only the constraints whose
                                response support holds a node with a changed bond (Algorithm 1,
                                update of Y); the others are unchanged bit for bit */
} mts_info;

/* Energies of the current state (J, per unit thickness in 2D) and the bonds
 * broken since setup (pre-crack cuts excluded). */
typedef struct mts_energy_info {
  double kinetic;        /* 1/2 v^T M v, weighted PD and FE masses (Eq. 17-18) */
  double strain_pd;      /* 1/4 sum_i sum_k mu w c (xi.eta)^2 V_i V_k (Eq. 6-7) */
  double strain_fe;      /* 1/2 u^T K u, alpha-weighted FE stiffness (Eq. 34) */
  double external_work;  /* P . u of the constant loads */
  int64_t n_broken;
} mts_energy_info;

typedef struct mts_plan_info {
  int64_t n_pd, nnz_estimate, n_fe_nodes, n_constraints_estimate;
  int64_t device_bytes_estimate; /* upper estimate of what mts_create allocates, temporaries included */
} mts_plan_info;

/* Quantities for mts_read / mts_write (vectors node-major, dim per node). */
enum {
  MTS_PD_U = 0, MTS_PD_V, MTS_PD_A, MTS_FE_U, MTS_FE_V, MTS_FE_A,
  MTS_DAMAGE,       /* PD nodal damage phi (Eq. 5), n_pd values */
  MTS_LAMBDA,       /* multipliers lambda (n_constraints * dim) */
  MTS_PD_ALPHA,     /* Arlequin weight at PD nodes */
  MTS_PD_MASS, MTS_FE_MASS, MTS_FE_X,
  MTS_CONSTRAINT_NODES, /* PD node ids of the constraint set, as doubles */
  MTS_H             /* multiplier matrix H of Eq. 49 at the last (re)build, row-major;
                       kept only when n_constraints * dim <= 4096 */
};

/* Kernels that mts_kernel_time reports. */
enum {
  MTS_KT_PD_SUBSTEP = 0, MTS_KT_LINK = 1, MTS_KT_FE = 2, MTS_KT_LAMBDA = 3,
  MTS_KT_REBUILD = 4, /* rebuilds of the unit-load responses, H and its inverse (Algorithm 1,
                         update of Y): stream time from the rebuild's first to its last
                         work, host waits inside it included */
  MTS_KT_COUNT = 5
};

typedef struct mts_solver mts_solver;

/* Host-only estimate of sizes and device bytes for a problem (no device use).
 * Errors: MTS_EINVAL for an inconsistent description. */
mts_status mts_plan(const mts_problem *p, mts_plan_info *out);

/* Build a solver on the current HIP device: neighbour lists (Sec. 2.1) built on
 * the device, Arlequin weights and masses (Eq. 17-18, 34), FE mesh, the
 * constraint set, the unit-load responses and the multiplier matrix (eq. unit,
 * Eq. 49), all enqueued on `hip_stream` (a hipStream_t, or NULL for the null
 * stream).  The solver owns its device memory.  On error *out stays NULL.
 * Errors: MTS_EINVAL (bad description: dim, m < 1, dt_pd <= 0 or above the PD
 * stability bound (mts_info.dt_bound_pd), horizon_factor < 1,
 * n_pd <= 0, a crack line off the FE node lines, a constraint node in an element
 * with no weight), MTS_ENOMEM, MTS_EDEVICE. */
mts_status mts_create(const mts_problem *p, void *hip_stream, mts_solver **out);

/* mts_create with all of the solver's device memory carved out of a
 * caller-owned region (for instance a torch uint8 tensor): dev_arena (256-byte
 * aligned) .. dev_arena + arena_bytes must stay valid until mts_destroy, and
 * the library never frees it.  mts_plan's device_bytes_estimate is enough;
 * a region that turns out too small fails with MTS_ENOMEM (also later, if a
 * rebuild of the unit-load responses needs more scratch than is left).
 * dev_arena = NULL behaves as mts_create.  Other errors as mts_create. */
mts_status mts_create_in(const mts_problem *p, void *dev_arena, int64_t arena_bytes, void *hip_stream,
                         mts_solver **out);

/* Enqueue n_macro macro steps (one FE step and m PD substeps each,
 * Algorithm 1).  Returns after enqueueing the last macro step; it may wait on
 * the device between macro steps while bonds inside the support of the
 * unit-load responses break (the responses are then rebuilt, Algorithm 1).
 * Errors: MTS_EUNSTABLE (sticky) once a non-finite value was seen, MTS_EDEVICE. */
mts_status mts_advance(mts_solver *s, int64_t n_macro);

/* Wait for all enqueued work and surface sticky errors. */
mts_status mts_sync(mts_solver *s);

/* Copy a quantity to host memory (synchronous).  `cap` is the capacity of
 * host_out in doubles; *n receives the count.  MTS_EINVAL if cap is too small
 * or the quantity does not exist in this mode. */
mts_status mts_read(mts_solver *s, int32_t what, double *host_out, int64_t cap, int64_t *n);

/* The same quantity, written into device memory (for instance a torch
 * tensor's storage) on the solver's stream: asynchronous, ordered after the
 * work enqueued before it; the caller synchronizes that stream (mts_sync)
 * before reading dev_out elsewhere.  Same layout, counts and errors as
 * mts_read (MTS_H needs a problem small enough for H to be kept); dev_out
 * stays owned by the caller. */
mts_status mts_read_device(mts_solver *s, int32_t what, double *dev_out, int64_t cap, int64_t *n);

/* Overwrite MTS_PD_U/V/A, MTS_FE_U/V/A or MTS_LAMBDA from host memory
 * (synchronous; n must equal the quantity's size). */
mts_status mts_write(mts_solver *s, int32_t what, const double *host_in, int64_t n);

/* Bond lists in canonical CSR (rows ascending) and the bond states
 * (1 intact, 0 broken or cut by a crack).  cap = capacity of col/intact.
 * row_ptr must hold n_pd + 1 entries.  Any pointer may be NULL. */
mts_status mts_read_bonds(mts_solver *s, int64_t *host_row_ptr, int32_t *host_col,
                          uint8_t *host_intact, int64_t cap, int64_t *nnz);

mts_status mts_query(mts_solver *s, mts_info *out);

/* Energies and broken bonds of the state after the work enqueued so far
 * (synchronous: waits for the solver's stream).  Each term is summed in a
 * fixed order, so repeated calls give identical values. */
mts_status mts_energy(mts_solver *s, mts_energy_info *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the values
 * of mts_energy, enqueued on the solver's stream without allocating anything
 * and without waiting.  dev_out (caller-owned device memory, 5 doubles)
 * receives kinetic, strain_pd, strain_fe, external_work and n_broken (as a
 * double), in that order, once the stream reaches the call; the values equal
 * mts_energy's bit for bit.  The partial sums live in one static device buffer
 * per GPU of 65,504 doubles (512 KiB, held by every GPU the library runs on
 * until the process ends), enough for about 5.5 million PD nodes; a larger
 * solver gets MTS_EINVAL.  Calls on one GPU share that buffer: calls whose
 * work overlaps on the device (solvers on different streams of one GPU, with
 * no ordering between them) race, so order them (one stream, or events).
 * Errors: MTS_EINVAL (NULL argument, solver too large), MTS_EDEVICE. */
mts_status mts_energy_noalloc(mts_solver *s, double *dev_out);

/* HIP-event timing on the solver's stream while enabled.  MTS_KT_PD_SUBSTEP:
 * one event pair brackets the m back-to-back substep launches of a macro step
 * and *launches counts the substeps; the other groups count one launch group
 * (FE free step, multiplier solve, link re-run) per macro step, or one per
 * rebuild (MTS_KT_REBUILD). */
mts_status mts_profile(mts_solver *s, int32_t enable);
mts_status mts_kernel_time(mts_solver *s, int32_t kernel, int64_t *launches, double *total_ms);

/* Frees everything the solver owns.  Accepts NULL. */
void mts_destroy(mts_solver *s);

const char *mts_status_str(mts_status st);
const char *mts_last_error(void);

/* ---------------------------------------------------------------------------
 * Serving pool: independent solves of one dimension and precision resident in
 * device memory together, admitted against a byte budget and advanced together
 * (continuous batching).  One pool step advances every running request by one
 * macro step of Algorithm 1; the PD substeps of all requests run as one batched
 * launch per substep index, and the per-step work is replayed from HIP graphs
 * while the set of running requests does not change.  A request's results equal
 * those of the same request running alone in a pool (same lane count, same
 * arithmetic order).
 * Threads: mts_pool_submit may run on other threads (several at once)
 * concurrently with the other pool calls (each call builds its request on a
 * stream of its own); all other pool calls must come from one thread.
 * ------------------------------------------------------------------------- */
enum { MTS_REQ_ACTIVE = 1, MTS_REQ_DONE = 2 };

typedef struct mts_pool mts_pool;

typedef struct mts_pool_info {
  int64_t budget_bytes, used_bytes;  /* device bytes charged to running and unreleased requests */
  int64_t ticks, graph_captures, graph_replays;
  int32_t n_running, n_ready, max_slots, lanes;
} mts_pool_info;

/* budget_bytes: device bytes the pool may hold (requests are charged their
 * mts_plan estimate while being built, then what they actually allocated);
 * max_slots: most requests admitted at once; dim, precision: of every request;
 * use_graphs: replay pool steps from HIP graphs; hip_stream: the stream pool
 * steps run on (caller-owned; NULL: the pool creates a non-blocking stream of
 * its own -- graphs cannot be captured on the null stream).
 * Errors: MTS_EINVAL, MTS_EDEVICE. */
mts_status mts_pool_create(int64_t budget_bytes, int32_t max_slots, int32_t dim, int32_t precision,
                           int32_t use_graphs, void *hip_stream, mts_pool **out);

/* Build a request (synchronous; may run concurrently with mts_pool_step and
 * with other submits on other threads) that will run n_macro macro steps; it joins the running set at
 * the next pool step.  *id identifies it.  Errors: MTS_EAGAIN (no slot or not
 * enough budget now: submit again after a release), MTS_ETOOBIG (the estimate
 * exceeds the whole budget), MTS_EINVAL (bad description, or dim/precision
 * differ from the pool's), MTS_ENOMEM, MTS_EDEVICE. */
mts_status mts_pool_submit(mts_pool *pool, const mts_problem *p, int64_t n_macro, uint64_t *id);

/* Enqueue one pool step.  *n_active: requests still running afterwards;
 * host_done_ids[0 .. min(*n_done, cap)): requests whose last step this was
 * (their results can be read once the stream reaches that point; the read
 * calls wait for it). */
mts_status mts_pool_step(mts_pool *pool, int32_t *n_active, uint64_t *host_done_ids, int32_t cap,
                         int32_t *n_done);

/* State (MTS_REQ_ACTIVE or MTS_REQ_DONE), macro steps enqueued and, when info
 * is not NULL, the request's mts_query record.  Any output may be NULL. */
mts_status mts_pool_poll(mts_pool *pool, uint64_t id, int32_t *state, int64_t *macro_done, mts_info *info);

/* mts_read for a finished request (waits for its last step only).
 * MTS_ESTATE if it has not finished. */
mts_status mts_pool_read(mts_pool *pool, uint64_t id, int32_t what, double *host_out, int64_t cap, int64_t *n);

/* Free a finished request's device memory and return its budget. */
mts_status mts_pool_release(mts_pool *pool, uint64_t id);

mts_status mts_pool_query(mts_pool *pool, mts_pool_info *out);

/* Waits for the pool stream, frees every request.  Accepts NULL. */
void mts_pool_destroy(mts_pool *pool);

#ifdef __cplusplus
}
#endif
#endif /* MTSPD_H */
