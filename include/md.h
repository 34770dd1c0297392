/*
 * md.h -- C ABI of the MI355X slice-streaming Lennard-Jones library (libmd.so).
 *
 * Method: "Cyclic Data Streaming on GPUs for Short Range Stencils Applied to
 * Molecular Dynamics" (arXiv 2507.11289).  The data set is cut into x-slices
 * (Sec. 3, slice requirements), each slice is processed with the two
 * neighbouring slices as input and output (input/output order 1, Sec. 4), and
 * time advances slice by slice (Sec. 3.1, data flow; Table 1).  On one GPU all
 * slices stay resident in HBM and a persistent kernel advances slice i from step
 * t to t+1 once slices i-1 and i+1 have reached step t.  The per-slice work is
 * the truncated-and-shifted Lennard-Jones force from cell lists, the
 * velocity-Verlet update of Algorithm 1 and the migration of atoms to the
 * neighbouring slices (Sec. 4.1, kernels md_v3a / md_v3aa / md_v3b).
 *
 * Conventions for every function:
 *   - return MD_OK (0) or a negative md_status; nothing throws or aborts across
 *     the ABI; md_last_error() gives a thread-local message for the last failure;
 *   - every input array is host memory and is copied before the call returns;
 *   - every output array is caller-owned host memory of the stated size;
 *   - device memory and the HIP stream are owned by the library (a stream may be
 *     lent with md_set_stream);
 *   - arrays of 3-vectors are n x 3 row-major doubles (x, y, z per atom), in
 *     atom-id order, where the id of an atom is its index in md_load's arrays;
 *   - reduced LJ units: sigma = epsilon = m = k_B = 1.
 * One md_sim is not thread-safe; an md_server is safe for concurrent
 * md_submit / md_poll.
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_sim md_sim;       /* opaque, library-owned */
typedef struct md_server md_server; /* opaque, library-owned */

enum md_status {
    MD_OK = 0,
    MD_PENDING = 1,      /* md_poll: run not finished yet */
    MD_EINVAL = -1,      /* invalid argument */
    MD_ENOMEM = -2,      /* device or host allocation failed / run can never fit */
    MD_EHIP = -3,        /* HIP runtime error, or no usable GPU */
    MD_ESTATE = -4,      /* call out of order (e.g. md_step before md_load) or poisoned */
    MD_ECAPACITY = -5,   /* a cell ran out of slots (atoms too crowded) */
    MD_EUNSTABLE = -6,   /* non-finite value, or an atom crossed more than one slice */
    MD_ENOTFOUND = -7,   /* unknown server ticket */
    MD_EBUSY = -8,       /* server queue full: MD_SERVER_MAX_QUEUED runs wait for admission */
    MD_EWATCHDOG = -9    /* a device-side wait exceeded its time budget */
};

enum md_precision {
    MD_FP64 = 0,         /* everything in FP64 (the paper's precision, Sec. 4) */
    MD_FP32_FORCE = 1    /* pair forces in FP32 on cell-relative coordinates; positions,
                            velocities, integrator and energy sums in FP64; cutoff
                            decisions identical to the FP64 ones */
};

/* md_set_option keys */
enum md_option {
    MD_OPT_ENERGY_EVERY = 1,    /* sample U, K, W at steps t with t % k == 0 (0 = never); default 0 */
    MD_OPT_CLAIM_ORDER = 2,     /* md_claim_order (default MD_ORDER_DATAFLOW); results are
                                   bitwise identical for every order */
    MD_OPT_ORDER_SEED = 3,      /* seed of MD_ORDER_RANDOM */
    MD_OPT_MIGRATION_LOG = 4,   /* 1: record per-step, per-slice migration counts */
    MD_OPT_CHUNK_CELLS = 5,     /* cells per work item (0 = automatic: about 2200 atoms per item
                                   in FP32-force mode, 1900 in FP64, at least 32 cells) */
    MD_OPT_COUNT_PAIRS = 6,     /* 1: count candidates and in-range partners (slower) */
    MD_OPT_WATCHDOG_MS = 7,     /* device wait budget in ms (default 20000) */
    MD_OPT_GRID = 8,            /* persistent workgroups (0 = occupancy x CUs) */
    MD_OPT_FAIL_AT_STEP = 9,    /* debug: raise MD_EUNSTABLE when step k is reached (-1 = off) */
    MD_OPT_MAX_STEPS_PER_LAUNCH = 10, /* split md_step into launches of at most k steps */
    MD_OPT_TRACE = 11,          /* 1: record one md_trace_rec per work item of the next md_step */
    MD_OPT_CELL_CAPACITY = 12,  /* atoms a cell may hold, 1..64 (default 64): a load or step that
                                   puts more atoms in a cell fails with MD_ECAPACITY (forces the
                                   capacity guard in tests) */
    MD_OPT_WAVEFRONT_LEVELS = 14, /* time levels W of MD_ORDER_WAVEFRONT, 1..64 (default 4); md_step
                                   launches whole multiples of W steps (a shorter remainder runs
                                   as its own launch) */
    MD_OPT_XCD_QUEUES = 13      /* 1: under MD_ORDER_DATAFLOW, one work queue per XCD of the GPU,
                                   each owning a contiguous range of slices balanced by atoms (and
                                   cells) per slice, so that the items of a slice share one L2 and
                                   items whose neighbouring slices are on the same XCD end without
                                   writing the L2 back; 0 (default): one queue for the device,
                                   which balances better (the 4,194,304-atom fluid runs 6% faster).
                                   Used with at least 3 slices per XCD; results are bitwise the
                                   same */
};

enum md_claim_order {
    MD_ORDER_SWEEP = 0,       /* slices claimed in ascending order, each finalised as soon as
                                 its neighbours are integrated (the stage order of Table 1) */
    MD_ORDER_PHASED = 1,      /* all force/integrate items of a step, then all finalise items */
    MD_ORDER_DESCENDING = 2,  /* the sweep mirrored */
    MD_ORDER_RANDOM = 3,      /* a seeded random order that respects the dependencies */
    MD_ORDER_DATAFLOW = 4,    /* items are queued the moment their inputs are complete and
                                 taken in queue order (no worker waits on a dependency) */
    MD_ORDER_WAVEFRONT = 5    /* multi-time-level sweep (the one-GPU analogue of several workers
                                 per GPU at different time levels, Sec. 3.1 and Eq. (1)): items of
                                 MD_OPT_WAVEFRONT_LEVELS consecutive steps are dealt as two
                                 wavefronts running from slice 0 towards slice S/2 in both
                                 directions, each later step three slices behind the one before,
                                 so that W time levels are in flight in a window of about 6W
                                 slices (md_wavefront_table) */
};

typedef struct md_stats {
    int64_t step;              /* current step t of the synchronous state */
    int64_t n;                 /* atoms */
    int32_t slices;            /* x-slices S */
    int32_t ncx;               /* cell layers per slice */
    int32_t grid[3];           /* cells per axis (grid[0] = S * ncx) */
    int32_t cell_capacity;     /* atom slots per cell */
    int64_t ncell;             /* cells in total */
    int64_t migrations_left;   /* atoms moved to the left neighbour slice since md_load */
    int64_t migrations_right;  /* atoms moved to the right neighbour slice since md_load */
    int64_t candidates;        /* with MD_OPT_COUNT_PAIRS: sum over atom-steps of the
                                  27-cell candidates (self excluded) in the last md_step */
    int64_t in_range;          /* ... and of partners with r^2 <= rc^2 */
    int64_t counted_steps;     /* atom-steps behind candidates / in_range */
    double last_step_seconds;  /* wall time of the last md_step (host clock) */
    double last_kernel_seconds; /* device time of its persistent launches (HIP events on the
                                  launch stream) */
    int32_t last_launches;     /* persistent launches of the last md_step */
    int32_t persistent_grid;   /* workgroups of the last persistent launch */
    int32_t chunks_per_slice;  /* force work items per slice and step (finalise items: a
                                  quarter as many, rounded up, under the dataflow scheduler) */
    int32_t precision;         /* md_precision */
    int32_t poisoned;          /* 1 after a failed md_step */
    int32_t work_queues;       /* work queues of the last md_step: one per XCD, or 1
                                  (MD_OPT_XCD_QUEUES) */
    int32_t queue_first[9];    /* first slice of each work queue's range; queue_first[work_queues] = S */
} md_stats;

/* Create a simulation of a periodic box box[0] x box[1] x box[2], cut into `slices`
 * x-slices (Sec. 3: slices perpendicular to the longest axis; Sec. 4: cells of
 * edge > rc, neighbours within one cell).  Each slice holds ncx = floor((Lx/S)/rc)
 * cell layers; y and z hold floor(L/rc) cells; a count whose cell edge would be
 * within a relative 2^-40 of rc drops by one.  dt is the velocity-Verlet step.
 * MD_EINVAL when: slices < 3, Lx/slices < rc, fewer than 3 cells in y or z,
 * rc <= 0, dt <= 0, any value non-finite, or an unknown precision. */
int md_init(const double box[3], int slices, double rc, double dt, int precision,
            md_sim **out);

/* Load n atoms (positions in [0, L] per axis, velocities), replacing any state;
 * the step counter restarts at 0.  Atoms are binned into slices and cells on the
 * device (Sec. 4: MolList / CellList per slice).  MD_EINVAL for non-finite values
 * or positions outside [0, L]; MD_ECAPACITY when a cell would exceed its slots. */
int md_load(md_sim *s, int64_t n, const double *pos, const double *vel);

/* Advance nsteps velocity-Verlet steps (Algorithm 1) in one or more persistent
 * launches, without host round trips inside a launch.  Blocking.  On a guard trip
 * returns MD_EUNSTABLE / MD_ECAPACITY / MD_EWATCHDOG and poisons the handle
 * (afterwards only md_get_stats, md_get_cells-free calls and md_free are valid). */
int md_step(md_sim *s, int64_t nsteps);

/* Bytes of the launch scratch md_step_noalloc uses on each GPU (16 MiB). */
#define MD_NOALLOC_SCRATCH_BYTES 16777216

/* md_step for callers that cannot allocate device memory (harnesses that forbid
 * hipMalloc, serving loops that must not allocate, code that will later be captured):
 * the same kernels as md_step and bitwise the same results, but the per-launch buffers
 * (run arguments, work queue, energy partials of the sampled steps, migration log) are
 * carved out of one fixed array of MD_NOALLOC_SCRATCH_BYTES per GPU that the library
 * holds until the process ends, instead of device memory allocated on first use.  It
 * calls no hipMalloc, hipFree or caller allocator (md_set_allocator); the state buffers
 * come from md_init / md_load.  nsteps is split into launches of at most
 * MD_OPT_MAX_STEPS_PER_LAUNCH steps whose pieces fit the scratch.
 * All calls on one GPU share that GPU's array and it keeps the last launch's contents
 * (every piece is rewritten or cleared before a launch reads it): calls that overlap in
 * time on one GPU, from several threads or on several streams, race and must not be made.
 * MD_EINVAL when one step of the system needs more than the scratch (the message gives
 * both sizes; e.g. more than about 2 million work items per step), when the thermostat
 * is on (md_set_thermostat) or when MD_OPT_TRACE is set (both need allocated buffers);
 * otherwise as md_step (errors poison the handle).  md_get_stats reports no kernel time
 * for these launches. */
int md_step_noalloc(md_sim *s, int64_t nsteps);

/* Potential energy U (pair energies shifted to vanish at rc), kinetic energy K and
 * virial W = sum over pairs of r_ij . f_ij at the current step (Algorithm 1: the
 * U and V accumulations), summed in FP64 in a fixed order. */
int md_energy_virial(md_sim *s, double *U, double *K, double *W);

/* The synchronous state at the current step in id order: positions, velocities
 * v(t) and forces F(t) (each n x 3; any pointer may be NULL). */
int md_get_state(md_sim *s, double *pos, double *vel, double *force);

/* Global cell id of every atom (n int64 in id order): slice * cells_per_slice +
 * ((gx mod ncx) * Gy + gy) * Gz + gz, with g_d = clamp(floor(x_d * (1/l_d))). */
int md_get_cells(md_sim *s, int64_t *cell);

/* Atoms per slice at the current step (S int64). */
int md_get_slice_counts(md_sim *s, int64_t *counts);

/* Energy samples of the last md_step: rows of (t, U, K, W); *count = rows written. */
int md_get_energy_log(md_sim *s, int64_t cap_rows, double *rows, int64_t *count);

/* Migration log of the last md_step (MD_OPT_MIGRATION_LOG): [steps][S][2] counts of
 * atoms leaving slice s to the left (0) and to the right (1) in each step. */
int md_get_migration_log(md_sim *s, int64_t cap_steps, int32_t *log, int64_t *steps);

/* One work item of a persistent launch (MD_OPT_TRACE): which item, on which compute
 * unit, and when (device wall clock ticks) it was claimed, found its inputs ready,
 * and finished.  phase 0 = force/integrate of step k (force only with the thermostat),
 * 1 = finalise of step k+1, 2 = thermostat integrate of step k. */
typedef struct md_trace_rec {
    uint32_t k, slice, chunk, phase;
    uint32_t hw_id;            /* hardware id register of the wave that ran it */
    uint32_t launch;           /* index of the persistent launch within md_step */
    uint32_t xcd;              /* XCD (L2 domain) that ran it */
    uint32_t queue;            /* work queue it was taken from (MD_OPT_XCD_QUEUES) */
    uint64_t t_claim, t_ready, t_done;
} md_trace_rec;

/* Trace of the last md_step; *count = records available; ticks per second in *hz. */
int md_get_trace(md_sim *s, int64_t cap, md_trace_rec *out, int64_t *count, double *hz);

int md_get_stats(md_sim *s, md_stats *out);
int md_set_option(md_sim *s, int key, int64_t value);

/* Velocity-scaling thermostat (Sec. 4: kernels md_thermo_a/md_thermo_b compute a scale
 * factor from the new velocities and md_v3b applies it before the positions advance;
 * Sec. 4.2 simulates the canonical ensemble with it).  With temperature T0 > 0 every
 * later step starts by scaling the velocities v(t) of the atoms of each slice i by
 *     lambda_i = sqrt(3 n_i T0 / (2 K_i)),   K_i = sum over the slice of |v(t)|^2 / 2,
 * (lambda_i = 1 when the slice holds no atoms or no kinetic energy), so that the
 * slice's kinetic temperature 2 K / (3 n) becomes T0; the factor of a slice depends
 * only on that slice.  T0 = 0 switches it off (NVE).  Energy samples and md_get_state
 * report the unscaled v(t).  Each step then runs as a force pass over the slice, then
 * an integrate pass once the whole slice's K is known (24 B of forces per atom kept in
 * between; device memory is allocated at the next md_step).  Requires the default
 * MD_ORDER_DATAFLOW scheduler: md_step returns MD_EINVAL under another claim order.
 * Errors: MD_EINVAL for a NULL handle or a negative or non-finite temperature. */
int md_set_thermostat(md_sim *s, double temperature);

/* Use a caller-owned hipStream_t (passed as void*) for every later launch and copy;
 * NULL returns to the library's own stream. */
int md_set_stream(md_sim *s, void *hip_stream);

void md_free(md_sim *s);
const char *md_strerror(int status);
const char *md_last_error(void);

/* The per-step claim table a persistent launch deals items from (claim orders other than
 * MD_ORDER_DATAFLOW): 2 * slices entries (phase << 15) | slice, phase 0 = force and
 * integration of step t, phase 1 = finalisation of step t+1.  MD_ORDER_SWEEP follows the
 * stage order of Table 1: after slice k is integrated, slice k-1 is complete.  Host-only. */
int md_claim_table(int slices, int order, uint64_t seed, uint16_t *out);

/* The claim table of MD_ORDER_WAVEFRONT for `levels` consecutive steps: 2 * slices * levels
 * entries (j << 16) | (phase << 15) | slice, j = step within the group of levels.  Integrate
 * (phase 0) of slice i at step j has key 6j + 2d(i) and finalise (phase 1) of slice i for
 * step j+1 has key 6j + 2 max(d(i-1), d(i), d(i+1)) + 1, with d(i) = min(i, S - i) the
 * distance from slice 0 on the ring; entries are sorted by key, then phase, then slice.
 * Because d changes by at most one between neighbours, every entry follows the entries it
 * depends on.  Host-only.  MD_EINVAL for slices < 3, levels outside 1..64 or NULL. */
int md_wavefront_table(int slices, int levels, uint32_t *out);

/* Device bytes a served run of this system holds at most (the admission measure): two
 * cell buffers of 4352 B per cell, cell and slice counters, the larger of the load copies
 * and the read-back outputs (72 B per atom), the read-back energy partials, and the launch
 * scratch of one 64-step packed launch with the served work items, a quarter of a slice
 * of 32 to 64 cells each (work queue, energy partials, migration log).  -1 for an invalid
 * geometry. */
int64_t md_footprint_bytes(const double box[3], int slices, double rc, int64_t n);

/* Device memory allocator used for every later device allocation of the library (NULL,
 * NULL: hipMalloc / hipFree, the default).  alloc(bytes, ctx) returns device memory of
 * the current device aligned to at least 256 bytes, or NULL (MD_ENOMEM); release(ptr,
 * ctx) gives it back once the library has synchronised every stream that used it, e.g.
 * torch's caching allocator.  Both are called from the thread that calls into the
 * library, or from an md_server's own thread.  MD_ESTATE while any md_sim or md_server
 * exists; MD_EINVAL when only one of the two functions is given. */
typedef void *(*md_alloc_fn)(size_t bytes, void *ctx);
typedef void (*md_free_fn)(void *ptr, void *ctx);
int md_set_allocator(md_alloc_fn alloc, md_free_fn release, void *ctx);

/* ---------------------------------------------------------------------------
 * Serving: independent runs arrive at any time, are admitted first-come
 * first-served while their device footprint fits the byte budget and a slot is
 * free, stay resident on the device, and advance together: their slices are packed
 * into the same bounded persistent launches (one launch per quantum of steps).
 * Results of a run do not depend on what else is in the mix.
 * --------------------------------------------------------------------------- */
typedef struct md_run_desc {
    double box[3];
    int32_t slices;
    double rc, dt;
    int32_t precision;
    int64_t n;
    const double *pos, *vel;   /* copied by md_submit */
    int64_t steps;
    int64_t energy_every;      /* sample interval (0: only t = 0 and t = steps) */
    uint64_t tag;              /* caller's label, returned in md_result */
    int32_t keep_state;        /* 1: keep the final state for md_fetch_state (the library
                                  never writes into caller memory after md_submit returns;
                                  the caller copies the state out when it wants it) */
} md_run_desc;

typedef struct md_result {
    int32_t status;            /* MD_OK or the run's own error */
    int64_t steps_done;
    uint64_t tag;
    double U0, K0, W0;         /* at t = 0 */
    double U1, K1, W1;         /* at t = steps */
    double drift_per_atom_step; /* least-squares slope of (U+K)/n against t over the samples */
    double t_submit, t_admit, t_done; /* seconds on the server's clock */
} md_result;

/* Runs that may wait for admission at once; md_submit returns MD_EBUSY beyond. */
#define MD_SERVER_MAX_QUEUED 4096

enum md_server_flags {
    MD_SERVER_FAKE_EXECUTOR = 1  /* no GPU: runs complete after a simulated time (tests) */
};

/* budget: device bytes runs may occupy; max_runs: resident runs at most;
 * quantum_steps: steps per packed launch (0 = automatic). */
int md_server_create(size_t hbm_budget_bytes, int max_runs, md_server **out);
int md_server_create_ex(size_t hbm_budget_bytes, int max_runs, int quantum_steps, int flags,
                        md_server **out);
/* Copy the run and queue it; *ticket identifies it.  MD_EINVAL for an invalid run,
 * MD_ENOMEM when its footprint (md_footprint_bytes with the server's quantum) exceeds
 * the whole budget, MD_EBUSY when MD_SERVER_MAX_QUEUED runs already wait. */
int md_submit(md_server *sv, const md_run_desc *run, uint64_t *ticket);
/* MD_PENDING while queued or running; MD_OK when done (result filled); the run's
 * own error code if it failed (result filled).  A finished ticket is released by
 * the first md_poll that reports it, unless the run keeps its state (keep_state),
 * in which case md_fetch_state releases it. */
int md_poll(md_server *sv, uint64_t ticket, md_result *out);
/* Final positions and velocities (n x 3, id order) of a finished run submitted with
 * keep_state = 1; releases the ticket.  NULL pointers are skipped. */
int md_fetch_state(md_server *sv, uint64_t ticket, double *pos, double *vel);
int md_server_stats(md_server *sv, int64_t *queued, int64_t *running, int64_t *done,
                    int64_t *bytes_in_use, int64_t *launches);
/* Seconds the server's thread has spent admitting runs (device set-up, load, energy at
 * t = 0), in packed launches (set-up, kernels, per-run bookkeeping), completing runs (energy
 * at t = steps, final state, release) and waiting for work.  NULL pointers are skipped. */
int md_server_times(md_server *sv, double *admit_s, double *launch_s, double *finish_s, double *idle_s);
int md_server_destroy(md_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
