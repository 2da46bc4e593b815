/*
 * shsph.h -- C ABI of the MI355X (gfx950) SPH hot path: on-the-fly Morton /
 * radix tree, two-stage neighbour cache, smoothing-length iteration and the
 * SPH force / energy equations, after Shamrock (arXiv 2503.09713).
 *
 * Conventions (every entry point):
 *   - Returns SHSPH_OK (0) or a negative SHSPH_E* code; nothing throws.
 *     shsph_last_error() gives a message for the last failure on a context.
 *   - Particle arrays are DEVICE pointers owned by the caller, structure of
 *     arrays, one element per particle, element type given by `dtype`
 *     (float or double).  They are borrowed only for the duration of the
 *     work enqueued by the call.
 *   - Work is enqueued on the context's stream (shsph_set_stream).  A call
 *     may synchronise that stream to read small counters (leaf count,
 *     neighbour-cache sizes, the h-iteration outcome); results in caller
 *     arrays are complete when the call returns.
 *   - Indices into the neighbour cache and the tree are positions in Morton
 *     (key) order; the permutation `eps` (sorted slot i <- input index
 *     eps[i]) maps them back to the caller's order.
 *   - Calls on one context are serialised by a lock inside the context; the
 *     serving loop (shsph_serve_start) is one more user of that lock.  The
 *     plain calls (build / density / force / step) keep their tree and
 *     caches in the context only until the next call that builds one,
 *     pooled passes included.
 */
#ifndef SHSPH_H
#define SHSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHSPH_OK 0
#define SHSPH_EINVAL (-1)     /* null pointer, size, dtype or box error, h <= 0 */
#define SHSPH_ENOMEM (-2)     /* device allocation failed */
#define SHSPH_ENOCONV (-3)    /* h iteration did not converge in max_iter; h is the last iterate */
#define SHSPH_ECAPACITY (-4)  /* traversal stack or cache capacity exceeded */
#define SHSPH_EHIP (-5)       /* HIP runtime failure */
#define SHSPH_ESTATE (-6)     /* calls out of order (e.g. density before build_tree) */

typedef enum { SHSPH_F32 = 0, SHSPH_F64 = 1 } shsph_dtype;

typedef struct shsph_ctx shsph_ctx;

/* Method parameters.  Defaults (shsph_params_default) follow the paper:
 *   hfact = 1.2 for the M4 kernel and rho(h) = m (hfact/h)^3 (App. F, Eq. rhoh);
 *   chi = 1.1 ghost/cache tolerance and lambda = 1.2 Newton clamp (App. F);
 *   alpha_av = 1, beta_av = 2 artificial viscosity, beta_u = 1 conductivity
 *   (Sect. 2.1 and Sect. 4.2); c_cour = 0.3, c_force = 0.25 (App. G.2);
 *   gamma = 5/3 adiabatic EOS; eps_h = 1e-6 Newton tolerance (the paper
 *   leaves it open), max_iter = 50; n_red = 3 reduction passes (App. C.2). */
typedef struct {
    double hfact;
    double gamma;
    double alpha_av;
    double beta_av;
    double beta_u;
    double chi;
    double lambda;
    double eps_h;
    double c_cour;
    double c_force;
    int32_t max_iter;
    int32_t n_red;
    int32_t max_restarts;   /* cache rebuilds allowed when h exceeds chi h (default 8) */
    int32_t spread_slots;   /* serial stage-1 walk only: a group whose union, gathered
                               with the group's box, passes this many particles is
                               gathered again leaf by leaf (default 8192; 1 = always) */
    int32_t stage1_serial;  /* 1: stage 1 by the serial per-group walk for every group
                               (default 0: one wave per group, serial walk only for
                               groups that outgrow its buffers).  Work, not results. */
    int32_t stage2_mode;    /* stage-2 walk: 1 = per lane (default), 2 = per wave (all
                               lanes take the wave's joint candidates; pays off when h is
                               large against the wave's extent), 0 = chosen per wave by
                               its estimated cost.  Work, not results. */
    int32_t kernel;         /* smoothing kernel f (Sect. 2.1.1), SHSPH_KERNEL_*: support
                               radius R h; the cache radius is R chi h.  Default M4.
                               The paper's physics tests use M6 with hfact = 1.0. */
    int32_t key_bits;       /* Morton code width (App. B.1, Sect. 5.2.1): 63 = 21 bits per
                               axis in a 64-bit code (default), 30 = 10 bits per axis in
                               a 32-bit code (faster tree build, coarser cells) */
    double eps_v;           /* corrector re-run tolerance (App. G.1): after the
                               corrector, if max |dv| > eps_v times the rms velocity the
                               force is evaluated again with v* <- v^{n+1} and the
                               corrector re-applied; 0 (default) = never */
    int32_t max_reruns;     /* corrector re-runs allowed per step (default 3) */
    int32_t alpha_switch;   /* 1: per-particle viscosity alpha evolved by the shock
                               detector (App. G, Shock detection) in shsph_step, read
                               from and written to shsph_particles.alpha; 0 (default):
                               the constant alpha_av */
    double lambda_stiff;    /* CFL multiplier stiffness (App. G, CFL multiplier): the
                               multiplier halves after a re-run and relaxes as
                               (1 + s l) / (1 + s) otherwise (default 1; only with
                               eps_v > 0 and a CFL dt) */
    double alpha_min, alpha_max;  /* bounds of the switch (0, 1) */
    double sigma_decay;     /* decay time tau = h / (sigma_decay c_s) (0.1) */
    int32_t force_split;    /* threads per particle in the force kernel: 1 (workgroups
                               of 256 threads) or 2 (512; default), each summing its
                               share of the particle's list, combined in a fixed
                               order.  Work, not results (the sums' rounding order
                               follows the split).  Chosen by shsph_autotune. */
    int32_t fused_density_force;  /* 1: the h iteration and the force run in one
                               persistent cooperative launch (as many workgroups as
                               the device holds, the grid synchronised between the
                               two; one thread per particle in the force), falling
                               back to the separate kernels when a cache rebuild is
                               needed, the alpha switch is on, or the launch is not
                               possible.  Same results as force_split = 1.
                               Default 0; shsph_autotune may choose it. */
    int32_t graph_batch;    /* 1 (default): a batched pass (shsph_step_batch,
                               shsph_eval_batch, the serving loop) whose shape
                               repeats the previous pass's (particle and group
                               counts, instance boundary types, parameters,
                               buffers) is recorded once as a hipGraph and
                               replayed, with no host read until the pass ends;
                               a pass that needs a capacity regrow, a cache
                               rebuild or a fallback is switched off on the
                               device and run again launch by launch.  Same
                               results, bit for bit.  Not used while profiling.
                               0: every pass launch by launch. */
} shsph_params;

#define SHSPH_KERNEL_M4 0
#define SHSPH_KERNEL_M5 1
#define SHSPH_KERNEL_M6 2
#define SHSPH_KERNEL_C2 3
#define SHSPH_KERNEL_C4 4
#define SHSPH_KERNEL_C6 5

/* One SPH instance.  x..h are read; h, rho, omega, ax..dudt are written as
 * documented per call.  `pid` (optional) is a per-particle id carried
 * through the reordering of shsph_step.  Equal-mass particles (mass).
 * periodic = 1: box [lo, hi) with minimum-image separations (requires
 * 2.2 max(h) < (hi-lo)/2 on every axis); periodic = 0: isolated, the box is
 * the data extent (lo/hi are ignored). */
typedef struct {
    int64_t n;
    int32_t dtype;          /* shsph_dtype */
    int32_t periodic;
    double mass;
    double lo[3];
    double hi[3];
    void *x, *y, *z;        /* positions */
    void *vx, *vy, *vz;     /* velocities */
    void *u;                /* specific internal energy */
    void *h;                /* smoothing length */
    void *ax, *ay, *az;     /* dv/dt */
    void *dudt;             /* du/dt */
    void *rho, *omega;      /* optional outputs */
    uint32_t *pid;          /* optional */
    void *alpha;            /* per-particle viscosity alpha (optional): read by the
                               force and, with params.alpha_switch, evolved by
                               shsph_step; NULL = the constant alpha_av */
} shsph_particles;

/* Counters of the last build / evaluation / step. */
typedef struct {
    int64_t n;
    int64_t n_leaf;          /* leaves after dedupe + reduction */
    int64_t n_groups;        /* groups of 256 key-order particles */
    int64_t n_leaf_neigh;    /* stage-1 cache entries (group -> leaves) */
    int64_t n_neigh;         /* stage-2 cache entries (particle -> particles) */
    int32_t n_red;
    int32_t restarts;        /* cache rebuilds caused by h > chi h_cache */
    int32_t max_iter_seen;   /* largest Newton iteration count of any particle */
    int32_t n_noconv;        /* particles that did not converge */
    double dt_cfl;           /* CFL dt from the last force evaluation */
    double dv_max;           /* max |dv| of the last corrector */
    double dv2_sum;          /* sum |dv|^2 */
    double v2_sum;           /* sum |v^{n+1}|^2 */
    int32_t reruns;          /* corrector re-runs of the last step (App. G.1) */
    int32_t cache_capacity;  /* neighbour-cache entries per particle the context holds
                                room for (grows when a build needs more) */
    double cfl_multiplier;   /* CFL multiplier for the next CFL step (App. G) */
    int64_t graph_passes;    /* batched passes run from a captured graph (context total) */
    int64_t graph_aborts;    /* captured passes switched off and run launch by launch */
    int32_t graph_abort_why; /* why the last one was: bit 0 a capacity / stack / box-record
                                overflow of the build (its flag word in bits 8-15: 1 stack,
                                2 union leaves, 4 ELL words, 16 box records, 32 layout),
                                1 a sort look-back overrun, 2 the leaf pass's fallback,
                                3 a periodic box below twice the cache radius, 4 the
                                same flags in a cache-rebuild round (bits 16-23), 5 an h
                                still past chi h_cache after the rebuild rounds */
    int32_t pad1;
} shsph_info;

/* Host buffers receiving the tree of the last build (test and debug use).
 * Any pointer may be NULL.  Sizes: n = particles, L = n_leaf, I = L - 1,
 * NN = 2L - 1, G = n_groups, E1 = n_leaf_neigh, E2 = n_neigh.  Node arrays
 * are indexed by node: internal nodes 0..I-1, then leaves I..NN-1.  The
 * first stage of the cache is kept per group of 256 consecutive key-order
 * particles (group g = slots [256 g, 256 g + 256)); the second stage is
 * returned in the plain offsets + list form of Alg. 5.  T = the dtype. */
typedef struct {
    uint64_t *keys;      /* n   Morton keys in the caller's order (App. B.1) */
    uint32_t *eps;       /* n   sort permutation: key slot i <- input eps[i] */
    uint64_t *mu;        /* n   sorted keys */
    uint8_t *xi;         /* n   keep mask after reduction (App. C, Alg. 1) */
    uint32_t *id;        /* L+1 first key slot of each leaf, id[L] = n */
    uint64_t *mu_leaf;   /* L   leaf codes */
    uint32_t *lchild, *rchild, *endrange;  /* I  Karras tables (App. B.7) */
    uint8_t *lflag, *rflag;                /* I */
    uint32_t *parent;    /* NN  (root: 0xffffffff) */
    void *bmin;          /* 3*NN T  tight box lower corner */
    void *bmax;          /* 3*NN T  tight box upper corner */
    void *hmax;          /* NN  T   max h of the cell */
    uint32_t *pbox;      /* 6*NN  integer prefix box X0 Y0 Z0 X1 Y1 Z1 (App. B.6) */
    int32_t *plen;       /* NN    prefix length of the box */
    uint64_t *group_off;    /* G+1  stage-1 offsets, G = n_groups */
    uint32_t *group_leaves; /* E1   neighbour leaves of each group (ascending) */
    uint64_t *neigh_off; /* n+1  stage-2 offsets (Alg. 5) */
    uint32_t *neigh_list;/* E2   neighbours in key slots (ascending, self included) */
    void *h_sorted;      /* n T  h in key order (after a density call: converged h) */
    void *h_cache;       /* n T  h the neighbour cache was built with (key order): the
                            step-start h, or the h of the last cache rebuild */
} shsph_tree_export;

/* Fill *p with the defaults listed above. */
void shsph_params_default(shsph_params *p);

/* Create a context on HIP device `device` (parameters copied; NULL = defaults).
 * EINVAL for a bad device or parameter, EHIP on runtime failure. */
int shsph_create(int device, const shsph_params *p, shsph_ctx **out);

/* Release the context and all its device memory (waits for its stream). */
int shsph_destroy(shsph_ctx *ctx);

/* Replace the context's parameters (checked as at create; not while
 * serving).  Later calls use them; the tree and caches of an earlier build
 * stay valid only if kernel, chi, n_red and key_bits are unchanged.
 * EINVAL for a parameter out of range, ESTATE while serving. */
int shsph_set_params(shsph_ctx *ctx, const shsph_params *p);

/* Copy the context's current parameters into *out. */
int shsph_get_params(shsph_ctx *ctx, shsph_params *out);

/* Use `stream` (a hipStream_t, NULL = the null stream) for all later work. */
int shsph_set_stream(shsph_ctx *ctx, void *stream);

/* Message of the last failure on this context ("" if none).  Valid until the
 * next call on the context. */
const char *shsph_last_error(const shsph_ctx *ctx);

/* The tree half of the hot path, on the particles as given (App. B-E):
 * Morton keys (App. B.1) -> stable radix sort -> keep mask + n_red reduction
 * passes (App. C, Alg. 1) -> compaction -> Karras radix tree (App. B.7) ->
 * bottom-up tight cell boxes with h_max -> two-stage neighbour cache with the
 * chi-extended object-object criterion (App. D.4, Alg. 5, App. E).
 * Reads x, y, z, h.  The tree and caches stay in the context until the next
 * build or step.  EINVAL on bad input, ECAPACITY if the traversal stack
 * overflows. */
int shsph_build_tree(shsph_ctx *ctx, const shsph_particles *p);

/* Smoothing length and density (App. F, Alg. 7; Sect. 2.1 Eq. sphomega): h and
 * rho = m (hfact/h)^3 by per-particle Newton iteration over the cache, with
 * cache rebuilds when h leaves chi times its cache h; then Omega.  Needs a
 * build on the same particles.  Writes h (in place), rho and omega (if
 * non-NULL) in the caller's order.  Reads u (if non-NULL) for the pressure
 * used by a following shsph_force.  ENOCONV if some particle did not
 * converge (its h is the last iterate). */
int shsph_density(shsph_ctx *ctx, shsph_particles *p);

/* Derivatives (Sect. 2.1 Eqs. sphvel, sphuint, with artificial viscosity and
 * conductivity): writes ax, ay, az, dudt in the caller's order from the h,
 * rho, Omega of the preceding shsph_density and the caller's v and u.  Also
 * reduces the CFL dt (App. G.2), readable with shsph_get_info.  ESTATE if no
 * density result is held. */
int shsph_force(shsph_ctx *ctx, shsph_particles *p);

/* The whole hot path: one kick-drift-kick step (App. G.1) of dt (dt <= 0: the CFL
 * dt of the previous force evaluation).  Reads the state at t^n and
 * ax..dudt = derivatives at t^n; writes the state at t^{n+1} with its
 * derivatives, h, and rho/omega/pid when non-NULL.  The particles come back
 * REORDERED into the new Morton order (all arrays consistently).  dt_used
 * (optional) receives the dt taken.  Errors as for the calls above. */
int shsph_step(shsph_ctx *ctx, shsph_particles *p, double dt, double *dt_used);

/* shsph_step without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as shsph_step, bit for
 * bit.  All device working memory of the call (keys, tree, caches, sorted
 * fields, reductions) comes from one static array per device of 128 MiB,
 * held by that device from the library's first use until the process ends;
 * its address is taken once per device by shsph_create.  Nothing is
 * allocated or freed by the call (it makes no hipMalloc, hipFree or
 * allocating library call); it waits for its stream before returning.
 * Limits: n <= 131072 particles (ECAPACITY beyond, with nothing enqueued);
 * a step whose neighbour caches outgrow the array (far more than ~100
 * neighbours per particle) also fails with ECAPACITY.  The array is shared
 * by every call on its device and keeps the last call's contents: calls
 * that overlap on one device (other contexts, other threads, other streams)
 * race and must be serialised by the caller.  A CFL step (dt <= 0) takes
 * the CFL dt of this context's previous shsph_step_noalloc (kept on the
 * host, so other users of the array in between do not disturb it);
 * ESTATE if there is none.  State of shsph_build_tree / _density / _force /
 * _step on the same context is neither used nor changed. */
int shsph_step_noalloc(shsph_ctx *ctx, shsph_particles *p, double dt, double *dt_used);

/* Counters of the last build / density / force / step. */
int shsph_get_info(shsph_ctx *ctx, shsph_info *out);

/* Copy the tree of the last build to host buffers (see shsph_tree_export). */
int shsph_export_tree(shsph_ctx *ctx, const shsph_tree_export *out);

/* Optional per-stage timing: with `on`, every stage of the calls above is
 * bracketed by HIP events on the context's stream and the calls wait for
 * them at their end.  Turning it on (or off) clears the totals. */
#define SHSPH_NUM_STAGES 12
int shsph_set_profiling(shsph_ctx *ctx, int on);

/* Totals since profiling was turned on: ms[i] = summed event time of stage i,
 * launches[i] = how many times it ran (arrays of n <= SHSPH_NUM_STAGES). */
int shsph_get_stage_times(shsph_ctx *ctx, double *ms, int64_t *launches, int32_t n);

/* Name of stage i ("" when out of range); static storage. */
const char *shsph_stage_name(int32_t i);

/* Work counted by the neighbour kernels while profiling is on (totals since
 * it was turned on), 6 doubles: particle cache {candidate pair tests, leaf
 * box prune tests}, density {pair evaluations summed over Newton passes,
 * force {cache entries visited, interacting pairs}; density's second entry
 * counts the evaluations within 2h. */
int shsph_get_work(shsph_ctx *ctx, double *out6);

/* ------------------------------------------------------------------------
 * Pooled instances and batched passes.
 *
 * Many independent instances (uneven sizes, periodic or isolated, one dtype
 * per context) live in a device pool owned by the context.  A batched pass
 * runs every stage of the step once over all the instances it names: the
 * sort is segmented by instance, each instance gets its own tree, cache,
 * h iteration, reductions and CFL dt, and each result is the same as the
 * instance would get alone (the kernels never mix instances).  The pooled
 * state is kept in Morton order after each pass; `pid` maps it back.
 * ---------------------------------------------------------------------- */

/* Copy an instance into the pool: reads x..h, vx..u (required) and ax..dudt,
 * rho, omega, pid when non-NULL (zeros, and pid = 0..n-1, otherwise).  The
 * pointers may be device or host memory; the call waits for the copy.
 * *handle receives a positive id.  EINVAL on bad input or a dtype other
 * than the pool's, ENOMEM when the pool cannot grow. */
int shsph_instance_create(shsph_ctx *ctx, const shsph_particles *init, int64_t *handle);

/* Return the instance's range to the pool.  ESTATE while a serving job
 * holds it. */
int shsph_instance_destroy(shsph_ctx *ctx, int64_t handle);

/* Copy the instance's current state (Morton order) into the non-NULL
 * arrays of `out` (device or host memory; out->n and out->dtype must match);
 * waits for the copy. */
int shsph_instance_read(shsph_ctx *ctx, int64_t handle, const shsph_particles *out);

/* The instance's reductions from its last pass: n, dt_cfl, dv_max, dv2_sum,
 * v2_sum, max_iter_seen, n_noconv (tree counters are 0). */
int shsph_instance_info(shsph_ctx *ctx, int64_t handle, shsph_info *out);

/* One kick-drift-kick step (App. G.1) of every listed instance in a single
 * batched pass; dt[k] > 0 is a fixed step, dt[k] <= 0 (or dt NULL) the
 * instance's CFL dt (App. G.2).  A CFL instance that has no derivatives yet
 * first gets a derivative pass (as shsph_eval_batch).  dt_used (optional)
 * receives the dt taken per instance.  1..2048 distinct handles.  ENOCONV
 * when some instance's h iteration did not settle: the step is complete,
 * shsph_instance_info tells which. */
int shsph_step_batch(shsph_ctx *ctx, const int64_t *handles, int32_t count, const double *dt,
                     double *dt_used);

/* Derivatives at the current state of every listed instance in one batched
 * pass: h (Newton iteration, App. F), rho, Omega, a, du/dt and the CFL dt;
 * positions, velocities and u are unchanged (values; the order becomes the
 * new Morton order). */
int shsph_eval_batch(shsph_ctx *ctx, const int64_t *handles, int32_t count);

/* Autotuner for batched passes: times evaluation passes of the listed
 * instances (as shsph_eval_batch: positions, velocities and u unchanged) for
 * leaf sizes n_red = 2, 3, 4, stage-2 walks 0, 1, 2 and three shapes of the
 * derivative kernels: the fused persistent density + force launch, or
 * separate launches with force workgroups of 256 or 512 threads
 * (force_split 1, 2), and keeps the fastest in the context's parameters for
 * later passes.  The leaf size and the walk change no result; the force
 * split changes only the rounding order of the force sums.  Outputs
 * (optional): the chosen n_red, walk and force shape (0 = fused, else the
 * force split), and the pass time in ms. */
int shsph_autotune(shsph_ctx *ctx, const int64_t *handles, int32_t count, int32_t *n_red,
                   int32_t *stage2_mode, int32_t *force_split, double *pass_ms);

/* Pool occupancy: particles held by instances, pool capacity, instances. */
int shsph_pool_usage(shsph_ctx *ctx, int64_t *particles_used, int64_t *particles_cap,
                     int64_t *n_instances);

/* ------------------------------------------------------------------------
 * Serving: a request loop on a host thread of the context.
 *
 * Jobs (advance an instance by nsteps steps, or evaluate its derivatives)
 * are queued in arrival order.  A job is admitted when the HBM it needs fits
 * the budget (its instance, if the job brings one, plus the working memory
 * of its particles while it runs) and the pass has room; admitted jobs run
 * together: every pass is one batched pass over all running jobs, and jobs
 * join and leave at pass boundaries (continuous batching).  The
 * one-at-a-time policy runs the same queue with a single job on the device.
 * ---------------------------------------------------------------------- */
#define SHSPH_SERVE_CONTINUOUS 0
#define SHSPH_SERVE_ONE_AT_A_TIME 1

#define SHSPH_JOB_STEP 0
#define SHSPH_JOB_EVAL 1

#define SHSPH_JOB_PENDING 0
#define SHSPH_JOB_RUNNING 1
#define SHSPH_JOB_DONE 2
#define SHSPH_JOB_FAILED 3

typedef struct {
    double budget_bytes;          /* HBM for resident instances + running work */
    int64_t max_batch_particles;  /* particles in one pass (0: no limit) */
    int32_t max_batch;            /* jobs in one pass (1..2048) */
    int32_t policy;               /* SHSPH_SERVE_* */
} shsph_serve_config;

typedef struct {
    int64_t handle;               /* pooled instance to work on, or 0 with init */
    const shsph_particles *init;  /* if non-NULL: the job's instance is created from
                                     these arrays when the job is admitted; the struct
                                     is copied at submit, the arrays must stay valid
                                     until the job has left PENDING */
    int32_t kind;                 /* SHSPH_JOB_STEP or SHSPH_JOB_EVAL */
    int32_t nsteps;               /* STEP: steps to take (>= 1) */
    double dt;                    /* STEP: > 0 fixed dt, <= 0 CFL dt */
    int32_t release;              /* 1: destroy the instance when the job ends */
    int32_t reserved;
} shsph_job;

typedef struct {
    int32_t state;                /* SHSPH_JOB_* */
    int32_t error;                /* SHSPH_E* when FAILED */
    int64_t handle;               /* the job's instance (0 before admission) */
    int32_t steps_done;
    int32_t passes;               /* batched passes the job took part in */
    double t_submit, t_start, t_done;   /* shsph_clock() seconds */
} shsph_job_status;

typedef struct {
    int64_t jobs_done;
    int64_t jobs_failed;
    int64_t passes;
    int64_t peak_jobs;            /* most jobs in one pass */
    double particle_passes;       /* sum over passes of the particles in them */
    double busy_s;                /* time inside passes */
    double peak_bytes;            /* largest accounted footprint */
} shsph_serve_counters;

/* Start the loop.  EINVAL for a bad config, ESTATE if already serving. */
int shsph_serve_start(shsph_ctx *ctx, const shsph_serve_config *cfg);

/* Queue a job; *ticket identifies it.  ENOMEM if the job can never fit the
 * budget, EINVAL for a bad job (unknown handle, nsteps < 1, dtype other
 * than the pool's), ESTATE if not serving. */
int shsph_submit(shsph_ctx *ctx, const shsph_job *job, uint64_t *ticket);

/* Status of a job (does not wait).  EINVAL for an unknown ticket. */
int shsph_poll(shsph_ctx *ctx, uint64_t ticket, shsph_job_status *st);

/* Wait until no job is pending or running, at most timeout_s seconds
 * (ESTATE on time-out). */
int shsph_serve_drain(shsph_ctx *ctx, double timeout_s);

/* Counters of the loop since it started. */
int shsph_serve_stats(shsph_ctx *ctx, shsph_serve_counters *out);

/* Finish pending and running jobs, then stop the loop (shsph_destroy calls it). */
int shsph_serve_stop(shsph_ctx *ctx);

/* HBM the admission rule charges for an instance of n particles of the
 * context's dtype: pooled state, and the working memory while it runs. */
int shsph_footprint(shsph_ctx *ctx, int64_t n, int32_t dtype, double *state_bytes,
                    double *work_bytes);

/* Seconds on the steady clock used for job timestamps. */
double shsph_clock(void);

#ifdef __cplusplus
}
#endif
#endif /* SHSPH_H */
