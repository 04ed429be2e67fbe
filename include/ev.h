/*
 * libev - evaluation of prefix-linear GP trees on one AMD Instinct MI355X
 * (gfx950).  C ABI: plain pointers and sizes only.
 *
 * Method: Langdon & Banzhaf, "Faster Genetic Programming GPquick via
 * multicore and Advanced Vector Extensions" (2019).
 *
 *   Trees (Sec. 2.2): each tree is flattened into a buffer of one-byte
 *   opcodes, root first, children in order.  Tokens:
 *       EV_ADD 0, EV_SUB 1, EV_MUL 2, EV_DIV 3  functions of two arguments
 *       EV_X   4                                the input
 *       EV_C0 + i (6 + i), i < n_consts         ephemeral random constant i
 *                                               (Sec. 2.1, Table 1; see
 *                                               ev_set_constants)
 *   "op A B" is A op B; EV_DIV is protected division,
 *   (B != 0) ? A / B : 1.0f (Sec. 2.1 and the footnote of Table 1).
 *   All arithmetic is IEEE binary32, round to nearest even, subnormals
 *   kept, no contraction.
 *
 *   Fitness (Table 1, Sec. 3.2): mean over the N cases of |tree(x_i) - y_i|,
 *   the absolute errors summed in ascending case order in binary32 and the
 *   sum divided by (float)N (Sec. 2.2, last paragraph: fixed order so that
 *   every run gives identical results).  Lower is better.
 *
 *   Crossover (Sec. 3.1): one child from two parents; the child is the
 *   mum's tokens before point p, then the dad's whole subtree rooted at q,
 *   then the mum's tokens after the subtree rooted at p.
 *
 *   Selection (Table 1): tournaments choose both parents.
 *
 * Error behaviour: every call returns an ev_status; 0 is success, negative
 * values are errors, and no exception or abort crosses the ABI.
 * ev_last_error() returns a message for the calling thread's last error.
 *
 * Ownership: the library copies caller buffers during a call and keeps no
 * caller pointer after it returns, except that output pointers passed to
 * ev_submit are not used at all (results are fetched with ev_result).
 * Populations live in device memory owned by the context until ev_free_pop
 * or ev_destroy.
 *
 * Threads: a context may be used by one thread at a time, except that
 * ev_submit, ev_poll, ev_result and ev_wait may be called concurrently
 * from any threads.
 */
#ifndef EV_H
#define EV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ev_status;
typedef struct ev_ctx ev_ctx;
typedef int32_t ev_pop;
typedef uint64_t ev_ticket;

enum {
    EV_OK = 0,
    EV_EINVAL = -1,     /* bad argument or handle */
    EV_EMALFORMED = -2, /* a tree is not a valid prefix word over tokens 0..4 */
    EV_ENOMEM = -3,     /* device memory or the context's memory budget exhausted */
    EV_ECAP = -4,       /* a size limit was exceeded */
    EV_EBUSY = -5,      /* job can never fit the memory budget */
    EV_ENOTFOUND = -6,  /* unknown population or ticket */
    EV_EDEVICE = -7     /* HIP runtime error */
};

enum { EV_ADD = 0, EV_SUB = 1, EV_MUL = 2, EV_DIV = 3, EV_X = 4, EV_C0 = 6, EV_MAX_CONSTS = 250 };

/* flags */
#define EV_DEVICE_PTR 0x1u /* ev_load_trees: bytes/off are device pointers */
#define EV_OUT_DEVICE 0x2u /* ev_eval_fitness: outputs are device pointers;
                              the call returns once the work is queued on
                              the context's stream */

/* Where the context's device memory comes from.  alloc(bytes, user) returns
 * a block of device memory on the context's device, aligned to 256 bytes, or
 * NULL when it has none; free(ptr, user) takes back a block alloc returned.
 * The context keeps freed blocks for reuse (so a generation allocates
 * nothing once the sizes have been seen) and hands a block back only after
 * the work queued on its stream has finished.  Both may be called from the
 * serving workers' threads. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} ev_allocator;

/* Create a context on HIP device `device` with case table 0: x[n_cases],
 * y[n_cases] (host pointers; the paper's fitness cases are x inputs with
 * their Sextic targets y = x^6 - 2x^4 + x^2, Sec. 3 and Table 1).
 * mem_budget_bytes bounds the device memory held by populations, plans and
 * jobs (0 = all the device has free at creation, less a margin; a larger
 * value is lowered to that).  alloc, if not NULL, supplies every device block
 * the context holds (for example a framework's caching allocator); NULL uses
 * hipMalloc/hipFree.  The struct is copied.  stream is a hipStream_t to order
 * all work on, or NULL for a stream owned by the context.
 * Errors: EV_EINVAL (n_cases < 1, NULL pointers, an allocator without both
 * functions), EV_EDEVICE. */
ev_status ev_create(ev_ctx **out, int device, const float *x, const float *y, int32_t n_cases,
                    uint64_t mem_budget_bytes, const ev_allocator *alloc, void *stream);

/* Add another case table (host x[n], y[n]); *table receives its index. */
ev_status ev_add_cases(ev_ctx *ctx, const float *x, const float *y, int32_t n_cases, int32_t *table);

/* The context's ephemeral random constants (Sec. 2.1, Table 1: about 250
 * constants drawn at random from -1.000 .. +1.000, a terminal like x whose
 * value is the same on every case): token EV_C0 + i stands for consts[i],
 * i < n <= EV_MAX_CONSTS; trees holding a token EV_C0 + n or above (or 5)
 * are malformed.  Host array, copied.  Only while the context holds no
 * population and serving has not started (EV_EINVAL otherwise).  Trees with
 * constants are evaluated by the token-reading interpreter, and children in
 * a context with constants are planned from scratch. */
ev_status ev_set_constants(ev_ctx *ctx, const float *consts, int32_t n);

/* Release every population, plan, job and device buffer of the context. */
ev_status ev_destroy(ev_ctx *ctx);

/* Thread-local message for the last failing call on this thread. */
const char *ev_last_error(void);

/* Load n_trees trees.  bytes holds every tree back to back, tree t at
 * bytes[off[t], off[t+1]); off has n_trees+1 entries, off[0] = 0.  With
 * EV_DEVICE_PTR both are device pointers, else host pointers.  Every tree
 * is validated (Sec. 2.2 word: tokens 0..4 and the context's constant
 * tokens, one complete prefix tree); on
 * failure nothing is loaded, EV_EMALFORMED is returned and *bad_tree
 * (nullable) is the first bad tree.  The structure plan used by
 * ev_eval_fitness is built here.  *out_pop receives the handle. */
ev_status ev_load_trees(ev_ctx *ctx, const uint8_t *bytes, const uint64_t *off, int32_t n_trees,
                        uint32_t flags, ev_pop *out_pop, int32_t *bad_tree);

/* Number of trees and total bytes of a population. */
ev_status ev_pop_info(ev_ctx *ctx, ev_pop pop, int32_t *n_trees, uint64_t *total_bytes);

/* Copy a population to host memory: bytes (cap_bytes >= total bytes) and
 * off[n_trees+1]. */
ev_status ev_get_trees(ev_ctx *ctx, ev_pop pop, uint8_t *bytes, uint64_t *off, uint64_t cap_bytes);

ev_status ev_free_pop(ev_ctx *ctx, ev_pop pop);

/* Evaluate every tree of pop on case table `table` (Sec. 2.2, one pass
 * over each tree for all cases) and compute its fitness (Table 1).
 * fitness[n_trees] receives the MAE, per_case[n_trees * N] (nullable) the
 * tree outputs, row-major by tree, and hits[n_trees] (nullable) the number of
 * cases within 0.01 of the target (Sec. 3.2: |out - y| <= 0.01f with the
 * fitness's own binary32 error term; reported only, not used by selection).
 * Host pointers unless EV_OUT_DEVICE.  The fitness is also kept with the
 * population for ev_generation. */
ev_status ev_eval_fitness(ev_ctx *ctx, ev_pop pop, int32_t table, float *fitness, float *per_case,
                          int32_t *hits, uint32_t flags);

/* Subtree crossover (Sec. 3.1) with caller-chosen parents and points.
 * Child j = crossover(mums_pop tree mum[j] at point p[j],
 *                     dads_pop tree dad[j] at point q[j]).
 * mum, dad, p, q are host arrays of n_children entries; p[j] must be below
 * the mum's size and q[j] below the dad's.  A child larger than size_cap
 * nodes is replaced by a copy of its mum and counted in *n_capped
 * (nullable).  *out_children receives the new population (planned, ready
 * for ev_eval_fitness).  Errors: EV_EINVAL (bad index or point). */
ev_status ev_crossover(ev_ctx *ctx, ev_pop mums_pop, ev_pop dads_pop, const int32_t *mum,
                       const int32_t *dad, const uint64_t *p, const uint64_t *q, int32_t n_children,
                       uint64_t size_cap, ev_pop *out_children, int32_t *n_capped);

/* One generation (Sec. 2.3, Sec. 3.1, Table 1) on the device: for every
 * child j of the n_trees children, tournaments of size `tournament` over
 * the parents' fitness pick mum and dad (fitness: a device pointer to the
 * parents' n_trees values, complete when the call is made, or NULL for those
 * of their last ev_eval_fitness),
 * Philox4x32-10 draws keyed by (seed, gen, j) pick p and q uniformly over
 * all nodes, and the child is made by subtree crossover (size_cap as in
 * ev_crossover).  The draw layout is:
 *   key = {seed lo32, seed hi32}; ctr = {j, purpose, gen lo32, gen hi32};
 *   candidate c of role r (0 mum, 1 dad) is word c%4 of purpose
 *   ((r+1) << 8) | (c/4), mapped to [0, M) by (w * M) >> 32; the points use
 *   purpose 0x300, p from (w1:w0) and q from (w3:w2), each mapped to
 *   [0, n) by the high 64 bits of the 128-bit product; better = lower MAE,
 *   NaN worst, ties keep the earlier candidate.
 * The children are planned without waiting for the validation of their last
 * plan level: their interpreter launches check its result on the device and
 * run none of that level's codes if it failed, and their first
 * ev_eval_fitness reads it and then fails with EV_EDEVICE (an internal
 * fault: the plan builder emitted a stream it should not have). */
ev_status ev_generation(ev_ctx *ctx, ev_pop parents, const float *fitness, uint64_t seed, uint64_t gen,
                        int32_t tournament, uint64_t size_cap, ev_pop *out_children, int32_t *n_capped);

/* Sec. 2.3's generational loop: n_gen generations of ev_generation, each
 * followed by the children's evaluation on case table `table`, starting
 * from `parents` (fitness as in ev_generation: a device pointer to their
 * values, or NULL for those of their last ev_eval_fitness) at generation
 * number gen0.  Generation i uses gen0 + i in its draws, so the trees and
 * fitness values are those of the loop written out with ev_generation and
 * ev_eval_fitness, bit for bit.
 *
 * Each generation (selection, crossover, the children's split plan, their
 * evaluation and fitness) is replayed from a HIP graph captured once, with
 * no host wait inside it: buffers are sized for capacities (twice the sizes
 * last seen) and the plan is made on the device.  A generation that exceeds
 * a capacity is void and done again on the host-driven path; the graphs are
 * then captured again for new capacities.  Graphs and buffers stay with the
 * context for the next call with the same population size, case table,
 * tournament, seed, size cap and tuning (ev_destroy frees them).  With
 * EV_EVOLVE_NO_GRAPH every generation runs on the host-driven path (the
 * plain form); so does a context with ephemeral constants.
 *
 * With EV_EVOLVE_LEAN the loop keeps the population as a heap of trees
 * (Sec. 2.3's early deletion of parents, with a heap of the population's
 * own): one device arena, every tree anywhere in it.  Each generation's
 * children are made in batches, in the order of their lower parent index,
 * and a parent's bytes are reused for later children as soon as its last
 * child is made, so about 1.25 populations' worth of trees are alive at
 * once instead of 2.  The children are evaluated in place; the draws and
 * results are those of the other forms, bit for bit.  Host-driven (one wait
 * for the children's lengths per generation, then one per plan level).
 *
 * Outputs: *out the last generation as a new population (planned, its
 * fitness as of its evaluation); fit_history[n_gen * n_trees] (host,
 * nullable) each generation's children's fitness; capped_history[n_gen]
 * (host, nullable) each generation's children over size_cap; *report
 * (nullable) the counts of replayed and fallen-back generations and
 * captures, and the loop's wall time.  Errors: as ev_generation and
 * ev_eval_fitness; a graph that cannot be captured gives EV_EDEVICE. */
typedef struct {
    int32_t generations;  /* generations run */
    int32_t replayed;     /* ... replayed from a captured graph */
    int32_t fallbacks;    /* ... done again on the host-driven path (a capacity was exceeded) */
    int32_t captures;     /* graphs captured */
    uint64_t capped;      /* children over the size cap, over all generations */
    uint64_t nodes;       /* children's nodes, over all generations */
    double ms;            /* wall time of the call */
    double ms_capture;    /* of which capturing and instantiating graphs */
    /* EV_EVOLVE_LEAN: the most tree bytes alive at once in a generation, what
     * separate parent and child buffers would hold (parents + children), the
     * heap's capacity, and how often it was replaced by a larger one */
    uint64_t lean_peak_bytes, lean_two_buffer_bytes, lean_arena_bytes;
    int32_t lean_repacks, pad;
} ev_evolve_report;
#define EV_EVOLVE_NO_GRAPH 0x1u
#define EV_EVOLVE_TEST_TIGHT 0x2u /* capacities of exactly the sizes last seen: exercises the fallback */
#define EV_EVOLVE_LEAN 0x4u       /* the memory-lean loop (below) */
ev_status ev_evolve(ev_ctx *ctx, ev_pop parents, const float *fitness, int32_t table, uint64_t seed,
                    uint64_t gen0, int32_t n_gen, int32_t tournament, uint64_t size_cap, uint32_t flags,
                    ev_pop *out, float *fit_history, int32_t *capped_history, ev_evolve_report *report);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ev_eval_fitness of a population with device outputs (as with
 * EV_OUT_DEVICE) that allocates nothing.  The work counters, the plan
 * levels' intermediate result slots and the interpreter's spill slabs live
 * in a static device array of EV_STATIC_SCRATCH_BYTES, which each device
 * the library runs on holds until the process ends; the spill slabs take
 * what the result slots leave, and a level runs on as many waves as have a
 * slab there.  fitness[n_trees] (required), per_case[n_trees * N] and
 * hits[n_trees] (nullable) are device pointers; the call returns once the
 * work is queued on the context's stream and does not change the fitness
 * kept with the population.  Every call on a device shares that device's
 * array, and it keeps the last call's contents: calls on one context are
 * ordered by its stream, but calls that overlap on one device from
 * different contexts race.  Errors: EV_EINVAL (bad arguments, or a
 * population whose plan's validation verdict is still to be read: a child of
 * ev_generation not yet evaluated with ev_eval_fitness), EV_ENOTFOUND,
 * EV_ECAP (the result slots need more than the array). */
#define EV_STATIC_SCRATCH_BYTES 0x4000000u /* 64 MiB */
ev_status ev_eval_fitness_static(ev_ctx *ctx, ev_pop pop, int32_t table, float *fitness, float *per_case,
                                 int32_t *hits);

/* Statistics of a population's last ev_eval_fitness, as the paper reports
 * its runs generation by generation (Sec. 4: the columns of its result
 * tables, and its plots of size, depth and fitness convergence). */
typedef struct {
    float best_fitness;  /* least MAE (NaN is worst) */
    int32_t best_tree;   /* its index, the first of equals */
    int32_t best_hits;   /* its hits (Sec. 3.2); -1 unless that evaluation
                            returned hits to host memory */
    int32_t converged;   /* trees whose MAE equals the best's bit for bit, or
                            is NaN with a NaN best (the convergence column) */
    double mean_fitness; /* over trees with a finite MAE; NaN if none */
    uint64_t best_size, min_size, max_size; /* nodes */
    double mean_size;
    uint32_t best_depth, min_depth, max_depth; /* edges on the longest path from the root */
    uint32_t pad;
    double mean_depth;
} ev_pop_stats;

/* depth (nullable): host array of n_trees receiving every tree's depth.
 * Errors: EV_EINVAL (no evaluation yet), EV_ENOTFOUND, EV_ENOMEM. */
ev_status ev_population_stats(ev_ctx *ctx, ev_pop pop, ev_pop_stats *stats, uint32_t *depth);

/* ---- serving: continuously batched evaluation / crossover requests ---- */

enum { EV_JOB_EVAL = 0, EV_JOB_CROSSOVER = 1 };

typedef struct {
    int32_t kind;          /* EV_JOB_EVAL or EV_JOB_CROSSOVER */
    int32_t table;         /* case table for evaluation */
    /* EV_JOB_EVAL: host trees, copied during ev_submit */
    const uint8_t *bytes;
    const uint64_t *off;
    int32_t n_trees;
    /* EV_JOB_CROSSOVER: parents from a resident population; the children
     * are evaluated and their fitness returned */
    ev_pop parents;
    const int32_t *mum, *dad;
    const uint64_t *p, *q;
    int32_t n_children;
    uint64_t size_cap;
} ev_job;

/* Queue a job (thread-safe).  Inputs are copied before returning.  A job is
 * admitted to the device when its memory footprint fits the context's
 * budget beside the jobs in flight; jobs arriving while others run are
 * batched into the next device launch.  EV_EBUSY: the job can never fit;
 * EV_EINVAL / EV_EMALFORMED: bad arguments, offsets or an empty tree.  A
 * tree that is not a valid prefix tree is found on the device when its
 * batch is planned: that job alone ends with EV_EMALFORMED (ev_wait /
 * ev_result), and the jobs batched with it run again without it. */
ev_status ev_submit(ev_ctx *ctx, const ev_job *job, ev_ticket *out);

/* Non-blocking: *done = 1 once the job finished; *job_status its result. */
ev_status ev_poll(ev_ctx *ctx, ev_ticket t, int32_t *done, ev_status *job_status);

/* Block until the job finishes. */
ev_status ev_wait(ev_ctx *ctx, ev_ticket t, ev_status *job_status);

/* Copy a finished job's fitness (n entries) and, if per_case is not NULL,
 * its per-case outputs (n * N); releases the ticket.  *n_out receives n. */
ev_status ev_result(ev_ctx *ctx, ev_ticket t, float *fitness, float *per_case, int32_t cap,
                    int32_t *n_out);

/* Steady-clock nanoseconds at which the job was submitted, started on the
 * device and finished (0 while not yet reached). */
ev_status ev_job_timing(ev_ctx *ctx, ev_ticket t, uint64_t *submit_ns, uint64_t *start_ns, uint64_t *done_ns);

/* ---- introspection used by tests and the benchmark ---- */

typedef struct {
    int32_t levels;          /* levels of the split plan */
    uint64_t chunks;         /* work items over all levels */
    uint64_t slots;          /* intermediate result slots over all levels */
    uint64_t max_stack;      /* deepest operand stack of any work item */
    uint64_t plan_bytes;     /* device bytes held by the plan */
} ev_plan_info;

ev_status ev_get_plan_info(ev_ctx *ctx, ev_pop pop, ev_plan_info *info);

/* One level of the split plan.  Each tree with work at the level is one
 * prefix tree over the functions and leaves of its sequence there (at the
 * skeleton levels a leaf stands for a value an earlier level computed), so
 * the level holds (tokens - trees) / 2 functions, and the functions its own
 * launch evaluates are those less the next level's. */
typedef struct {
    uint64_t tokens;  /* tokens of the level's sequence, over all its trees */
    uint32_t trees;   /* trees with work at this level */
    uint32_t items;   /* work items */
    uint32_t slots;   /* result slots the level writes */
    uint32_t launch;  /* the launch of an evaluation (on the context's own stream) that runs the
                         level: levels with the same value run in one chained launch */
    uint64_t codes;   /* threaded codes of its register-stack work items (0 for the general kernel's) */
} ev_level_info;

/* Errors: EV_EINVAL (level out of range), EV_ENOTFOUND. */
ev_status ev_get_level_info(ev_ctx *ctx, ev_pop pop, int32_t level, ev_level_info *info);

/* Tuning knobs (0 keeps the current value): chunk = tokens per work item
 * of the split at level 0, chunk_hi = at the skeleton levels (default:
 * twice chunk: a skeleton level is short, and a longer work item there
 * saves whole levels), lds_depth = operand-stack entries kept in LDS
 * per wave by the general interpreter (64 or 128).  flags (each call
 * replaces the previous ones; 0 is the default behaviour):
 * EV_TUNE_NO_REGSTACK runs every work item on the general interpreter
 * instead of the register-stack one.  EV_TUNE_NO_RECORD makes the plan
 * builder emit codes by a second pass of the structure machine instead of
 * placing what its counting pass recorded (levels too large to record,
 * over about 300 million tokens, always do).  EV_TUNE_NO_REUSE plans the
 * children of ev_crossover and ev_generation from scratch instead of taking
 * over the code streams and skeleton fragments of their mum's level-0 work
 * items that crossover leaves intact (a child is its mum with one subtree
 * replaced, Sec. 3.1).  EV_TUNE_NO_CHAIN evaluates each skeleton level in
 * a launch of its own instead of all of them in one launch where a tree's
 * work items at a level start as soon as its items of the level before are
 * done.  Plans made and evaluations run afterwards use them; results never
 * depend on them.  EV_TUNE_TEST_FAIL_CHECK is a test hook
 * for the error path of code-stream validation: plans made afterwards
 * record their last level as failing it (the plan is refused, or, for the
 * children of ev_generation, whose verdict is read with their first
 * evaluation, that evaluation fails with EV_EDEVICE and runs none of the
 * level's codes). */
#define EV_TUNE_NO_REGSTACK 0x1u
#define EV_TUNE_NO_RECORD 0x2u
#define EV_TUNE_NO_REUSE 0x4u
#define EV_TUNE_NO_CHAIN 0x8u
#define EV_TUNE_TEST_FAIL_CHECK 0x100u
ev_status ev_set_tuning(ev_ctx *ctx, uint32_t chunk, uint32_t chunk_hi, uint32_t lds_depth, uint32_t flags);

/* Autotuner: re-plans population pop at each candidate work-item size
 * (1024 .. 65536 tokens), times `reps` evaluations on case table `table`
 * with device events, and keeps the fastest: pop is left planned with it and
 * it becomes the context's work-item size for later plans.  Results never
 * depend on the choice (every function node combines the same operands,
 * Sec. 2.2).  *best_chunk and *best_ms (nullable) receive the choice and its
 * median evaluation time.  Errors: EV_EINVAL, EV_ENOTFOUND, EV_ENOMEM,
 * EV_EDEVICE. */
ev_status ev_autotune(ev_ctx *ctx, ev_pop pop, int32_t table, int32_t reps, uint32_t *best_chunk,
                      float *best_ms);

/* The autotuner's search (ev_autotune_ex): the work-item size of level 0
 * and of the skeleton levels, and how many waves per compute unit the
 * register-stack interpreter's persistent grid runs (fewer waves give each
 * more of a SIMD's issue slots).  Results never depend on them. */
typedef struct {
    uint32_t chunk;         /* tokens per level-0 work item */
    uint32_t chunk_hi;      /* tokens per work item at the skeleton levels */
    uint32_t waves_per_cu;  /* interpreter waves per compute unit (0: as many as fit) */
    uint32_t from_cache;    /* 1: taken from the tuning cache, no search */
    float ms;               /* median evaluation time with them */
} ev_tune_choice;

#define EV_AUTOTUNE_NO_CACHE 0x1u /* search even if the cache holds a choice */

/* Coordinate search: the level-0 work-item size among 1024 .. 32768 tokens
 * (the skeleton levels at twice it), then the skeleton size (1, 2 or 4 times
 * it), then the waves per compute unit (all that fit, or 4 or 8 fewer), each
 * timed by `reps` evaluations of pop on case table `table` with device
 * events.  The choice is applied to the context (and pop is left planned
 * with it) and kept in a per-process cache keyed by (device architecture,
 * number of cases, the population's size in powers of two of nodes and of
 * trees); a later call for a population of the same key takes it from there
 * unless EV_AUTOTUNE_NO_CACHE.  Errors: EV_EINVAL, EV_ENOTFOUND, EV_ENOMEM,
 * EV_EDEVICE. */
ev_status ev_autotune_ex(ev_ctx *ctx, ev_pop pop, int32_t table, int32_t reps, uint32_t flags,
                         ev_tune_choice *choice);

/* The tuning cache as text (one line per key) to a file, and read back
 * (merged; later lines win).  Errors: EV_EINVAL (unreadable or unwritable
 * file, malformed line). */
ev_status ev_tune_cache_save(const char *path);
ev_status ev_tune_cache_load(const char *path);

/* Device time in milliseconds of each plan level of the last
 * ev_eval_fitness on this context (levels in evaluation order; the first
 * also holds the counter reset before it).  ms[0..min(cap, levels)) is
 * filled; *n_levels (nullable) receives the number of levels. */
ev_status ev_last_level_times(ev_ctx *ctx, float *ms, int32_t cap, int32_t *n_levels);

/* Device time in milliseconds of the last ev_eval_fitness on this context
 * (HIP events around the evaluation kernels) and of its dominant kernel
 * (the level-0 interpreter launch). */
ev_status ev_last_timing(ev_ctx *ctx, float *eval_ms, float *interp_ms);

#ifdef __cplusplus
}
#endif
#endif
