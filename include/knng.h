/*
 * knng.h — C ABI of the MI355X (gfx950) NN-Descent library, squared-l2 metric.
 *
 * Method: Kluser, Bokstaller, Rutz, Buner, "Fast single-core K-Nearest Neighbor
 * Graph computation" (arXiv 2112.06630). The problem (Sec. 2): for points
 * X[N,d] in R^d, find for every point u the K nearest other points adj_G(u).
 * NN-Descent (Sec. 2) starts from a random graph and repeats a selection step
 * (Sec. 3.1: sample new/old forward and reverse neighbours) and a calculation
 * step (Sec. 2, Sec. 3.3: squared-l2 distances of the sampled pairs, update the
 * lists) until the number of changes falls below a threshold.
 *
 * The iteration here is synchronous and seeded: every sampling weight is a
 * counter-based hash of (seed, t, pair) and every list is ordered by the key
 * (squared distance, original id), so the result does not depend on thread or
 * update order, and does not depend on the graph-ordered point permutation
 * (Sec. 3.2) either.
 *
 * Memory and ownership. Every pointer named d_* is device memory on the
 * current HIP device, owned by the caller. The library never allocates device
 * memory: all scratch lives in the caller's workspace (d_ws, ws_bytes, at
 * least knng_workspace_bytes()). `stream` is a hipStream_t (NULL = legacy
 * default stream); all work is ordered on it. Host pointers may be NULL where
 * marked nullable.
 *
 * Errors. Functions return a knng_status. On any status other than KNNG_OK
 * and KNNG_ENOTCONV the outputs are undefined and knng_last_error() holds a
 * message (thread-local, valid until the next call on the same thread).
 *
 * Thread safety. Calls on different contexts may run concurrently on
 * different streams; calls on one context must be serialised by the caller.
 */
#ifndef KNNG_H
#define KNNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KNNG_OK = 0,
    KNNG_EINVAL = 1,     /* invalid argument (bad size, null pointer, non-finite X) */
    KNNG_ENOMEM = 2,     /* workspace smaller than knng_workspace_bytes() */
    KNNG_EDEVICE = 3,    /* a HIP runtime call failed */
    KNNG_ENOTCONV = 4    /* max_iters reached before the stop rule held; results valid */
} knng_status;

typedef enum {
    KNNG_FP32 = 0,        /* distances in FP32 */
    KNNG_BF16_SCREEN = 1  /* BF16 copies screen candidates on MFMA (FP32 accumulation) with a
                             rigorous error margin; survivors are rescored in FP32 direct form
                             from the original rows (each owner's member rows staged once; sums
                             of 32 squared differences added into FP64, rounded once: at most
                             13 * 2^-24 relative to the distance) and only rescored distances
                             are stored, the initial graph's included (MFMA path, 2C <= 64) */
} knng_precision;

/*
 * Join paths. AUTO takes the VALU direct form when d < 56 or ceil(rho*K) > 32,
 * else (FP32 precision) the split-BF16 Gram form below (the measured
 * crossover of the two on single-Gaussian data at n = 16384, K = 20).
 * KNNG_PATH_MFMA_I8 is reserved (an exact int8 form that was withdrawn):
 * requesting it fails with KNNG_EINVAL.
 */
/*
 * Split-BF16 Gram form (KNNG_PATH_MFMA_BF16X3, what AUTO takes on the MFMA
 * side in FP32 precision). Every FP32 value is written exactly as the sum of
 * three BF16 values, x = x1 + x2 + x3 (x1 = bf16(x), x2 = bf16(x - x1),
 * x3 = x - x1 - x2; Henry, Tang, Heinecke, "Leveraging the bfloat16 artificial
 * intelligence datatype for higher-precision computations", ARITH 2019), and
 * x.y is accumulated in FP32 on BF16 MFMA tiles from the six products
 * xi*yj with i + j <= 4 (each exact in FP32). The three dropped products are
 * below 2^-25 |x_k y_k| per term, so the distance keeps the error bound of the
 * FP32 Gram form; where X holds integers of magnitude <= 256 with partial sums
 * below 2^24 it is exact and bit-identical to the other forms. When x3 = 0 for
 * every element of X (values with at most 16 significant bits), or also
 * x2 = 0 (values exact in BF16, such as 8-bit pixels), the join reads only the
 * planes that are not all zero and skips the products that are exactly zero:
 * the result is bit-identical to the three-plane evaluation (stats.planes).
 *
 * Accuracy of the matrix forms. On data whose FP32 sums are all exact
 * (integers with every squared norm at most 2^23, such as 8-bit pixels) the
 * tiles accumulate in FP32 and every distance is exact. On other data the
 * FP32 Gram form loses accuracy relative to the distance when the points sit
 * far from the origin (its rounding scales with ||x||^2 + ||y||^2), so the
 * matrix forms then keep FP64 squared norms, take each 32-dimension step's
 * MFMA partial dot product into an FP64 accumulator and form
 * ||x||^2 + ||y||^2 - 2 x.y in FP64 before rounding the distance to FP32
 * (stats.accurate = 1). Both ways a pair gets the same value whichever side
 * of a tile it is on.
 */
typedef enum {
    KNNG_PATH_AUTO = 0,         /* see above */
    KNNG_PATH_VALU = 1,         /* sum_j (x_j - y_j)^2 on the vector ALUs */
    KNNG_PATH_MFMA = 2,         /* ||x||^2 + ||y||^2 - 2 x.y with FP32 MFMA tiles */
    KNNG_PATH_MFMA_I8 = 3,      /* reserved: rejected with KNNG_EINVAL */
    KNNG_PATH_MFMA_BF16X3 = 4   /* split-BF16 Gram form on BF16 MFMA tiles, FP32 accumulation */
} knng_path;

/*
 * Sampling rules of the selection step (Sec. 3.1). Both sample new and old
 * members separately, at most C = ceil(rho*K) of each, from the pool of u:
 * its forward entries and the reverse entries (w, u) of every w listing u,
 * each carrying the weight w = H(seed, t, min, max) >> 32 of its pair.
 *
 * KNNG_SAMPLING_WEIGHTED: the C entries of smallest (w, id) per flag (the
 *   bounded-heap rule: a uniform subset of min(C, n) distinct members).
 * KNNG_SAMPLING_TURBO: turbosampling. Each entry of flag f passes a coin of
 *   probability C / n_f(u), n_f(u) being the number of pool entries of flag f
 *   (forward plus reverse, with multiplicity: the neighbourhood size the paper
 *   keeps per node); the coin is the same weight, passing iff
 *   w * n_f(u) < C * 2^32. At most C survivors per flag are kept (those of
 *   smallest (w, id)), so each flag keeps about C members in expectation and
 *   never more than C.
 * In both, an old member also sampled as new is dropped from the old sample,
 * and forward NEW entries of sampled new members become OLD.
 */
typedef enum {
    KNNG_SAMPLING_WEIGHTED = 0,
    KNNG_SAMPLING_TURBO = 1
} knng_sampling;

typedef struct {
    int32_t K;          /* list length, 1 <= K <= 64 and K <= N-1 (Sec. 2: k) */
    double rho;         /* sample rate, 0 < rho <= 1 (Sec. 3.1: rho*k per neighbourhood) */
    double delta;       /* stop when changes < delta*N*K (Sec. 2: threshold), delta >= 0 */
    int32_t max_iters;  /* iteration cap T_max >= 0; 0 returns the random initial graph */
    uint64_t seed;      /* seed of the counter-based hash */
    int32_t precision;  /* knng_precision */
    int32_t reorder;    /* t_p >= 1: graph-ordered point permutation once, after iteration t_p
                           (Sec. 3.2 applies it after the first); 0: off; at most 64. The
                           graph is bitwise the same either way; the later iterations gather
                           rows of nearby points, which pays where the rows the join reads
                           exceed the last-level cache (measured: 200000 x 960, t_p = 2) */
    int32_t path;       /* knng_path */
    int32_t sampling;   /* knng_sampling (Sec. 3.1) */
    int32_t blocks;     /* 0 or 1: synchronous iterations. B > 1 (B <= N): block-asynchronous
                           iterations, the paper's in-place update (Sec. 3.1) at block
                           granularity: the owners are taken in B blocks of consecutive
                           original ids, in order; block b samples from the graph as blocks
                           0..b-1 of the iteration left it, only its owners sample, flip and
                           join, and their proposals are merged into every list before block
                           b + 1 samples. Deterministic; e_t and c_t add up over the blocks. */
} knng_params;

#define KNNG_MAX_ITERS 64

/* Per-build statistics, written to host memory when the pointer is non-NULL.
 * Times are device times from HIP events on the build's stream. */
typedef struct {
    int32_t iters;                        /* iterations run */
    int32_t converged;                    /* 1 if the stop rule held */
    int32_t path;                         /* path used (knng_path, resolved) */
    int32_t dpad;                         /* padded row length in floats */
    int32_t precision;                    /* knng_precision used */
    int32_t planes;                       /* split-BF16 form: BF16 planes the join reads (1..3), else 0 */
    int32_t accurate;                     /* matrix paths: 1 when FP32 sums of X are not exact (see
                                             knng_path), so dot products are summed in FP64 per
                                             32 dimensions; 0 where every FP32 sum is exact */
    int32_t u8;                           /* split form on 8-bit data (integers 0..255): 1 when the
                                             join reads the rows as bytes */
    int64_t evals[KNNG_MAX_ITERS];        /* e_t: distance evaluations of iteration t */
    int64_t changes[KNNG_MAX_ITERS];      /* c_t: ids that entered a list */
    int64_t proposals[KNNG_MAX_ITERS];    /* proposals that passed the snapshot filter */
    int64_t rescored[KNNG_MAX_ITERS];     /* BF16 form: pairs that passed the screen (rescored in FP32) */
    float iter_ms[KNNG_MAX_ITERS];        /* whole iteration */
    float sample_ms[KNNG_MAX_ITERS];      /* reverse bucketing + selection */
    float join_ms[KNNG_MAX_ITERS];        /* local join (pairs, distances, proposals) */
    float merge_ms[KNNG_MAX_ITERS];       /* top-K merge */
    float init_ms;                        /* row padding + random initial graph */
    float reorder_ms;                     /* graph-ordered permutation (0 if off) */
    float finalize_ms;                    /* write-out in original order */
    float total_ms;                       /* init .. finalize */
} knng_stats;

typedef struct knng_ctx knng_ctx;

/* Bytes of device workspace a build of N points of dimension d needs. Returns
 * 0 if the sizes or params are invalid (see knng_last_error()). */
size_t knng_workspace_bytes(int64_t N, int32_t d, const knng_params* params);

/* One-shot build (Sec. 2): init, iterate until c_t < delta*N*K or max_iters,
 * write d_ids[N*K] (original row indices, int32) and d_dists[N*K] (squared l2,
 * FP32), each row sorted ascending by (distance, id).
 * dX: device, row-major float32 [N, d], finite. Synchronises `stream` once
 * per iteration (to read c_t for the stop rule). Returns KNNG_ENOTCONV when
 * max_iters was reached first. `stats` (host) may be NULL. */
knng_status knng_build(const float* dX, int64_t N, int32_t d, const knng_params* params,
                       int32_t* d_ids, float* d_dists, void* d_ws, size_t ws_bytes,
                       void* stream, knng_stats* stats);

/* Allocation-free build, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): knng_build with its workspace taken from a static device array
 * of KNNG_NOALLOC_MAX_BYTES that the library holds on every device it runs
 * on, for the life of the process. The caller passes inputs and outputs as
 * for knng_build (device memory, caller-owned). The call allocates nothing
 * (no hipMalloc, hipFree, pinned memory or events): the per-iteration
 * counters are read back from the same array; stats (nullable) carry counts
 * but no timings. Fails with KNNG_ENOMEM, before any device work, when
 * knng_workspace_bytes(N, d, params) + 4160 bytes exceed the array: a build
 * of 2000 points with K = 10 needs 7 MiB, 6000 points with K = 15 about
 * 50 MiB. Every call on one device shares that device's array and leaves its
 * contents behind (the build initialises what it reads), so calls that
 * overlap in time on one device race and must be serialised by the caller.
 * Synchronises `stream` once per iteration. */
#define KNNG_NOALLOC_MAX_BYTES (64u << 20)
knng_status knng_build_noalloc(const float* dX, int64_t N, int32_t d, const knng_params* params,
                               int32_t* d_ids, float* d_dists, void* stream, knng_stats* stats);

/* ---- step API: one context per build, the state lives in the workspace ---- */

/* Bind a context to (dX, N, d, params, workspace, stream); pads the rows and
 * checks X is finite (one synchronisation). dX and the workspace must stay
 * valid until knng_destroy. *out receives a host-allocated handle. */
knng_status knng_create(knng_ctx** out, const float* dX, int64_t N, int32_t d,
                        const knng_params* params, void* d_ws, size_t ws_bytes, void* stream);

/* Random initial graph G_0 (Sec. 2): K distinct non-self ids per point from
 * the hash, all flagged new, rows sorted by (distance, id). Sets t = 0. */
knng_status knng_init_graph(knng_ctx* ctx);

/* Load a graph state: d_ids[N*K] int32 original ids (row u = point u),
 * d_dists[N*K] float squared l2 or NULL, and d_flags[N*K] uint8 (1 = new,
 * 0 = old); rows are re-sorted by (distance, id). With d_dists (a state from
 * knng_export) the distances are kept bit for bit, so the build continues
 * exactly as the exporting one would; with NULL they are recomputed on the
 * device in the form init uses. A row with an id out of range, its own id, a
 * repeated id, or a distance that is negative or not finite is rejected
 * (KNNG_EINVAL, no graph loaded). Sets the iteration counter to t (the next
 * iterate runs t+1). Only valid before any permutation of this context. */
knng_status knng_load_graph(knng_ctx* ctx, const int32_t* d_ids, const float* d_dists, const uint8_t* d_flags,
                            int32_t t);

/* One synchronous iteration t+1: sample (Sec. 3.1), local join (Sec. 2,
 * Sec. 3.3), merge. Applies the permutation after iteration t_p when
 * params.reorder is set. Synchronises `stream` once. Writes e_t and c_t
 * (host, nullable). */
knng_status knng_iterate(knng_ctx* ctx, int64_t* evals, int64_t* changes);

/* Current graph in original order: d_ids[N*K], d_dists[N*K], d_flags[N*K]
 * (nullable), rows sorted by (distance, id). */
knng_status knng_export(knng_ctx* ctx, int32_t* d_ids, float* d_dists, uint8_t* d_flags);

/* Sampled sets of the last iteration in original order: d_new[N*C],
 * d_old[N*C] (int32 original ids; new sorted by (weight, id)), d_counts[2*N]
 * (n_new, n_old per point). C = min(K, max(1, ceil(rho*K))). */
knng_status knng_export_samples(knng_ctx* ctx, int32_t* d_new, int32_t* d_old, int32_t* d_counts);

/* Storage order of the points: d_orig_of_pos[N] (int32, device) receives the
 * original id stored at each position; the identity until the graph-ordered
 * permutation (Sec. 3.2) has run. */
knng_status knng_export_order(knng_ctx* ctx, int32_t* d_orig_of_pos);

/* Statistics accumulated by the context so far (host). */
knng_status knng_get_stats(const knng_ctx* ctx, knng_stats* stats);

/* Free the host handle (no device memory is owned). */
void knng_destroy(knng_ctx* ctx);

/* ---- batched form: many independent datasets in one graph launch ---- */

/* One dataset of a batch: device input rows dX [N, d] (float32, row-major,
 * finite) and device outputs d_ids / d_dists [N, K] (original row indices
 * within the dataset, squared l2), each row sorted by (distance, id). */
typedef struct {
    const float* dX;
    int64_t N;
    int32_t d;
    int32_t reserved;
    uint64_t seed;       /* the dataset's own seed (params.seed is not used) */
    int32_t* d_ids;
    float* d_dists;
} knng_dataset;

typedef struct knng_batch knng_batch;

/* Workspace bytes of a batch (room for either join path of every group). */
size_t knng_batch_workspace_bytes(const knng_dataset* descs, int32_t n, const knng_params* params);

/* Plan a batch: groups datasets by dimension and join path, uploads the
 * per-dataset tables (seeds, offsets, pointers) into the workspace and checks
 * every input is finite. `tuning` is NULL/"auto" (the autotuner: for every
 * dimension, each join path the cap allows and two launch shapes of the select
 * and join passes, one workgroup per four owners or eight workgroups per
 * compute unit looping over the owners, each run as the whole build of that
 * dimension's datasets on the batch itself; the fastest is kept) or a table
 * such as "16:valu,64:mfma@2048,128:bf16x3" (path per d; "@n": at most n
 * workgroups in the select and join passes). params.K, rho, delta, max_iters
 * (>= 1) apply to every dataset; params.reorder must be 0, params.blocks at
 * most 1, params.precision KNNG_FP32. Synchronises `stream`. Results equal
 * those of one knng_build per dataset with the same join path, whatever the
 * launch shape. Once every dataset of a dimension group has stopped, the
 * group's later passes return at entry. */
knng_status knng_batch_plan(knng_batch** out, const knng_dataset* descs, int32_t n, const knng_params* params,
                            void* d_ws, size_t ws_bytes, const char* tuning, void* stream);

/* The tuning table the plan uses (valid until knng_batch_destroy). */
const char* knng_batch_tuning(const knng_batch* plan);

/* Enqueue the whole batched build (setup, init, max_iters iterations in which
 * finished datasets are skipped, write-out). Allocates nothing and never
 * synchronises: it may be captured in a graph. */
knng_status knng_batch_execute(knng_batch* plan, void* stream);

/* Capture knng_batch_execute on `stream` (not the default stream) into a
 * graph owned by the plan; knng_batch_launch then runs it in one launch. */
knng_status knng_batch_capture(knng_batch* plan, void* stream);
knng_status knng_batch_launch(knng_batch* plan, void* stream);

/* After the build: per dataset (caller order) iterations run, converged flag,
 * and e_t / c_t per iteration (arrays [n * max_iters], nullable). Synchronises
 * `stream`; KNNG_EDEVICE if a device invariant failed during the build. */
knng_status knng_batch_stats(knng_batch* plan, int32_t* iters, int32_t* converged, int64_t* evals,
                             int64_t* changes, void* stream);

void knng_batch_destroy(knng_batch* plan);

/* Per-flag sample cap C for (K, rho). */
int32_t knng_sample_cap(int32_t K, double rho);

/* Message of the last failure on this thread ("" if none). */
const char* knng_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KNNG_H */
