/*
 * gbf — generalized Bellman-Ford solver for symbolic optimal control on
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The library solves optimal control problems (X, U, F, G, g) as defined in
 * Weber, Kreuzer, Knoll, "A generalized Bellman-Ford Algorithm for
 * Application in Symbolic Optimal Control", Sect. III-C (Definition of an
 * optimal control problem): a finite state set X = {0..n-1}, a finite input
 * set U = {0..K-1}, a strict transition map F: X x U => X (every F(x,u) is
 * non-empty, Sect. II / III-A), a terminal cost G: X -> R u {inf} and a
 * running cost g.  Running costs are per pair, g(x,u), i.e. the cost does
 * not depend on the successor y (the paper allows g(x,y,u); with per-pair
 * costs the sup over y of g + W(y) is g(x,u) + max_y W(y)).
 *
 * It returns the value function V, the maximal fixed point of the dynamic
 * programming operator
 *     P(W)(x) = min{ G(x), min_u max_{y in F(x,u)} g(x,u) + W(y) }
 * (Theorem on dynamic programming, Sect. III-C), computed by the frontier
 * iteration of Algorithm 1 (Sect. IV-A), and a controller that realizes it.
 *
 * Conventions
 *   - INF is INT32_MAX for int32 costs and +infinity for float costs.
 *   - Pair (x,u) has id p = x*K + u.  State x of a grid with dims
 *     (N0,N1,N2,N3) is x = x0 + N0*(x1 + N1*(x2 + N2*x3)).
 *   - Avoid cells (optional byte mask) are states the controller must never
 *     enter: their value is pinned to INF and no pair leading into them is
 *     ever chosen.  A finite G on an avoid cell is rejected.
 *   - Every call returns a status code (GBF_OK = 0, errors < 0); no call
 *     throws or aborts.  gbf_last_error() returns a message for the last
 *     failing call of the calling thread.
 *   - All device work is ordered on the HIP stream given at load time.
 *     Calls return after their work has completed.
 *   - A handle must not be used by two threads at once; gbf_solve_batch
 *     calls are serialised inside the library.  Freeing a handle also drops
 *     the batch state (and captured HIP graph) of every batch it was in.
 *   - "Memory space" arguments say whether a pointer is host (GBF_HOST) or
 *     device (GBF_DEVICE) memory of the current device.
 */
#ifndef GBF_H
#define GBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GBF_OK 0
/* The round cap was reached with a non-empty frontier (the second condition
 * of the while loop of Algorithm 1).  V_out then holds the capped iterate,
 * which is >= V but not certified to equal it.  On ordinary graphs this
 * means a negative cycle; on hypergraphs it can also mean that more rounds
 * are needed, see gbf_opts.max_rounds. */
#define GBF_ENEGCYCLE 1
#define GBF_EINVAL (-1)      /* invalid argument or problem */
#define GBF_ENOMEM (-2)      /* device or host allocation failed */
#define GBF_EHIP (-3)        /* a HIP runtime call failed */
#define GBF_ENOTSOLVED (-4)  /* gbf_extract_policy before a successful solve */
#define GBF_ETIMEOUT (-5)    /* a device-side bounded wait expired */

/* ---- enums ------------------------------------------------------------ */
#define GBF_I32 0 /* int32 costs and values */
#define GBF_F32 1 /* float costs and values */

#define GBF_CSR 0 /* explicit successor lists */
#define GBF_BOX 1 /* implicit boxes: 8 bytes per pair, successors on the fly */

#define GBF_HOST 0
#define GBF_DEVICE 1

#define GBF_ORDER_PLAIN 0   /* frontier rounds as in Algorithm 1 */
#define GBF_ORDER_BUCKETS 1 /* frontier drained in ascending bucket key */
#define GBF_BUCKET_SPAN_DEFAULT 32

#define GBF_MODE_AUTO 0       /* single block up to 65536 pairs (one instance), else host loop */
#define GBF_MODE_HOSTLOOP 1   /* one launch sequence per round from the host */
#define GBF_MODE_PERSISTENT 2 /* all rounds in one cooperative launch */
#define GBF_MODE_SINGLE_BLOCK 3 /* all rounds in one workgroup (small single instances) */

/* policy sentinels (Algorithm 1 leaves mu(x) = U for such states) */
#define GBF_HANDOVER (-1) /* V(x) = G(x): hand over now */
#define GBF_NONE (-2)     /* V(x) = INF: no controller exists */

/* ---- problem ------------------------------------------------------------
 * The optimal control problem (X, U, F, G, g) of Sect. III-C.
 * Arrays are read during gbf_load_graph only; the library keeps its own
 * device copies, so the caller may free them on return.                   */
typedef struct gbf_problem {
    int64_t n_states;   /* |X| >= 1 */
    int32_t n_inputs;   /* |U| = K >= 1 */
    int32_t dtype;      /* GBF_I32 or GBF_F32: type of G, g and V */
    int32_t encoding;   /* GBF_CSR or GBF_BOX */
    int32_t memspace;   /* GBF_HOST or GBF_DEVICE: where the arrays live */
    const void* G;      /* [n] terminal cost; INF = not a target */
    const void* g;      /* [n*K] running cost of pair (x,u); INF = forbidden */
    const uint8_t* avoid; /* [n] 1 = avoid cell, or NULL */
    /* GBF_CSR: F(x,u) = { succ_idx[e] : succ_ptr[p] <= e < succ_ptr[p+1] }.
     * Rows must be non-empty (strictness); total m < 2^31. */
    const int64_t* succ_ptr; /* [n*K+1] */
    const int32_t* succ_idx; /* [m], values in [0,n) */
    /* GBF_BOX: the states form a grid with dims[0..3] (unused axes = 1,
     * prod = n); F(x,u) is the box whose low corner is the cell
     * (uint32)box[p] and whose extent on axis a is byte a of box[p] >> 32,
     * i.e. the cells c with lo_a <= c_a <= lo_a + ext_a.  Boxes must lie in
     * the grid.  This is the rectangular over-approximation of attainable
     * sets used in Sect. V-B; successors are decoded on the fly and
     * predecessors are searched in a window per input, which the loader
     * derives from the boxes (a superset of pred, allowed by Sect. V-B). */
    int32_t dims[4];
    const uint64_t* box; /* [n*K] */
    /* GBF_BOX only (Sect. IV-B: keeping images of F and pred in memory vs
     * recomputing them):
     *   0 = implicit: successors decoded from the boxes, predecessors
     *       searched in per-input windows (least memory);
     *   1 = expand the boxes into explicit successor lists and a reverse
     *       CSR on the device at load time (~8 bytes per successor);
     *   2 = successors decoded from the boxes, predecessors from a reverse
     *       CSR built at load time (~4 bytes per successor);
     *   3 = memory-budgeted images (Sect. VI-A: the paper's implementation
     *       keeps computed images of F and pred in memory up to a user
     *       threshold of its RAM, 68%, and recomputes beyond it): the
     *       predecessor images of 2 are built if the handle's peak memory
     *       at load stays within mem_budget, else the problem stays
     *       implicit as in 0.  gbf_stats.enc_used reports the choice. */
    int32_t expand_box;
    /* Width of the (x,u) pair ids inside the solver.  Problems with
     * n_states * n_inputs < 2^31 use 32-bit ids; larger ones (up to the
     * 2^32 - 1 states that the box encoding addresses) use 64-bit ids, with
     * GBF_BOX and expand_box 0, 2 or 3 only: one instance per solve, the
     * host-loop mode and the plain order (Sect. VI-A solves a problem of
     * 141.7 M states and 35 inputs, about 5 G pairs).  1 = 64-bit ids at any
     * size (same restrictions); 0 = by size. */
    int32_t pair_ids64;
    /* Optional per-edge part of the running cost (Sect. III-B defines the
     * running cost on transitions, g(x,y,u); the operator of Sect. III-C
     * and the sup of Algorithm 1 take g(x,y,u) + W(y) per successor).  The
     * cost of the transition from x under u to the successor listed at
     * succ_idx[e] is g[x*K+u] + g_edge[e], so the backup of a pair is
     *   g(x,u) + max over its row of (g_edge[e] + W(succ_idx[e])).
     * [m] values of the problem's dtype, in succ_idx order; NULL = all 0.
     * GBF_CSR only (GBF_EINVAL with GBF_BOX).  Every value must be finite
     * (int32: not INT32_MAX; fp32: not NaN or +-inf), else GBF_EINVAL.
     * int32 sums are exact in int64 with the rules of g; fp32 adds
     * g_edge[e] + W(y) with one round-to-nearest-even addition and the
     * pair cost with one more.  Same memspace as the other arrays; copied
     * at load. */
    const void* g_edge;
    /* expand_box 3: device memory budget in bytes for the handle at load;
     * 0 = 68% of the device memory free at load.  Must be >= 0. */
    int64_t mem_budget;
} gbf_problem;

/* ---- solve options --------------------------------------------------- */
typedef struct gbf_opts {
    int32_t order;          /* GBF_ORDER_PLAIN or GBF_ORDER_BUCKETS */
    int32_t mode;           /* GBF_MODE_* */
    const uint16_t* bucket_key; /* BUCKETS: [n] device array, key of state x;
                                   only the processing order depends on it */
    int64_t max_rounds;     /* round cap; 0 = n (the paper's i < |X|) */
    int32_t lanes;          /* lanes per frontier pair in the relax step:
                               1, 2, 4, 8, 16 or 32; 0 = default (4) */
    int32_t grid;           /* blocks; 0 = default */
    int32_t v_memspace;     /* where V_out lives: GBF_HOST or GBF_DEVICE */
    int32_t profile;        /* 1 = time every relax launch with HIP events */
    int32_t batch_hint;     /* host-loop mode: rounds launched before the first
                               frontier-size check; 0 = default (8) */
    int32_t bucket_span;    /* BUCKETS: k >= 1 = each round lists the dirty pairs
                               of the k buckets from the lowest occupied one up;
                               -1 = ascending sweeps, one bucket per round;
                               0 = default (GBF_BUCKET_SPAN_DEFAULT) */
    int32_t bucket_budget;  /* BUCKETS: work budget in percent of the reference
                               (the pair evaluations of the handle's last
                               plain solve, and twice its rounds; without
                               one, 16 evaluations per pair): past it, or
                               when from round 24 on the pair evaluations so
                               far fall below 0.6 of that plain solve's at
                               the same round (host-loop plain solves keep
                               that profile), the solve finishes in plain
                               order (gbf_stats.fallback 1).  0 = 100;
                               -1 = no budget (the switch still comes by
                               round 65536, so that the plain continuation
                               keeps the plain round cap) */
    int32_t mem_floor_mib;  /* handles holding predecessor images (box successors
                               with a reverse CSR): if at a frontier-size check of
                               a host-loop solve the device's free memory is
                               below this many MiB, the reverse CSR is released
                               and the rest of the solve, and later solves of
                               the handle, search predecessors in the per-input
                               windows as the implicit form does
                               (gbf_stats.images_dropped, enc_used 1); the
                               values are the same.  0 = never. */
    int32_t block;          /* host-loop mode: threads per block of the relax
                               kernel, a multiple of 64 from 64 to 1024;
                               0 = default (512).  `grid` still counts
                               256-thread blocks: the launch has
                               grid * 256 / block blocks. */
    int32_t compact_grid;   /* host-loop mode: blocks of the frontier
                               compaction (a frontier chunk is 16 pairs, a
                               block scans 256 chunks per tile); 0 = default
                               (512) */
} gbf_opts;

/* ---- statistics ------------------------------------------------------- */
typedef struct gbf_stats {
    int32_t status;         /* status of this solve */
    int32_t fallback;       /* bucket order: 0 = ran in bucket order to the end;
                               1 = exceeded its work budget
                               (gbf_opts.bucket_budget) and finished in plain
                               order from the current iterate; 2 = reached
                               its round cap and
                               the plain order was rerun from scratch.  The
                               values and policy are the same in every case. */
    int64_t rounds;         /* rounds executed (passes of the while loop) */
    int64_t pair_evals;     /* pairs (x,u) whose successors were read */
    int64_t edge_relax;     /* sum of |F(x,u)| over those pairs */
    int64_t improvements;   /* successful strict decreases of V */
    int64_t saturations;    /* int32 sums clamped at -INT32_MAX */
    int64_t expansions;     /* states whose predecessors were marked */
    int64_t marks;          /* predecessor pairs (or box candidates) visited */
    double solve_ms;        /* HIP-event time of the solve on its stream */
    double relax_ms;        /* profile=1: summed time of the relax launches */
    int64_t relax_launches; /* profile=1: number of relax launches timed */
    double barrier_ms;      /* persistent mode: time block 0 spent in grid barriers */
    int64_t device_bytes;   /* device memory held by the graph handle */
    int32_t mode_used;      /* GBF_MODE_HOSTLOOP or GBF_MODE_PERSISTENT */
    int32_t grid_used;      /* host-loop mode: in 256-thread blocks (gbf_opts.grid) */
    int32_t block_used;     /* threads per block of the relax (host loop) or round kernel */
    int32_t lanes_used;
    int32_t graph_used;     /* 1 = batched solve replayed from a HIP graph */
    int32_t sweeps;         /* bucket order: ascending passes over the buckets */
    int32_t enc_used;       /* representation the handle holds: 0 CSR, 1 implicit
                               boxes, 2 boxes + reverse CSR (expand_box 2, or
                               3 when the predecessor images fit the budget),
                               3 aircraft abstraction (gbf_load_aircraft) */
    int32_t images_dropped; /* 1 = this solve released the predecessor images
                               (gbf_opts.mem_floor_mib) */
} gbf_stats;

typedef struct gbf_graph gbf_graph;

/* Validates a problem, copies it to device memory owned by the handle and
 * builds what the solver needs: the reverse adjacency pred (Sect. IV-A,
 * pred(x,u) = { y : x in F(y,u) }) as a pair-level reverse CSR for
 * GBF_CSR (and GBF_BOX with expand_box 1 or 2, or 3 within the memory
 * budget), or per-input predecessor windows for GBF_BOX with expand_box 0
 * (or 3 over the budget); pairs that can
 * never improve a value (g = INF, avoid source, or a successor in the avoid
 * set) are pruned.  `hip_stream` is a hipStream_t (NULL = default stream)
 * on which all later work of this handle is ordered.
 * Errors: GBF_EINVAL (n or K <= 0, empty F(x,u), index or box outside the
 * grid, NaN or -inf cost, finite G on an avoid cell, m >= 2^31, per-edge
 * costs that are not finite or come with GBF_BOX, expand_box outside 0..3,
 * mem_budget < 0, n_states * n_inputs >= 2^31 or pair_ids64 = 1 without
 * GBF_BOX and expand_box 0, 2 or 3, n_states >= 2^32, predecessor offsets
 * of 2^31 pairs or more with 64-bit ids and expand_box 2), GBF_ENOMEM,
 * GBF_EHIP.  On error *out is NULL. */
int gbf_load_graph(const gbf_problem* p, void* hip_stream, gbf_graph** out);

/* Runs Algorithm 1 (Sect. IV-A) until the frontier is empty or the round
 * cap is reached and writes V to V_out ([n] of the problem's dtype, in
 * opts->v_memspace).  Also keeps V inside the handle for
 * gbf_extract_policy.  `opts` may be NULL (defaults); `st` may be NULL.
 * Returns GBF_OK, GBF_ENEGCYCLE (V_out holds the capped iterate),
 * GBF_EINVAL (BUCKETS without a key), GBF_ETIMEOUT, GBF_EHIP. */
int gbf_solve(gbf_graph* g, const gbf_opts* opts, void* V_out, gbf_stats* st);

/* Allocation-free form of gbf_solve, for callers that cannot allocate
 * device memory at solve time (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same semantics and results as
 * gbf_solve with the plain order; it calls no hipMalloc, hipFree,
 * hipHostMalloc or hipEventCreate.  All solver scratch (frontier byte
 * maps, frontier list, per-round counts, statistics, barrier and status
 * words) lives in one static device array of the library, ~57 MiB, which
 * every device the library runs on holds until the process ends.  Limits:
 * n_states * n_inputs <= GBF_NOALLOC_MAX_PAIRS and a round cap (max_rounds,
 * or n_states when it is 0) <= GBF_NOALLOC_MAX_ROUNDS; larger problems get
 * GBF_EINVAL before any device work.  GBF_ORDER_BUCKETS gets GBF_EINVAL;
 * opts->profile is ignored (no per-launch timing) and st->solve_ms is
 * host wall time.  V_out as for gbf_solve (host or device, per
 * opts->v_memspace).  Every call on one device shares that device's array
 * and overwrites it (each solve clears what must start at zero), so calls
 * that overlap in time on one device race: serialise them.  gbf_extract_policy
 * works after it as after gbf_solve. */
#define GBF_NOALLOC_MAX_PAIRS (1 << 23)
#define GBF_NOALLOC_MAX_ROUNDS (1 << 21)
int gbf_solve_noalloc(gbf_graph* g, const gbf_opts* opts, void* V_out, gbf_stats* st);

/* Canonical controller from the last solve (Algorithm 1's mu, made
 * independent of processing order): policy[x] = the smallest input u with
 * g(x,u) + max_{y in F(x,u)} V(y) = V(x) < G(x); GBF_HANDOVER if
 * V(x) = G(x) < INF; GBF_NONE if V(x) = INF.  policy_out is [n] int32 in
 * `memspace`.  If `residual` is non-NULL it receives the number of states
 * where P(V)(x) != V(x) (0 certifies a fixed point).
 * Errors: GBF_ENOTSOLVED, GBF_EHIP. */
int gbf_extract_policy(gbf_graph* g, int32_t* policy_out, int32_t memspace, int64_t* residual);

/* Solves `count` independent problems in one persistent launch (or one
 * launch sequence per round), with one frontier spanning all of them.
 * Results are identical to gbf_solve on each handle.  All handles must be
 * on the same device and stream.  V_outs[i] receives instance i's values
 * (in opts->v_memspace); st (may be NULL) is an array of `count` stats.
 * Returns the worst status over the instances. */
int gbf_solve_batch(gbf_graph* const* graphs, int32_t count, const gbf_opts* opts,
                    void* const* V_outs, gbf_stats* st);

/* Autotuner: times gbf_solve (count == 1) or gbf_solve_batch (count > 1)
 * on the given handles for each candidate launch configuration (host-loop
 * mode: lanes per pair 2/4/8 x relax grid 4/8/16 256-thread blocks per CU x
 * relax block 256/512/1024 threads, then the compaction grid 256/512/1024
 * blocks for the best of those; persistent mode: lanes 2/4/8; for one
 * instance of at most 262144 pairs, single-block mode: lanes 2/4/8) and writes the fastest into *best (the other
 * fields are copied from `base`, which may be NULL).  Each candidate runs
 * one untimed and `reps` (0 = 3) timed solves; the median decides.
 * best_ms (may be NULL) receives its median solve time.  A base->mode
 * other than GBF_MODE_AUTO times that mode's candidates only (GBF_EINVAL if
 * it has none, e.g. single-block for a batch).  The handles keep
 * the last candidate's solve.  The encoding is fixed by the handles: load
 * an instance in several encodings to choose between them.
 * Errors: GBF_EINVAL, GBF_EHIP (no candidate ran). */
int gbf_tune(gbf_graph* const* graphs, int32_t count, const gbf_opts* base, int32_t reps, gbf_opts* best,
             double* best_ms);

/* Releases a handle (NULL is allowed). */
void gbf_free_graph(gbf_graph* g);

/* Releases the state the library keeps across calls: the batch contexts of
 * gbf_solve_batch (their scratch, private streams and captured HIP graphs).
 * Handles stay valid; a later batch call rebuilds its context.  The library
 * never releases this state from a static destructor (those run at process
 * exit, possibly after the HIP runtime has shut down), so a program that
 * wants it freed calls this while the runtime is up, e.g. from an exit
 * handler after freeing its handles.  It waits for a batch call running in
 * another thread to finish. */
void gbf_shutdown(void);

/* ---- frontier-ordering network -----------------------------------------
 * A multilayer perceptron 4 -> 64 -> 64 -> 1 with ReLU, trained on value
 * functions the solver produced, that predicts V from the coordinates of a
 * grid cell.  Its predictions only order the frontier (GBF_ORDER_BUCKETS:
 * the buckets are drained lowest first, which cuts re-evaluations of pairs
 * whose successors are not final yet); the fixed point of Sect. III-C, and
 * so every value and the policy, does not depend on them.
 *
 * Features of cell x = x0 + N0*(x1 + N1*(x2 + N2*x3)) of a grid with dims
 * N: ((x0+.5-tcx)/N0, (x1+.5-tcy)/N1, (x2+.5)/N2, (x3+.5)/N3), where
 * (tcx, tcy) is the centre of the target in cell units.  The network output
 * is V/scale.  Parameters: 4545 floats, W1 [64][4], b1 [64], W2 [64][64]
 * (W2[j][k] feeds hidden unit k of layer 1 into unit j of layer 2), b2 [64],
 * W3 [64], b3.  They are kept as an fp32 master copy (trained with Adam,
 * beta1 0.9, beta2 0.999, eps 1e-8) and a bfloat16 working copy (round to
 * nearest even) that every forward and backward pass uses, accumulating in
 * fp32.  Device arrays are on the current device; all work is ordered on
 * the stream given at creation, and calls return after it has completed.
 * Errors: GBF_EINVAL, GBF_ENOMEM, GBF_EHIP (message in gbf_last_error). */
#define GBF_MLP_NPARAMS 4545
typedef struct gbf_mlp gbf_mlp;

/* New network with the given initial parameters (host [4545], finite). */
int gbf_mlp_create(const float* params, void* hip_stream, gbf_mlp** out);
/* Replaces the parameters (host [4545]) and resets the Adam state. */
int gbf_mlp_set_params(gbf_mlp* net, const float* params);
/* Copies the fp32 master copy and/or the bf16 working copy (bit patterns)
 * to host arrays of 4545 entries (either may be NULL). */
int gbf_mlp_get_params(gbf_mlp* net, float* master_out, uint16_t* bf16_out);
/* Training samples: for each cells[s] (device int64 [count]) writes its
 * features to feat_out (device float [count][4]) and, if target_out (device
 * float [count]) is non-NULL, the label V[cell]/scale from V (device [n],
 * v_dtype GBF_I32 or GBF_F32), NaN where V is INF (no label).  A cell
 * outside the grid gives NaN features and no label. */
int gbf_mlp_samples(gbf_mlp* net, const int32_t dims[4], float tcx, float tcy, const void* V, int32_t v_dtype,
                    float scale, const int64_t* cells, int64_t count, float* feat_out, float* target_out);
/* Network outputs (device float [count]) for feature rows (device float
 * [count][4]). */
int gbf_mlp_forward(gbf_mlp* net, const float* feat, int64_t count, float* out);
/* Gradient of the mean squared error over the labelled samples (target not
 * NaN) with respect to the bf16 parameters.  The samples are rows idx[s]
 * (device int64 [count]; NULL = rows 0..count-1) of feat (device [rows][4])
 * and target (device [rows]); an index outside [0, rows) is skipped.
 * grad_out: host [4545] or NULL; loss_out / labels_out: host or NULL. */
int gbf_mlp_grad(gbf_mlp* net, const float* feat, const float* target, int64_t rows, const int64_t* idx,
                 int64_t count, float* grad_out, double* loss_out, int64_t* labels_out);
/* One Adam step (learning rate lr) on the minibatch given as for
 * gbf_mlp_grad; refreshes the bf16 working copy.  loss_out (host, or NULL
 * to return without waiting for it) receives the minibatch loss before the
 * step. */
int gbf_mlp_train_step(gbf_mlp* net, const float* feat, const float* target, int64_t rows, const int64_t* idx,
                       int64_t count, float lr, float* loss_out);
/* Bucket keys for every cell of the grid (n = product of dims < 2^32):
 * vhat = scale * output, key = clamp(floor((vhat - min vhat) / width), 0,
 * 65535) into key_out (device uint16 [n]), usable as gbf_opts.bucket_key.
 * vhat_out (device float [n]) and vhat_min_out (host) may be NULL. */
int gbf_mlp_bucket_keys(gbf_mlp* net, const int32_t dims[4], float tcx, float tcy, float scale, float width,
                        uint16_t* key_out, float* vhat_out, float* vhat_min_out);
/* Releases a network (NULL is allowed). */
void gbf_mlp_free(gbf_mlp* net);

/* ---- aircraft abstraction ------------------------------------------------
 * The discrete abstraction of a sampled system (Sect. V-B) for the
 * point-mass aircraft of Sect. VI-A,
 *     x1' = x4 cos x3, x2' = x4 sin x3, x3' = p_L x4 sin(u2) / m,
 *     x4' = (u1 - p_D x4^2) / m,
 * computed on the device and solved without stored images.  The state space
 * [0, x_max[0]] x [0, x_max[1]] x [-pi, pi] x [v_range[0], v_range[1]] is
 * covered by dims[0..3] compact cells (the heading is periodic); cell ids are
 * x = i1 + dims[0] (i2 + dims[1] (i3 + dims[2] i4)), pair ids x K + u.
 * Inputs u = a n_bank + b are the vertices of an even subdivision of
 * [0, thrust_max] x [-bank_max_deg, bank_max_deg] degrees: thrust
 * a thrust_max / (n_thrust - 1), bank angle
 * ((2 b - (n_bank - 1)) bank_max_deg / (n_bank - 1)) pi / 180.
 * F(x,u) is the set of cells met by an enclosure of the attainable set of
 * cell x after tau seconds under u (Sect. V-B over-approximates attainable
 * sets by hyper-rectangles).  Enclosure: `steps` steps of the first-order
 * interval Taylor method with a priori enclosures, in double precision
 * with outward rounding; the positions do not enter the dynamics, so one
 * enclosure per (heading cell, speed cell, input) serves every position.
 * Predecessors come from reverse rows of that table (exact).
 * Costs (fp32 values): a transition into a cell inside a reward box costs
 * reward_cost, any other tau + u2^2 (u2 in radians); a pair whose
 * enclosure leaves the grid on x1, x2 or the speed has infinite cost; a
 * cell meeting an avoid box is an obstacle (V = inf).  G: the device array
 * G (fp32 [n], e.g. the value function of a first problem, Sect. VI-A's
 * G_2 = V_1), or, if NULL, 0 on cells inside a target box and inf
 * elsewhere.  Boxes are closed, with integer bounds per axis: metres,
 * degrees within [-180, 180] for the heading, m/s. */
typedef struct gbf_ac_box {
    int32_t lo[4];
    int32_t hi[4];
} gbf_ac_box;

typedef struct gbf_aircraft {
    int32_t dims[4];        /* >= 1; dims[2], dims[3] <= 255; n = product < 2^32 - 1 */
    int32_t x_max[2];       /* > 0 */
    int32_t v_range[2];     /* 0 < v_range[0] < v_range[1] */
    double mass, p_D, p_L, tau;  /* > 0 (p_D, p_L >= 0) */
    int32_t steps;          /* integration steps per sampling period, 1..64 */
    int32_t n_thrust, n_bank;  /* >= 1, K = n_thrust * n_bank <= 255 */
    double thrust_max, bank_max_deg;  /* >= 0; bank_max_deg < 90 */
    const gbf_ac_box* target; int32_t n_target;  /* host arrays, <= 16 boxes each */
    const gbf_ac_box* avoid; int32_t n_avoid;
    const gbf_ac_box* reward; int32_t n_reward;
    float reward_cost;      /* finite */
    const float* G;         /* device [n] or NULL */
    int32_t pair_ids64;     /* 1 = 64-bit pair ids at any size; 0 = by size (n K >= 2^31) */
} gbf_aircraft;

/* The enclosure table: table (device int32 [dims[3] * dims[2] * K * 8]) gets,
 * at ((i4 dims[2] + i3) K + u) * 8, the cells met by the enclosure of the
 * cell (0, 0, i3, i4) moved by the input u: x1 and x2 cell offsets
 * (lo, hi), heading cells (lo, hi, not reduced mod dims[2]), speed cells
 * (lo, hi; outside [0, dims[3]) the set leaves the speed range).
 * Synchronises the stream.  Errors: GBF_EINVAL (bad scenario, or an
 * enclosure without an a priori enclosure: its ranges are then empty),
 * GBF_ENOMEM, GBF_EHIP. */
int gbf_aircraft_table(const gbf_aircraft* a, int32_t* table, void* hip_stream);
/* Builds the abstraction on the device and returns a handle for gbf_solve
 * (host-loop mode, plain order, one instance; 64-bit pair ids when
 * n K >= 2^31) and gbf_extract_policy.  Device memory: about 6 bytes per
 * state, 2 bytes per pair for the solver's frontiers, the table and its
 * reverse rows; no per-pair images.  The scenario is read during the call
 * only.  Errors: GBF_EINVAL (bad scenario; table offsets beyond +-127
 * cells; an enclosure not found), GBF_ENOMEM, GBF_EHIP. */
int gbf_load_aircraft(const gbf_aircraft* a, void* hip_stream, gbf_graph** out);

/* Message for the last failing call of this thread ("" if none). */
const char* gbf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GBF_H */
