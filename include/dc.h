/*
 * dc.h -- C ABI of the MI355X (gfx950) library for Delta-screening incremental
 * dynamic community detection (Zarayeneh & Kalyanaraman, "A Fast and
 * Efficient Incremental Approach toward Dynamic Community Detection",
 * arXiv 1904.08553).
 *
 * Problem (Sec. 3.2, Definition 3.1): given a dynamic graph G_1..G_T, report
 * at every time step a partition C_t of the vertices that maximises the
 * modularity Q_t of Eq. (1).  The incremental procedure of Sec. 3.4 is
 * followed: Static(G_1) at t = 1, and for t > 1 the previous labels are
 * inherited, Delta-screening (Alg. 2, Sec. 3.5) selects R_t from the batch,
 * and the multi-level local-moving method (Alg. 1) evaluates only R_t at its
 * first level.
 *
 * Conventions
 *   - Every call returns a dc_status: 0 on success, a negative code on error.
 *     No call throws.  A failing dc_apply_batch leaves the context exactly as
 *     it was (checks run before anything is changed) except DC_E_DEVICE, after
 *     which the context refuses further work with DC_E_STATE.
 *   - Vertices are int32 ids in [0, n); n is fixed by dc_init.  Edges are
 *     undirected, without self-loops, with int32 weights >= 1.  The total
 *     weight 2m must stay below 2^31, so every gain fits int64 exactly.
 *   - Pointer arguments are borrowed for the duration of the call only; the
 *     context owns all device memory it allocates (hipMalloc) and frees it in
 *     dc_destroy.  Input arrays may live on the host or on the device
 *     (dc_edges.on_device).  All device work is enqueued on the stream given
 *     in dc_options.stream (a hipStream_t; NULL = the default stream) and
 *     every call returns after its results are written (stream-synchronous).
 *   - One context per host thread at a time.
 */
#ifndef DC_H
#define DC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dc_status;

enum {
  DC_OK = 0,
  DC_E_ARG = -1,       /* null pointer, bad size or bad option            */
  DC_E_RANGE = -2,     /* a vertex id outside [0, n)                       */
  DC_E_SELF_LOOP = -3, /* an edge (v, v)                                   */
  DC_E_WEIGHT = -4,    /* an insertion weight < 1                          */
  DC_E_NO_EDGE = -5,   /* a deletion of an edge absent from G_{t-1}        */
  DC_E_DUP = -6,       /* the same undirected pair deleted twice           */
  DC_E_OVERFLOW = -7,  /* 2m would reach 2^31                              */
  DC_E_OOM = -8,       /* device allocation failed                         */
  DC_E_DEVICE = -9,    /* a HIP call failed; the context is poisoned       */
  DC_E_STATE = -10,    /* the context was poisoned by an earlier failure   */
  DC_PENDING = 1       /* dc_server_poll: the batch has not finished (not
                          an error)                                       */
};

/* How the first level chooses its start partition and its active set. */
enum {
  DC_MODE_DELTA = 0,  /* inherit C_{t-1}; level 0 visits R_t from Alg. 2 */
  DC_MODE_ALL = 1,    /* inherit C_{t-1}; level 0 visits every vertex (the
                         baseline of Sec. 3.4 with R_t = V_t)            */
  DC_MODE_STATIC = 2, /* restart from singletons (naive rerun, Sec. 3.3)  */
  DC_MODE_LEARNED = 3 /* inherit C_{t-1}; level 0 visits the touched
                         vertices whose screener logit is >= theta (see
                         dc_screener_set); plain Alg. 2 while no screener
                         is set                                          */
};

/* The multi-level method Delta-screening is plugged into (Sec. 3.4: the
 * paper modifies both).  LOUVAIN: levels of Alg. 1 (local moving, then
 * compaction by the communities).  SLM: smart local moving (the paper's
 * reference [waltman2013smart]): after the local moving of a level every
 * community is refined (local moving from singletons on the subgraph it
 * induces, with the whole graph's vertex weights), the level graph is
 * compacted by the refined communities and the next level starts from the
 * unrefined ones; levels continue while the compaction reduces the graph.
 * Delta-screening restricts the first local moving of level 0 to R_t in
 * both (dLouvain-DS, dSLM-DS); MODE_ALL gives dLouvain-base / dSLM-base. */
enum {
  DC_ALGO_LOUVAIN = 0,
  DC_ALGO_SLM = 1
};

/* Deletions are outside the paper (Sec. 5 lists them as future work). */
enum {
  DC_DEL_GAIN = 0,        /* a source of an intra-community deletion joins R
                             with Gamma(i) and its best community only when
                             its best move has a positive gain              */
  DC_DEL_CONSERVATIVE = 1 /* every such source joins R with Gamma(i)       */
};

typedef struct dc_options {
  int32_t mode;            /* DC_MODE_*; default DELTA                       */
  int32_t max_levels;      /* >= 1; default 32 (levels 0..max_levels-1)     */
  int32_t max_sweeps;      /* >= 1 sweeps per level; default 100            */
  int32_t singleton_guard; /* 1: two singletons merge only toward the
                              smaller label; default 1                      */
  int32_t del_rule;        /* DC_DEL_*; default GAIN                         */
  int32_t timing;          /* 1: time the level sweeps with hipEvents and
                              report them in dc_step_stats                  */
  int64_t tau_den;         /* a sweep gaining at most floor((2m)^2/tau_den)
                              in the exact numerator ends the level (the
                              threshold tau of Sec. 3.2); 0 = threshold 0;
                              default 10^6                                 */
  void* stream;            /* hipStream_t for all work; NULL = default       */
  int32_t collect;         /* 1: every dc_apply_batch also records screener
                              samples (dc_last_samples): features of the
                              touched vertices and their move labels under a
                              full re-evaluation of level 0; default 0      */
  int32_t full_coarsen;    /* 1: build every level-0 compaction from all of
                              G_t; 0 (default): from the previous step's
                              graph of communities, the batch's changes and
                              the level-0 movers' rows (same result)       */
  int64_t cascade_num;     /* cascade-aware screening (an extension for the
                              indirect effect noted after the proof of
                              Lemma 3.2): with cascade_den > 0 and theta =
                              cascade_num / cascade_den, every neighbour v of
                              an accepted addition source i with
                              C_{t-1}(v) = C_{t-1}(i) whose best move to
                              another neighbouring community has scaled gain
                              G1(v) >= -theta * 2m * k_v adds v and its
                              neighbours to R_t (DELTA and the screening pass
                              of LEARNED / collect); both >= 0              */
  int64_t cascade_den;     /* 0 (default): no cascade                        */
  int32_t algorithm;       /* DC_ALGO_*; default LOUVAIN                      */
  int32_t reserved;        /* must be zero                                   */
} dc_options;

/* An edge list: count entries (u[e], v[e], w[e]).  w is ignored (may be
 * NULL) for deletions.  on_device = 1 when the arrays are device pointers. */
typedef struct dc_edges {
  int64_t count;
  const int32_t* u;
  const int32_t* v;
  const int32_t* w;
  int32_t on_device;
  int32_t pad;
} dc_edges;

/* One record per executed synchronous sweep of the last call. */
typedef struct dc_sweep_rec {
  int32_t level;     /* 0 = the input graph                                */
  int32_t sweep;     /* index within the level                             */
  int32_t n_level;   /* vertices of the level graph                        */
  int32_t n_active;  /* vertices evaluated in the sweep                    */
  int64_t nnz_level; /* stored (directed) entries of the level graph       */
  int64_t moves;     /* vertices that changed community                    */
  int64_t dN;        /* exact change of N = 2m*I - sum a^2 (Q = N/(2m)^2)  */
  int32_t kept;      /* 1 applied, 0 reverted (dN < 0) or no move          */
  int32_t phase;     /* 0 local moving; 1 SLM refinement (local moving from
                        singletons inside each community; n_active = all,
                        nnz_level = entries inside communities)          */
} dc_sweep_rec;

typedef struct dc_step_stats {
  int64_t changes;        /* insertions + deletions of the batch            */
  int64_t R_size;         /* |R_t| (n for ALL and STATIC)                   */
  int64_t ds_sources;     /* addition sources examined by Alg. 2            */
  int64_t ds_accepted;    /* sources whose test passed                      */
  int64_t del_sources;    /* sources of intra-community deletions           */
  int64_t del_accepted;
  int32_t levels;         /* levels run                                     */
  int32_t sweeps;         /* sweeps run over all levels                     */
  int64_t moves;          /* vertex moves kept over all levels              */
  int64_t vertex_evals;   /* vertex-gain evaluations (active vertices summed
                             over sweeps, plus Alg. 2 sources)              */
  int64_t N;              /* exact numerator of Q_t                         */
  int64_t two_m;          /* 2m of G_t                                      */
  double q;               /* N / (2m)^2                                     */
  double ms_total;        /* host wall time of the call                     */
  double ms_sweep_kernel; /* device time of the sweep kernel for rows of at
                             most 64 entries (one launch per sweep), summed
                             over its launches; timing = 1 only            */
  int64_t sweep_launches; /* launches of that kernel timed                  */
  int64_t sweep_bytes;    /* their algorithmic bytes: 12 per adjacency entry
                             and 32 per evaluated vertex                    */
  int64_t level0_sweeps;  /* sweeps at level 0                              */
  int64_t level0_active;  /* active vertices summed over level-0 sweeps     */
  int64_t level0_volume;  /* adjacency entries of active vertices, summed
                             over level-0 sweeps                            */
  int64_t touched;        /* touched vertices of the batch (LEARNED mode or
                             collect = 1), else 0                          */
  int64_t screened;       /* 1 when the screener network chose R_t         */
  int64_t cascade_candidates; /* same-community neighbours of accepted
                                 addition sources examined by the cascade  */
  int64_t cascade_expanded;   /* those whose neighbourhood joined R_t      */
  /* timing = 1, dc_apply_batch only: device time (hipEvents on the call's
     stream) and algorithmic HBM bytes of the step's phases:
       [0] batch ingest and graph update: 12 B per change read + 16 B per
           change placed as two directed entries (the merge's rewrite of
           the whole CSR is implementation traffic, not counted);
       [1] screening (DELTA): 12 B per entry of the screened vertices' rows
           + 32 B per screened vertex + 20 B per insertion record (the
           gain2 of the mirror record) + 8 B per entry of the accepted
           sources' rows + 5 B per vertex and 4 B per member of R_t;
       [2] level-0 sweeps: 12 B per entry of the evaluated rows + 32 B per
           evaluated vertex (apply and Delta N included in the time);
       [3] compaction, levels >= 1 and the canonical labels: 12 B per entry
           and 32 B per vertex of every sweep above level 0 + 12 B per
           level-0 vertex for the labels.                               */
  double ms_phase[4];
  int64_t bytes_phase[4];
  int64_t screen_volume;      /* entries of the screened vertices' rows      */
  int64_t screen_vertices;    /* vertices the screening pass evaluated       */
  int64_t accepted_volume;    /* entries of the accepted sources' rows       */
} dc_step_stats;

typedef struct dc_ctx dc_ctx;

/* Defaults as documented in dc_options. */
void dc_default_options(dc_options* opt);

/* Builds G_1 on n vertices from g1 (duplicate pairs sum their weights) and
 * runs Static(G_1) (Sec. 3.4 step 1): Alg. 1 from singletons with every
 * vertex active.  *out receives the context; C_1 is read with
 * dc_communities.  Errors: ARG, RANGE, SELF_LOOP, WEIGHT, OVERFLOW, OOM,
 * DEVICE. */
dc_status dc_init(dc_ctx** out, int32_t n, const dc_edges* g1,
                  const dc_options* opt);

/* One time step (Sec. 3.4 step 2): deletions `del` are removed first (each
 * must exist in G_{t-1}), then insertions `add` are added (weights sum onto
 * an existing edge).  Either list may be NULL or empty.  Then R_t is chosen
 * per the mode (Alg. 2 for DELTA), the levels run from the inherited labels,
 * and the canonical labels C_t (each community labelled by its smallest
 * vertex id) are written to C_out[n] when C_out is not NULL (device memory
 * when out_on_device = 1).  stats may be NULL.  Checks, in this order, over
 * the whole batch: RANGE, SELF_LOOP, WEIGHT, DUP, NO_EDGE, OVERFLOW. */
dc_status dc_apply_batch(dc_ctx* ctx, const dc_edges* add, const dc_edges* del,
                         int32_t* C_out, int32_t out_on_device,
                         dc_step_stats* stats);

/* Modularity Q_t of Eq. (1) for the current (G_t, C_t), computed from its
 * definition over the whole graph: q = N / (2m)^2 with the exact int64
 * numerator N = 2m * sum_i e_{i->C(i)} - sum_C a_C^2.  Any pointer may be
 * NULL.  2m = 0 gives q = 0. */
dc_status dc_modularity(dc_ctx* ctx, double* q, int64_t* num, int64_t* two_m);

/* Current canonical labels into out[n] (device memory when on_device). */
dc_status dc_communities(dc_ctx* ctx, int32_t* out, int32_t on_device);

/* R_t of the last dc_apply_batch as n bytes of 0/1 (all ones after dc_init). */
dc_status dc_last_R(dc_ctx* ctx, uint8_t* out, int32_t on_device);

/* Sweep records of the last dc_init / dc_apply_batch: up to cap records are
 * copied to out; *count receives the total number of sweeps. */
dc_status dc_last_trace(dc_ctx* ctx, dc_sweep_rec* out, int32_t cap,
                        int32_t* count);

/* Statistics of the last dc_init / dc_apply_batch. */
dc_status dc_last_stats(dc_ctx* ctx, dc_step_stats* out);

/* Number of stored directed entries of G_t (2 per undirected edge). */
dc_status dc_num_entries(dc_ctx* ctx, int64_t* nnz);

/* G_t as a CSR in host memory: off[n+1] (int64), col[nnz], w[nnz]; rows are
 * sorted by neighbour id. */
dc_status dc_export_csr(dc_ctx* ctx, int64_t* off, int32_t* col, int32_t* w);

void dc_destroy(dc_ctx* ctx);

/* Device memory of the library comes from a block cache: buffers released by
 * dc_destroy (and by buffers that grow) stay cached and are handed to later
 * contexts before hipMalloc is called.  This call frees every cached block
 * (after one wait for each device that released a block); memory held by
 * live contexts is untouched.  The cache is also freed when a served graph
 * is evicted to host memory and when hipMalloc reports no memory (the
 * allocation is then tried once more).  Call it from no thread that is
 * stepping a context at the same time. */
void dc_trim_device_cache(void);

/* Checkpoint of a context: G_t as a CSR in host memory (as dc_export_csr,
 * sizes from dc_num_entries) and C_t[n]. */
dc_status dc_export_state(dc_ctx* ctx, int64_t* off, int32_t* col, int32_t* w,
                          int32_t* C);

/* A context resumed from a checkpoint (host memory): G_t as a CSR with rows
 * sorted by neighbour, symmetric, no self-loops, weights >= 1, 2m < 2^31;
 * C[n] a canonical labelling (C[C[v]] == C[v] <= v).  No levels run; the
 * next dc_apply_batch continues from (G_t, C_t) as the original context
 * would.  Errors: ARG (malformed checkpoint), OVERFLOW, OOM, DEVICE. */
dc_status dc_init_from_state(dc_ctx** out, int32_t n, const int64_t* off,
                             const int32_t* col, const int32_t* w,
                             const int32_t* C, const dc_options* opt);

/* ---- Serving many dynamic graphs (an extension: the paper treats one) ----
 *
 * A server keeps many graphs' state resident on one GPU and applies the
 * batches submitted for them with continuous batching: a worker thread
 * takes, round after round, the oldest waiting batch of up to max_inflight
 * distinct graphs (each graph's batches in submission order); batches that
 * arrive meanwhile join a later round.  In a round the graphs' level-0
 * sweeps run merged: one evaluation launch per row-length bin covers every
 * graph still sweeping (a graph leaves when its level stops), so the
 * graphs' work shares the device.  Each result equals that of the graph's
 * own context run alone.  Admission: a graph's device footprint (bytes of
 * all its buffers) counts against budget_bytes while resident; to admit a
 * graph the server moves idle graphs' state to host memory (least recently
 * used first) and brings it back when their next batch runs; a batch whose
 * graph cannot fit yet waits.  budget_bytes <= 0: no limit.  The options
 * (stream ignored: the server owns one stream) apply to every graph. */
typedef struct dc_server dc_server;

typedef struct dc_server_stats {
  int64_t graphs;          /* graphs added                                    */
  int64_t batches;         /* batches finished                                */
  int64_t rounds;          /* rounds run                                      */
  int64_t merged_rounds;   /* rounds with more than one graph                 */
  int64_t merged_graphs;   /* graphs summed over rounds                       */
  int64_t evictions;       /* graph states moved to host memory               */
  int64_t restores;        /* graph states brought back                       */
  int64_t deferred;        /* times a batch waited for memory                 */
  int64_t resident_bytes;  /* device bytes of resident graphs now             */
  int64_t peak_resident_bytes;
  int64_t reserved[6];
} dc_server_stats;

dc_status dc_server_create(dc_server** out, const dc_options* opt,
                           int64_t budget_bytes, int32_t max_inflight);
/* Adds a graph: builds G_1 and runs Static(G_1) as dc_init; blocks until
 * done; *gid receives its id (0, 1, ...).  Errors as dc_init; OOM when the
 * graph alone exceeds the budget. */
dc_status dc_server_add_graph(dc_server* s, int32_t n, const dc_edges* g1,
                              int32_t* gid);
/* Queues a batch (copied) for graph gid; arrival_ns is the caller's
 * CLOCK_MONOTONIC time of arrival (for latency); *ticket identifies it. */
dc_status dc_server_submit(dc_server* s, int32_t gid, const dc_edges* add,
                           const dc_edges* del, int64_t arrival_ns,
                           int64_t* ticket);
/* Result of a batch: DC_PENDING while it has not finished (wait = 0), else
 * the batch's own status; on DC_OK, C_out[n] (host, nullable) receives
 * C_t, stats (nullable) its statistics, times[3] (nullable) its arrival,
 * start and finish (CLOCK_MONOTONIC ns).  A finished ticket is released by
 * this call. */
dc_status dc_server_poll(dc_server* s, int64_t ticket, int32_t wait,
                         int32_t* C_out, dc_step_stats* stats, int64_t* times);
dc_status dc_server_stats_get(dc_server* s, dc_server_stats* out);
/* Finishes the queued batches, then frees everything. */
void dc_server_destroy(dc_server* s);

/* ---- Learned screener (an extension; the paper has no learned part) ----
 *
 * A vertex is touched by a batch when it is an endpoint of a changed pair, a
 * neighbour in G_t of such an endpoint, or in the set Alg. 2 (plus the
 * deletion rule) selects.  Its eight features, computed on (G_t, C_{t-1},
 * community totals on G_t) from exact integers, each one correctly rounded
 * fp64 division, then rounded to bfloat16 (to fp32, then to nearest even):
 *   x0 = k/(k+16)        k: weighted degree in G_t
 *   x1 = (k-kp)/max(k,kp), 0 when both are 0; kp: degree in G_{t-1}
 *   x2 = t/(t+4)         t: changed pairs at the vertex
 *   x3 = e_own/k         e_own = e_{i->C(i)} (0 when k = 0)
 *   x4 = G1/(2m*k)       G1: scaled gain (Sec. 3.1) to the best other
 *                        neighbouring community (score descending, label
 *                        ascending); -3 when there is none
 *   x5 = G2/(2m*k)       the same for the second best; -3 when none
 *   x6 = 1 if Alg. 2 (or the deletion rule) selected the vertex, else 0
 *   x7 = a_{C(i)}/2m     (0 when 2m = 0)
 * The move label of a touched vertex is 1 when it ends level 0 in another
 * community if level 0 is run from C_{t-1} with every vertex active.
 *
 * The network: 8 -> 64 -> 64 -> 1, ReLU, ReLU, logit (sigmoid score), with
 * DC_MLP_PARAMS fp32 parameters in one flat vector
 *   W1[64][8] | b1[64] | W2[64][64] | b2[64] | w3[64] | b3
 * (row = output unit).  Device compute rounds every parameter and every
 * activation or back-propagated signal entering a matrix product to
 * bfloat16 and accumulates in fp32 on the matrix cores. */
#define DC_MLP_INPUTS 8
#define DC_MLP_HIDDEN 64
#define DC_MLP_PARAMS 4801

/* Sets (w != NULL: DC_MLP_PARAMS host floats, copied) or clears (w = NULL)
 * the screener of a context.  In LEARNED mode R_t becomes the touched
 * vertices whose logit is >= theta.  Setting a screener also allocates the
 * per-vertex buffers of the scoring pass (about 60 bytes per vertex), so
 * the first scored batch does not. */
dc_status dc_screener_set(dc_ctx* ctx, const float* w, float theta);

/* Samples of the last dc_apply_batch (LEARNED mode or collect = 1): *count
 * receives the number of touched vertices; then, for every non-NULL output
 * (device memory when on_device = 1): ids[count] (ascending vertex ids),
 * X[count][8] bfloat16 bit patterns, y[count] move labels (0/1; collect = 1
 * only, else ARG), logits[count] (when the screener scored the batch, else
 * ARG).  *count = 0 when nothing was recorded. */
dc_status dc_last_samples(dc_ctx* ctx, int64_t* count, int32_t* ids,
                          uint16_t* X, uint8_t* y, float* logits,
                          int32_t on_device);

/* A trainable copy of the network on the device: fp32 master parameters,
 * Adam moments (beta1 0.9, beta2 0.999, eps 1e-8) and the bfloat16 copy the
 * kernels read.  All work goes to `stream` (hipStream_t, NULL = default);
 * calls return after their results are written. */
typedef struct dc_mlp dc_mlp;

dc_status dc_mlp_create(dc_mlp** out, const float* w, void* stream);
dc_status dc_mlp_set_weights(dc_mlp* m, const float* w);  /* resets Adam */
dc_status dc_mlp_get_weights(dc_mlp* m, float* w);
/* logits[n] (device) of X[n][8] (device, bfloat16 bit patterns). */
dc_status dc_mlp_forward(dc_mlp* m, const uint16_t* X, int64_t n, float* logits);
/* Mean binary cross-entropy over the n samples (labels y[n] on the device,
 * 0/1; positives weighted by pos_weight > 0) and its gradient, into the host
 * arrays grad[DC_MLP_PARAMS] and *loss (either may be NULL).  No update. */
dc_status dc_mlp_grad(dc_mlp* m, const uint16_t* X, const uint8_t* y, int64_t n,
                      float pos_weight, float* grad, double* loss);
/* dc_mlp_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the same kernels, the same result bit for bit, but the
 * per-block partial sums and the reduced gradient live in a fixed device
 * array of the library (2.5 MB per device: 128 blocks of DC_MLP_PARAMS + 1
 * floats plus the gradient), held by each device the library runs on until
 * the process ends; nothing is allocated.  The gradient kernel launches at
 * most 128 blocks for any n, so every n >= 1 fits; a scratch need above the
 * array would be rejected with DC_E_ARG (dc_last_error names the sizes).
 * Inputs and outputs as dc_mlp_grad (X, y on the device; grad, loss on the
 * host, either may be NULL).  All calls on one device share that array:
 * calls that overlap on one device (other host threads, other streams)
 * race and must be serialised by the caller. */
dc_status dc_mlp_grad_noalloc(dc_mlp* m, const uint16_t* X, const uint8_t* y, int64_t n,
                              float pos_weight, float* grad, double* loss);
/* One Adam step of learning rate lr on the same loss; *loss (may be NULL)
 * receives the loss before the step. */
dc_status dc_mlp_train_step(dc_mlp* m, const uint16_t* X, const uint8_t* y,
                            int64_t n, float pos_weight, float lr, double* loss);
void dc_mlp_destroy(dc_mlp* m);

const char* dc_strerror(dc_status s);

/* Text of the last HIP failure seen by a call on this host thread (the failing
 * call, its error string and source location); "" if none.  The pointer stays
 * valid until the next call on the same thread. */
const char* dc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
