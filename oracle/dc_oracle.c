/*
 * dc_oracle.c -- plain single-threaded CPU oracle for Delta-screening
 * incremental dynamic community detection (arXiv 1904.08553).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no code
 * with the HIP library.
 *
 * Everything is int64 and recomputed from definitions where that is cheap
 * enough to stay obvious: community totals a_C and sizes are rebuilt from the
 * labels before every sweep, and the exact modularity numerator N is
 * recomputed over the whole level graph after every sweep.
 *
 * Paper passages followed:
 *   Sec. 3.1 notation and Eq. (1) ............ csr_numerator
 *   Sec. 3.1 gain, Appendix A algebra ........ score / csr_gain
 *   Sec. 3.2 Louvain move rule ............... decide
 *   Sec. 3.2 Alg. 1 (sweeps, compaction) ..... level_sweeps, coarsen, run_levels
 *   Sec. 3.4 SLM host (dSLM) ................. induced, run_levels_slm
 *   Sec. 3.4 incremental procedure ........... orc_stage_batch / orc_finish_batch
 *   learned screener samples (extension) ..... collect_samples, features_of
 *   Sec. 3.5 Alg. 2 (Delta-screening) ........ screen_additions
 *   deletions (paper: future work, Sec. 5) ... screen_deletions
 */
#include "dc_oracle.h"

#include <stdlib.h>
#include <string.h>

#define TWO_M_LIMIT ((int64_t)1 << 31)

/* ------------------------------------------------------------------------ */
/* CSR level graph (immutable within a level).  Diagonal entries allowed.     */

typedef struct {
  int32_t n;
  int64_t nnz;
  int64_t* off; /* n+1 */
  int32_t* col; /* nnz */
  int64_t* w;   /* nnz */
} csr_t;

static void csr_free(csr_t* g) {
  free(g->off);
  free(g->col);
  free(g->w);
  memset(g, 0, sizeof(*g));
}

/* Weighted degree k_u = sum of the row, diagonal included (Sec. 3.1). */
static void csr_degrees(const csr_t* g, int64_t* k) {
  for (int32_t u = 0; u < g->n; ++u) {
    int64_t s = 0;
    for (int64_t e = g->off[u]; e < g->off[u + 1]; ++e) s += g->w[e];
    k[u] = s;
  }
}

static int64_t csr_two_m(const csr_t* g) {
  int64_t s = 0;
  for (int64_t e = 0; e < g->nnz; ++e) s += g->w[e];
  return s;
}

/* Exact numerator of Eq. (1): Q = N / (2m)^2 with
 *   N = 2m * sum_i e_{i->C(i)} - sum_C a_C^2,
 * where sum_i e_{i->C(i)} counts every ordered intra-community pair (and the
 * diagonal of a coarse vertex, which already holds both orientations). */
static int64_t csr_numerator(const csr_t* g, const int32_t* C, int64_t two_m,
                             const int64_t* k, int64_t* a_scratch) {
  int64_t I = 0;
  for (int32_t u = 0; u < g->n; ++u)
    for (int64_t e = g->off[u]; e < g->off[u + 1]; ++e)
      if (C[g->col[e]] == C[u]) I += g->w[e];
  for (int32_t x = 0; x < g->n; ++x) a_scratch[x] = 0;
  for (int32_t u = 0; u < g->n; ++u) a_scratch[C[u]] += k[u];
  int64_t S = 0;
  for (int32_t x = 0; x < g->n; ++x) S += a_scratch[x] * a_scratch[x];
  return two_m * I - S;
}

/* ------------------------------------------------------------------------ */
/* Neighbour-community aggregation e_{i->X} with a dense accumulator.       */

typedef struct {
  int64_t* acc;
  uint8_t* seen;
  int32_t* touched;
  int32_t nt;
} agg_t;

static int agg_alloc(agg_t* ag, int32_t n) {
  ag->acc = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  ag->seen = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  ag->touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  ag->nt = 0;
  return ag->acc && ag->seen && ag->touched;
}

static void agg_free(agg_t* ag) {
  free(ag->acc);
  free(ag->seen);
  free(ag->touched);
}

/* e_{i->X} for every community X adjacent to i; the diagonal entry of i is
 * skipped (it stays inside i's community whatever i does). */
static void aggregate(const csr_t* g, const int32_t* C, int32_t i, agg_t* ag) {
  for (int64_t e = g->off[i]; e < g->off[i + 1]; ++e) {
    int32_t v = g->col[e];
    if (v == i) continue;
    int32_t X = C[v];
    if (!ag->seen[X]) {
      ag->seen[X] = 1;
      ag->touched[ag->nt++] = X;
    }
    ag->acc[X] += g->w[e];
  }
}

static void agg_clear(agg_t* ag) {
  for (int32_t t = 0; t < ag->nt; ++t) {
    ag->acc[ag->touched[t]] = 0;
    ag->seen[ag->touched[t]] = 0;
  }
  ag->nt = 0;
}

/* score(X) = 2m*e_{i->X} - k_i*a_X^{(-i)}; a^{(-i)} removes i from its own
 * community.  G(i->D) = score(D) - score(C(i)) and applying that single move
 * changes N by exactly 2G (the Appendix A gain times 2(2m)^2). */
static int64_t score(int64_t two_m, int64_t e, int64_t ki, int64_t aX,
                     int own) {
  return two_m * e - ki * (own ? aX - ki : aX);
}

/* Louvain local decision (Sec. 3.2): best neighbouring community by gain,
 * ties to the smallest label, move only on a strictly positive gain; with the
 * guard on, two singletons merge only toward the smaller label. */
static int32_t decide(const csr_t* g, const int32_t* C, const int64_t* a,
                      const int64_t* size, const int64_t* k, int64_t two_m,
                      int32_t i, int guard, agg_t* ag, int64_t* best_gain) {
  int32_t c = C[i];
  int64_t ki = k[i];
  *best_gain = 0;
  if (ki == 0) return c;
  aggregate(g, C, i, ag);
  int64_t e_c = ag->seen[c] ? ag->acc[c] : 0;
  int64_t s_own = score(two_m, e_c, ki, a[c], 1);
  int32_t best = -1;
  int64_t bs = 0;
  for (int32_t t = 0; t < ag->nt; ++t) {
    int32_t X = ag->touched[t];
    if (X == c) continue;
    int64_t s = score(two_m, ag->acc[X], ki, a[X], 0);
    if (best < 0 || s > bs || (s == bs && X < best)) {
      best = X;
      bs = s;
    }
  }
  agg_clear(ag);
  if (best < 0) return c;
  *best_gain = bs - s_own;
  if (bs <= s_own) return c;
  if (guard && size[c] == 1 && size[best] == 1 && best > c) return c;
  return best;
}

static void totals(const csr_t* g, const int32_t* C, const int64_t* k,
                   int64_t* a, int64_t* size) {
  for (int32_t x = 0; x < g->n; ++x) {
    a[x] = 0;
    size[x] = 0;
  }
  for (int32_t u = 0; u < g->n; ++u) {
    a[C[u]] += k[u];
    size[C[u]] += 1;
  }
}

/* ------------------------------------------------------------------------ */
/* Synchronous sweeps of one level (Alg. 1 inner loop).                      */

typedef struct {
  orc_sweep_rec* recs;
  int32_t cap;
  int32_t count;
} trace_t;

static void trace_push(trace_t* tr, const orc_sweep_rec* r) {
  if (tr && tr->count < tr->cap && tr->recs) tr->recs[tr->count] = *r;
  if (tr) tr->count++;
}

/* Runs sweeps over the active vertices; C is updated in place.  Returns the
 * total exact Delta N of the kept sweeps. */
static int64_t level_sweeps(const csr_t* g, int64_t two_m, int64_t T,
                            int32_t* C, const uint8_t* active,
                            const orc_options* opt, int32_t level,
                            trace_t* tr, int* oom, const int64_t* k_ext,
                            int32_t phase) {
  int32_t n = g->n;
  size_t nn = (size_t)(n > 0 ? n : 1);
  int64_t* k = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* a = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* size = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* a2 = (int64_t*)malloc(sizeof(int64_t) * nn);
  int32_t* C2 = (int32_t*)malloc(sizeof(int32_t) * nn);
  agg_t ag;
  int ok = k && a && size && a2 && C2 && agg_alloc(&ag, n);
  int64_t total = 0;
  if (!ok) {
    *oom = 1;
    goto done;
  }
  /* k_ext: the vertex weights of a larger graph g is a part of (SLM
   * refinement: degrees in the whole level graph) */
  if (k_ext)
    memcpy(k, k_ext, sizeof(int64_t) * nn);
  else
    csr_degrees(g, k);
  int32_t n_active = 0;
  for (int32_t u = 0; u < n; ++u) n_active += active[u] ? 1 : 0;
  int64_t N0 = csr_numerator(g, C, two_m, k, a2);
  for (int32_t s = 0; s < opt->max_sweeps; ++s) {
    totals(g, C, k, a, size);
    memcpy(C2, C, sizeof(int32_t) * nn);
    int64_t moves = 0;
    for (int32_t i = 0; i < n; ++i) {
      if (!active[i]) continue;
      int64_t bg;
      int32_t d = decide(g, C, a, size, k, two_m, i, opt->singleton_guard,
                         &ag, &bg);
      if (d != C[i]) {
        C2[i] = d;
        moves++;
      }
    }
    int64_t N1 = moves ? csr_numerator(g, C2, two_m, k, a2) : N0;
    int64_t dN = N1 - N0;
    orc_sweep_rec r;
    memset(&r, 0, sizeof(r));
    r.level = level;
    r.sweep = s;
    r.n_level = n;
    r.n_active = n_active;
    r.nnz_level = g->nnz;
    r.moves = moves;
    r.dN = dN;
    r.kept = (moves > 0 && dN >= 0) ? 1 : 0;
    r.phase = phase;
    trace_push(tr, &r);
    if (moves == 0) break;
    if (dN < 0) break; /* revert: C keeps the snapshot, the level ends */
    memcpy(C, C2, sizeof(int32_t) * nn);
    N0 = N1;
    total += dN;
    if (dN <= T) break;
  }
  agg_free(&ag);
done:
  free(k);
  free(a);
  free(size);
  free(a2);
  free(C2);
  return total;
}

/* ------------------------------------------------------------------------ */
/* Compaction (Alg. 1): one coarse vertex per non-empty community, numbered by
 * ascending label; A'_{XY} = sum of A_uv over u in X, v in Y (diagonal kept). */

static int coarsen(const csr_t* g, const int32_t* C, int32_t* rank,
                   csr_t* out) {
  int32_t n = g->n;
  size_t nn = (size_t)(n > 0 ? n : 1);
  uint8_t* used = (uint8_t*)calloc(nn, 1);
  if (!used) return 0;
  for (int32_t u = 0; u < n; ++u) used[C[u]] = 1;
  int32_t nc = 0;
  for (int32_t x = 0; x < n; ++x) rank[x] = used[x] ? nc++ : -1;
  free(used);

  /* member lists by coarse vertex (counting sort, ascending member id) */
  int64_t* mstart = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
  int32_t* members = (int32_t*)malloc(sizeof(int32_t) * nn);
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nc + 1));
  agg_t ag;
  int ok = mstart && members && fill && agg_alloc(&ag, nc > 0 ? nc : 1);
  if (!ok) {
    free(mstart);
    free(members);
    free(fill);
    return 0;
  }
  for (int32_t u = 0; u < n; ++u) mstart[rank[C[u]] + 1]++;
  for (int32_t r = 0; r < nc; ++r) mstart[r + 1] += mstart[r];
  for (int32_t r = 0; r <= nc; ++r) fill[r] = mstart[r];
  for (int32_t u = 0; u < n; ++u) members[fill[rank[C[u]]]++] = u;

  /* first pass counts row lengths, second pass fills */
  out->n = nc;
  out->off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nc + 1));
  if (!out->off) ok = 0;
  int64_t nnz = 0;
  for (int pass = 0; pass < 2 && ok; ++pass) {
    if (pass == 1) {
      out->nnz = nnz;
      out->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
      out->w = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
      if (!out->col || !out->w) {
        ok = 0;
        break;
      }
    }
    nnz = 0;
    for (int32_t r = 0; r < nc; ++r) {
      if (pass == 0) out->off[r] = nnz;
      for (int64_t p = mstart[r]; p < mstart[r + 1]; ++p) {
        int32_t u = members[p];
        for (int64_t e = g->off[u]; e < g->off[u + 1]; ++e) {
          int32_t Y = rank[C[g->col[e]]];
          if (!ag.seen[Y]) {
            ag.seen[Y] = 1;
            ag.touched[ag.nt++] = Y;
          }
          ag.acc[Y] += g->w[e];
        }
      }
      /* emit the row sorted by coarse neighbour (insertion sort is fine for
       * an oracle; rows are short relative to the graph) */
      for (int32_t t = 1; t < ag.nt; ++t) {
        int32_t key = ag.touched[t];
        int32_t q = t - 1;
        while (q >= 0 && ag.touched[q] > key) {
          ag.touched[q + 1] = ag.touched[q];
          --q;
        }
        ag.touched[q + 1] = key;
      }
      if (pass == 1)
        for (int32_t t = 0; t < ag.nt; ++t) {
          out->col[nnz + t] = ag.touched[t];
          out->w[nnz + t] = ag.acc[ag.touched[t]];
        }
      nnz += ag.nt;
      agg_clear(&ag);
    }
    if (pass == 0) out->off[nc] = nnz;
  }
  agg_free(&ag);
  free(mstart);
  free(members);
  free(fill);
  return ok;
}

/* ------------------------------------------------------------------------ */
/* Levels (Alg. 1 outer loop) and projection to canonical labels.            */

static int run_levels_slm(const csr_t* g0, int32_t* C0, const uint8_t* active0,
                          const orc_options* opt, trace_t* tr, int32_t* levels_out,
                          int64_t* N_out);

static int run_levels(const csr_t* g0, int32_t* C0, const uint8_t* active0,
                      const orc_options* opt, trace_t* tr, int32_t* levels_out,
                      int64_t* N_out) {
  if (opt->algorithm == ORC_ALGO_SLM)
    return run_levels_slm(g0, C0, active0, opt, tr, levels_out, N_out);
  int32_t n0 = g0->n;
  size_t nn = (size_t)(n0 > 0 ? n0 : 1);
  int64_t two_m = csr_two_m(g0);
  int64_t T = opt->tau_den > 0 ? (two_m * two_m) / opt->tau_den : 0;
  int oom = 0;
  int32_t* map = (int32_t*)malloc(sizeof(int32_t) * nn); /* level-0 -> current */
  int32_t* C = (int32_t*)malloc(sizeof(int32_t) * nn);
  int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * nn);
  uint8_t* all = (uint8_t*)malloc(nn);
  if (!map || !C || !rank || !all) {
    free(map);
    free(C);
    free(rank);
    free(all);
    return 0;
  }
  memset(all, 1, nn);
  for (int32_t v = 0; v < n0; ++v) {
    map[v] = v;
    C[v] = C0[v];
  }
  csr_t cur = *g0; /* borrowed at level 0 */
  int owns = 0;
  int32_t level = 0;
  for (;;) {
    const uint8_t* act = level == 0 ? active0 : all;
    int64_t gain = level_sweeps(&cur, two_m, T, C, act, opt, level, tr, &oom, NULL, 0);
    if (oom) break;
    int stop = (level + 1 >= opt->max_levels) || (level >= 1 && gain <= T);
    if (stop) break;
    csr_t nxt;
    memset(&nxt, 0, sizeof(nxt));
    if (!coarsen(&cur, C, rank, &nxt)) {
      oom = 1;
      break;
    }
    for (int32_t v = 0; v < n0; ++v) map[v] = rank[C[map[v]]];
    if (owns) csr_free(&cur);
    cur = nxt;
    owns = 1;
    for (int32_t x = 0; x < cur.n; ++x) C[x] = x;
    level++;
  }
  if (!oom) {
    /* final community of v is C[map[v]]; its canonical label is the smallest
     * member vertex id (first one met in ascending order). */
    int32_t* lab = rank; /* reuse: indexed by final community (< n0) */
    for (int32_t x = 0; x < n0; ++x) lab[x] = -1;
    for (int32_t v = 0; v < n0; ++v) {
      int32_t f = C[map[v]];
      if (lab[f] < 0) lab[f] = v;
      C0[v] = lab[f];
    }
    if (N_out) {
      int64_t* k = (int64_t*)malloc(sizeof(int64_t) * nn);
      int64_t* a = (int64_t*)malloc(sizeof(int64_t) * nn);
      if (k && a) {
        csr_degrees(g0, k);
        *N_out = csr_numerator(g0, C0, two_m, k, a);
      } else {
        oom = 1;
      }
      free(k);
      free(a);
    }
  }
  if (owns) csr_free(&cur);
  if (levels_out) *levels_out = level + 1;
  free(map);
  free(C);
  free(rank);
  free(all);
  return !oom;
}

/* ------------------------------------------------------------------------ */
/* Levels of the smart local moving method (the paper's second host method,
 * Sec. 3.4; the steps are those of its reference [waltman2013smart]):
 *   1. local moving on the level graph from the level's start partition
 *      (level 0: the inherited partition over the active set R; above: every
 *      vertex), the same synchronous sweeps as Louvain;
 *   2. if every vertex ended alone, or this is the last level allowed, the
 *      partition is final;
 *   3. refinement: inside each community, local moving from singletons on
 *      the subgraph the community induces (every vertex active; vertex
 *      weights and 2m those of the whole level graph, so a move's gain and
 *      the exact Delta N are the whole graph's);
 *   4. compaction of the level graph by the refined communities; if that
 *      does not reduce the graph the partition of step 1 is final;
 *   5. the next level starts from the communities of step 1: every coarse
 *      vertex (a refined community) joins its parent community, labelled by
 *      the smallest coarse id among the parent's refined communities.
 * The final partition of a level-0 vertex is the last level's partition of
 * the coarse vertex it belongs to. */

/* The entries of g inside one community of C (diagonal entries included). */
static int induced(const csr_t* g, const int32_t* C, csr_t* out) {
  int32_t n = g->n;
  out->n = n;
  out->off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!out->off) return 0;
  int64_t nnz = 0;
  for (int32_t u = 0; u < n; ++u) {
    out->off[u] = nnz;
    for (int64_t e = g->off[u]; e < g->off[u + 1]; ++e)
      if (C[g->col[e]] == C[u]) nnz++;
  }
  out->off[n] = nnz;
  out->nnz = nnz;
  out->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  out->w = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  if (!out->col || !out->w) return 0;
  int64_t q = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = g->off[u]; e < g->off[u + 1]; ++e)
      if (C[g->col[e]] == C[u]) {
        out->col[q] = g->col[e];
        out->w[q] = g->w[e];
        q++;
      }
  return 1;
}

static int run_levels_slm(const csr_t* g0, int32_t* C0, const uint8_t* active0,
                          const orc_options* opt, trace_t* tr, int32_t* levels_out,
                          int64_t* N_out) {
  int32_t n0 = g0->n;
  size_t nn = (size_t)(n0 > 0 ? n0 : 1);
  int64_t two_m = csr_two_m(g0);
  int64_t T = opt->tau_den > 0 ? (two_m * two_m) / opt->tau_den : 0;
  int oom = 0;
  int32_t* map = (int32_t*)malloc(sizeof(int32_t) * nn); /* level-0 -> current */
  int32_t* C = (int32_t*)malloc(sizeof(int32_t) * nn);   /* step-1 partition */
  int32_t* Rf = (int32_t*)malloc(sizeof(int32_t) * nn);  /* refined partition */
  int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * nn);
  int32_t* first = (int32_t*)malloc(sizeof(int32_t) * nn);
  int64_t* k = (int64_t*)malloc(sizeof(int64_t) * nn);
  uint8_t* all = (uint8_t*)malloc(nn);
  uint8_t* used = (uint8_t*)malloc(nn);
  if (!map || !C || !Rf || !rank || !first || !k || !all || !used) {
    oom = 1;
    goto out;
  }
  memset(all, 1, nn);
  for (int32_t v = 0; v < n0; ++v) {
    map[v] = v;
    C[v] = C0[v];
  }
  csr_t cur = *g0; /* borrowed at level 0 */
  int owns = 0;
  int32_t level = 0;
  for (;;) {
    /* 1. local moving (R at level 0) */
    const uint8_t* act = (level > 0) ? all : active0;
    (void)level_sweeps(&cur, two_m, T, C, act, opt, level, tr, &oom, NULL, 0);
    if (oom) break;
    /* 2. every vertex alone, or no level left */
    memset(used, 0, nn);
    int32_t ncomm = 0;
    for (int32_t u = 0; u < cur.n; ++u)
      if (!used[C[u]]) {
        used[C[u]] = 1;
        ncomm++;
      }
    if (ncomm == cur.n || level + 1 >= opt->max_levels) break;
    /* 3. refinement inside each community, from singletons */
    csr_t sub;
    memset(&sub, 0, sizeof(sub));
    if (!induced(&cur, C, &sub)) {
      csr_free(&sub);
      oom = 1;
      break;
    }
    csr_degrees(&cur, k);
    for (int32_t u = 0; u < cur.n; ++u) Rf[u] = u;
    (void)level_sweeps(&sub, two_m, T, Rf, all, opt, level, tr, &oom, k, 1);
    csr_free(&sub);
    if (oom) break;
    /* 4. compaction by the refined communities */
    csr_t nxt;
    memset(&nxt, 0, sizeof(nxt));
    if (!coarsen(&cur, Rf, rank, &nxt)) {
      oom = 1;
      break;
    }
    if (nxt.n == cur.n) {
      csr_free(&nxt);
      break;
    }
    /* 5. start partition of the next level: the parent communities */
    for (int32_t x = 0; x < cur.n; ++x) first[x] = -1;
    for (int32_t u = 0; u < cur.n; ++u) {
      int32_t y = rank[Rf[u]];
      if (first[C[u]] < 0 || y < first[C[u]]) first[C[u]] = y;
    }
    int32_t* Cn = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nxt.n > 0 ? (size_t)nxt.n : 1));
    if (!Cn) {
      csr_free(&nxt);
      oom = 1;
      break;
    }
    for (int32_t u = 0; u < cur.n; ++u) Cn[rank[Rf[u]]] = first[C[u]];
    for (int32_t v = 0; v < n0; ++v) map[v] = rank[Rf[map[v]]];
    for (int32_t y = 0; y < nxt.n; ++y) C[y] = Cn[y];
    free(Cn);
    if (owns) csr_free(&cur);
    cur = nxt;
    owns = 1;
    level++;
  }
  if (!oom) {
    /* canonical labels: smallest member vertex id of each final community */
    int32_t* lab = rank;
    for (int32_t x = 0; x < n0; ++x) lab[x] = -1;
    for (int32_t v = 0; v < n0; ++v) {
      int32_t f = C[map[v]];
      if (lab[f] < 0) lab[f] = v;
      C0[v] = lab[f];
    }
    if (N_out) {
      int64_t* a = (int64_t*)malloc(sizeof(int64_t) * nn);
      if (a) {
        csr_degrees(g0, k);
        *N_out = csr_numerator(g0, C0, two_m, k, a);
      } else {
        oom = 1;
      }
      free(a);
    }
  }
  if (owns) csr_free(&cur);
  if (levels_out) *levels_out = level + 1;
out:
  free(map);
  free(C);
  free(Rf);
  free(rank);
  free(first);
  free(k);
  free(all);
  free(used);
  return !oom;
}

/* ------------------------------------------------------------------------ */
/* Dynamic level-0 graph: one sorted adjacency row per vertex.               */

typedef struct {
  int32_t* nb;
  int64_t* w;
  int32_t deg;
  int32_t cap;
} row_t;

struct orc_state {
  int32_t n;
  row_t* rows;
  int64_t two_m;
  int32_t* C; /* canonical labels of the current partition */
  orc_options opt;
  /* a staged batch: G_t, the screened (or full) active set, counters */
  int staged;
  csr_t g;
  uint8_t* R;
  orc_step_info sinfo;
  /* screener samples of the last staged batch */
  int64_t ns;
  int32_t* s_ids;
  double* s_X;
  int64_t* s_raw;
  uint8_t* s_y;
};

static int64_t row_find(const row_t* r, int32_t v) {
  int64_t lo = 0, hi = r->deg;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (r->nb[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

static int row_add(row_t* r, int32_t v, int64_t w) {
  int64_t p = row_find(r, v);
  if (p < r->deg && r->nb[p] == v) {
    r->w[p] += w;
    return 1;
  }
  if (r->deg == r->cap) {
    int32_t nc = r->cap ? 2 * r->cap : 4;
    int32_t* nb = (int32_t*)realloc(r->nb, sizeof(int32_t) * (size_t)nc);
    if (!nb) return 0;
    r->nb = nb;
    int64_t* nw = (int64_t*)realloc(r->w, sizeof(int64_t) * (size_t)nc);
    if (!nw) return 0;
    r->w = nw;
    r->cap = nc;
  }
  memmove(r->nb + p + 1, r->nb + p, sizeof(int32_t) * (size_t)(r->deg - p));
  memmove(r->w + p + 1, r->w + p, sizeof(int64_t) * (size_t)(r->deg - p));
  r->nb[p] = v;
  r->w[p] = w;
  r->deg++;
  return 1;
}

static int64_t row_weight(const row_t* r, int32_t v) {
  int64_t p = row_find(r, v);
  return (p < r->deg && r->nb[p] == v) ? r->w[p] : 0;
}

static void row_remove(row_t* r, int32_t v) {
  int64_t p = row_find(r, v);
  if (p < r->deg && r->nb[p] == v) {
    memmove(r->nb + p, r->nb + p + 1, sizeof(int32_t) * (size_t)(r->deg - p - 1));
    memmove(r->w + p, r->w + p + 1, sizeof(int64_t) * (size_t)(r->deg - p - 1));
    r->deg--;
  }
}

static int snapshot(const orc_state* s, csr_t* g) {
  size_t nn = (size_t)(s->n > 0 ? s->n : 1);
  int64_t nnz = 0;
  for (int32_t u = 0; u < s->n; ++u) nnz += s->rows[u].deg;
  g->n = s->n;
  g->nnz = nnz;
  g->off = (int64_t*)malloc(sizeof(int64_t) * (nn + 1));
  g->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  g->w = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  if (!g->off || !g->col || !g->w) {
    csr_free(g);
    return 0;
  }
  int64_t p = 0;
  for (int32_t u = 0; u < s->n; ++u) {
    g->off[u] = p;
    for (int32_t q = 0; q < s->rows[u].deg; ++q) {
      g->col[p] = s->rows[u].nb[q];
      g->w[p] = s->rows[u].w[q];
      ++p;
    }
  }
  g->off[s->n] = p;
  return 1;
}

void orc_default_options(orc_options* o) {
  memset(o, 0, sizeof(*o));
  o->mode = ORC_MODE_DELTA;
  o->max_levels = 32;
  o->max_sweeps = 100;
  o->singleton_guard = 1;
  o->del_rule = ORC_DEL_GAIN;
  o->tau_den = 1000000;
}

static int options_ok(const orc_options* o) {
  return o && o->max_levels >= 1 && o->max_sweeps >= 1 &&
         (o->mode == ORC_MODE_DELTA || o->mode == ORC_MODE_ALL ||
          o->mode == ORC_MODE_STATIC || o->mode == ORC_MODE_LEARNED) &&
         (o->collect == 0 || o->collect == 1) &&
         (o->del_rule == ORC_DEL_GAIN || o->del_rule == ORC_DEL_CONSERVATIVE) &&
         o->tau_den >= 0 && o->cascade_num >= 0 && o->cascade_den >= 0 &&
         (o->algorithm == ORC_ALGO_LOUVAIN || o->algorithm == ORC_ALGO_SLM);
}

static void fill_info(orc_step_info* info, const trace_t* tr, int32_t levels,
                      int64_t N, int64_t two_m) {
  if (!info) return;
  info->levels = levels;
  info->n_sweeps = tr->count;
  info->N = N;
  info->two_m = two_m;
}

int32_t orc_init(orc_state** out, int32_t n, int64_t m, const int32_t* u,
                 const int32_t* v, const int32_t* w, const orc_options* opt,
                 int32_t* C_out, orc_sweep_rec* sweeps, int32_t cap,
                 orc_step_info* info) {
  if (!out || n < 1 || m < 0 || (m > 0 && (!u || !v || !w)) ||
      !options_ok(opt))
    return ORC_E_ARG;
  *out = NULL;
  for (int64_t e = 0; e < m; ++e)
    if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) return ORC_E_RANGE;
  for (int64_t e = 0; e < m; ++e)
    if (u[e] == v[e]) return ORC_E_SELF_LOOP;
  int64_t tot = 0;
  for (int64_t e = 0; e < m; ++e) {
    if (w[e] < 1) return ORC_E_WEIGHT;
    tot += 2 * (int64_t)w[e];
    if (tot >= TWO_M_LIMIT) return ORC_E_OVERFLOW;
  }
  orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
  if (!s) return ORC_E_OOM;
  s->n = n;
  s->opt = *opt;
  s->rows = (row_t*)calloc((size_t)n, sizeof(row_t));
  s->C = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!s->rows || !s->C) {
    orc_destroy(s);
    return ORC_E_OOM;
  }
  for (int64_t e = 0; e < m; ++e) {
    if (!row_add(&s->rows[u[e]], v[e], w[e]) ||
        !row_add(&s->rows[v[e]], u[e], w[e])) {
      orc_destroy(s);
      return ORC_E_OOM;
    }
  }
  s->two_m = tot;
  /* Static(G_1): singletons, every vertex active (Sec. 3.4 step 1). */
  for (int32_t x = 0; x < n; ++x) s->C[x] = x;
  csr_t g;
  memset(&g, 0, sizeof(g));
  uint8_t* act = (uint8_t*)malloc((size_t)n);
  if (!act || !snapshot(s, &g)) {
    free(act);
    orc_destroy(s);
    return ORC_E_OOM;
  }
  memset(act, 1, (size_t)n);
  trace_t tr = {sweeps, cap, 0};
  int32_t levels = 0;
  int64_t N = 0;
  int ok = run_levels(&g, s->C, act, &s->opt, &tr, &levels, &N);
  csr_free(&g);
  free(act);
  if (!ok) {
    orc_destroy(s);
    return ORC_E_OOM;
  }
  if (info) {
    memset(info, 0, sizeof(*info));
    info->R_size = n;
    fill_info(info, &tr, levels, N, s->two_m);
  }
  if (C_out) memcpy(C_out, s->C, sizeof(int32_t) * (size_t)n);
  *out = s;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Batch validation and application.                                         */

static int cmp_i64(const void* x, const void* y) {
  int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
  return (a > b) - (a < b);
}

static int64_t pair_key(int32_t a, int32_t b) {
  int32_t lo = a < b ? a : b, hi = a < b ? b : a;
  return ((int64_t)lo << 32) | (int64_t)(uint32_t)hi;
}

/* Check order: range, self-loop, weight, duplicate deletion, missing edge,
 * overflow of 2m.  Nothing is changed when a check fails. */
static int32_t validate_batch(const orc_state* s, int64_t na,
                              const int32_t* au, const int32_t* av,
                              const int32_t* aw, int64_t nd, const int32_t* du,
                              const int32_t* dv, int64_t* two_m_new) {
  int32_t n = s->n;
  for (int64_t e = 0; e < nd; ++e)
    if (du[e] < 0 || du[e] >= n || dv[e] < 0 || dv[e] >= n) return ORC_E_RANGE;
  for (int64_t e = 0; e < na; ++e)
    if (au[e] < 0 || au[e] >= n || av[e] < 0 || av[e] >= n) return ORC_E_RANGE;
  for (int64_t e = 0; e < nd; ++e)
    if (du[e] == dv[e]) return ORC_E_SELF_LOOP;
  for (int64_t e = 0; e < na; ++e)
    if (au[e] == av[e]) return ORC_E_SELF_LOOP;
  for (int64_t e = 0; e < na; ++e)
    if (aw[e] < 1) return ORC_E_WEIGHT;
  if (nd > 0) {
    int64_t* keys = (int64_t*)malloc(sizeof(int64_t) * (size_t)nd);
    if (!keys) return ORC_E_OOM;
    for (int64_t e = 0; e < nd; ++e) keys[e] = pair_key(du[e], dv[e]);
    qsort(keys, (size_t)nd, sizeof(int64_t), cmp_i64);
    for (int64_t e = 1; e < nd; ++e)
      if (keys[e] == keys[e - 1]) {
        free(keys);
        return ORC_E_DUP;
      }
    free(keys);
  }
  int64_t t = s->two_m;
  for (int64_t e = 0; e < nd; ++e) {
    int64_t wd = row_weight(&s->rows[du[e]], dv[e]);
    if (wd == 0) return ORC_E_NO_EDGE;
    t -= 2 * wd;
  }
  for (int64_t e = 0; e < na; ++e) {
    t += 2 * (int64_t)aw[e];
    if (t >= TWO_M_LIMIT) return ORC_E_OVERFLOW;
  }
  *two_m_new = t;
  return ORC_OK;
}

/* Delta-screening over the additions (Alg. 2), evaluated on G_t with the
 * previous labels C_{t-1} and community totals a recomputed on G_t.
 * For every source i (sinks T(i) = distinct new neighbours):
 *   j* = argmax_j G(i -> C(j)) (ties: smaller C(j), then smaller j),
 *   gain1 = G(i -> C(j*)), gain2 = G(j* -> C(i)) (0 inside one community),
 *   accept iff gain1 >= gain2 and gain1 > 0, and then add i, j*, Gamma(i) and
 *   every member of C_{t-1}(j*) to R.  Labels are never changed here. */
static void screen_additions(const csr_t* g, const int32_t* C,
                             const int64_t* k, const int64_t* a,
                             int64_t two_m, int64_t na, const int32_t* au,
                             const int32_t* av, uint8_t* R, uint8_t* cflag,
                             uint8_t* acc, agg_t* ag, orc_step_info* info) {
  int32_t n = g->n;
  /* directed pairs (source, sink), sorted by source then sink */
  int64_t* dir = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * na + 1));
  if (!dir) return;
  for (int64_t e = 0; e < na; ++e) {
    dir[2 * e] = ((int64_t)au[e] << 32) | (uint32_t)av[e];
    dir[2 * e + 1] = ((int64_t)av[e] << 32) | (uint32_t)au[e];
  }
  qsort(dir, (size_t)(2 * na), sizeof(int64_t), cmp_i64);
  int64_t p = 0;
  while (p < 2 * na) {
    int32_t i = (int32_t)(dir[p] >> 32);
    int64_t q = p;
    while (q < 2 * na && (int32_t)(dir[q] >> 32) == i) ++q;
    if (info) info->ds_sources++;
    int32_t ci = C[i];
    aggregate(g, C, i, ag);
    int64_t s_own = score(two_m, ag->seen[ci] ? ag->acc[ci] : 0, k[i], a[ci], 1);
    int32_t jstar = -1;
    int64_t g1 = 0;
    for (int64_t r = p; r < q; ++r) {
      int32_t j = (int32_t)(dir[r] & 0xffffffff);
      if (r > p && dir[r] == dir[r - 1]) continue; /* distinct sinks */
      int32_t X = C[j];
      int64_t gj = (X == ci) ? 0 : score(two_m, ag->acc[X], k[i], a[X], 0) - s_own;
      if (jstar < 0 || gj > g1 || (gj == g1 && (X < C[jstar] ||
                                              (X == C[jstar] && j < jstar)))) {
        jstar = j;
        g1 = gj;
      }
    }
    agg_clear(ag);
    int64_t g2 = 0;
    int32_t cj = C[jstar];
    if (cj != ci) {
      aggregate(g, C, jstar, ag);
      int64_t e_to_ci = ag->seen[ci] ? ag->acc[ci] : 0;
      int64_t e_own = ag->seen[cj] ? ag->acc[cj] : 0;
      g2 = score(two_m, e_to_ci, k[jstar], a[ci], 0) -
           score(two_m, e_own, k[jstar], a[cj], 1);
      agg_clear(ag);
    }
    if (g1 >= g2 && g1 > 0) {
      if (info) info->ds_accepted++;
      if (acc) acc[i] = 1;
      R[i] = 1;
      R[jstar] = 1;
      for (int64_t e = g->off[i]; e < g->off[i + 1]; ++e) R[g->col[e]] = 1;
      cflag[cj] = 1;
    }
    p = q;
  }
  (void)n;
  free(dir);
}

/* Cascade-aware screening (an extension).  After the proof of Lemma 3.2 the
 * paper notes an indirect effect it does not screen: a neighbour i1 of an
 * accepted source i that migrates in turn can pull its own neighbours along.
 * For every accepted addition source i and every neighbour v != i of i with
 * C(v) = C(i): G1(v) is the gain of v's best move to a neighbouring
 * community other than C(v) (the largest score over those communities minus
 * the score of C(v)); when G1(v) >= -theta * 2m * k_v, theta = num/den
 * (compared exactly in 128-bit integers), v and Gamma_t(v) join R.  A v with
 * no neighbouring community other than its own is skipped.  Same state as
 * Alg. 2: G_t, C_{t-1}, totals on G_t. */
static void screen_cascade(const csr_t* g, const int32_t* C, const int64_t* k,
                           const int64_t* a, int64_t two_m, const uint8_t* acc,
                           int64_t num, int64_t den, uint8_t* R, agg_t* ag,
                           orc_step_info* info) {
  int32_t n = g->n;
  uint8_t* cand = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!cand) return;
  for (int32_t i = 0; i < n; ++i) {
    if (!acc[i]) continue;
    for (int64_t e = g->off[i]; e < g->off[i + 1]; ++e) {
      int32_t v = g->col[e];
      if (v != i && C[v] == C[i]) cand[v] = 1;
    }
  }
  for (int32_t v = 0; v < n; ++v) {
    if (!cand[v]) continue;
    if (info) info->cascade_candidates++;
    int32_t c = C[v];
    aggregate(g, C, v, ag);
    int64_t s_own = score(two_m, ag->seen[c] ? ag->acc[c] : 0, k[v], a[c], 1);
    int have = 0;
    int64_t bs = 0;
    for (int32_t t = 0; t < ag->nt; ++t) {
      int32_t X = ag->touched[t];
      if (X == c) continue;
      int64_t sX = score(two_m, ag->acc[X], k[v], a[X], 0);
      if (!have || sX > bs) bs = sX;
      have = 1;
    }
    agg_clear(ag);
    if (!have) continue;
    __int128 lhs = (__int128)(bs - s_own) * den;
    __int128 rhs = -(__int128)num * two_m * k[v];
    if (lhs >= rhs) {
      if (info) info->cascade_expanded++;
      R[v] = 1;
      for (int64_t e = g->off[v]; e < g->off[v + 1]; ++e) R[g->col[e]] = 1;
    }
  }
  free(cand);
}

/* Deletions (extension; the paper covers additions only).  A source i that
 * lost an edge to a member of its own community is re-examined on G_t: if its
 * best move (no singleton guard) has a strictly positive gain, i, Gamma_t(i)
 * and the members of the best community join R.  With the conservative rule
 * every such source adds i and Gamma_t(i). */
static void screen_deletions(const csr_t* g, const int32_t* C,
                             const int64_t* k, const int64_t* a,
                             const int64_t* size, int64_t two_m, int64_t nd,
                             const int32_t* du, const int32_t* dv, int rule,
                             uint8_t* R, uint8_t* cflag, agg_t* ag,
                             orc_step_info* info) {
  int32_t n = g->n;
  uint8_t* src = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!src) return;
  for (int64_t e = 0; e < nd; ++e) {
    if (C[du[e]] == C[dv[e]]) {
      src[du[e]] = 1;
      src[dv[e]] = 1;
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    if (!src[i]) continue;
    if (info) info->del_sources++;
    if (rule == ORC_DEL_CONSERVATIVE) {
      if (info) info->del_accepted++;
      R[i] = 1;
      for (int64_t e = g->off[i]; e < g->off[i + 1]; ++e) R[g->col[e]] = 1;
      continue;
    }
    int64_t bg;
    int32_t d = decide(g, C, a, size, k, two_m, i, 0, ag, &bg);
    if (d != C[i]) {
      if (info) info->del_accepted++;
      R[i] = 1;
      for (int64_t e = g->off[i]; e < g->off[i + 1]; ++e) R[g->col[e]] = 1;
      cflag[d] = 1;
    }
  }
  free(src);
}

/* ------------------------------------------------------------------------ */
/* Screener samples (the learned screener; an extension, not in the paper).  */

static void free_samples(orc_state* s) {
  free(s->s_ids);
  free(s->s_X);
  free(s->s_raw);
  free(s->s_y);
  s->s_ids = NULL;
  s->s_X = NULL;
  s->s_raw = NULL;
  s->s_y = NULL;
  s->ns = 0;
}

/* The eight features of one vertex from its exact integer quantities; every
 * feature is one correctly rounded fp64 operation on exact integers. */
static void features_of(const int64_t* raw, int64_t two_m, double* x) {
  int64_t k = raw[0], kp = raw[1], t = raw[2];
  int64_t mx = k > kp ? k : kp;
  x[0] = (double)k / ((double)k + 16.0);
  x[1] = mx > 0 ? (double)(k - kp) / (double)mx : 0.0;
  x[2] = (double)t / ((double)t + 4.0);
  x[3] = k > 0 ? (double)raw[3] / (double)k : 0.0;
  x[4] = (k > 0 && raw[4] != ORC_NO_GAIN) ? (double)raw[4] / (double)(two_m * k) : -3.0;
  x[5] = (k > 0 && raw[5] != ORC_NO_GAIN) ? (double)raw[5] / (double)(two_m * k) : -3.0;
  x[6] = (double)raw[7];
  x[7] = two_m > 0 ? (double)raw[6] / (double)two_m : 0.0;
}

/* Records the samples of the staged batch.  src[v]: v is an endpoint of a
 * changed pair; touch[v]: number of changed pairs at v; kprev: degrees in
 * G_{t-1}; Rds: the Delta-screened set (0/1). */
static int collect_samples(orc_state* s, const csr_t* g, const int64_t* k,
                           const int64_t* kprev, const int64_t* a,
                           const int64_t* touch, const uint8_t* src,
                           const uint8_t* Rds, agg_t* ag) {
  int32_t n = s->n;
  size_t nn = (size_t)(n > 0 ? n : 1);
  const int32_t* C = s->C;
  int64_t two_m = s->two_m;
  free_samples(s);
  uint8_t* T = (uint8_t*)calloc(nn, 1);
  int32_t* Cl = (int32_t*)malloc(sizeof(int32_t) * nn);
  uint8_t* all = (uint8_t*)malloc(nn);
  if (!T || !Cl || !all) {
    free(T);
    free(Cl);
    free(all);
    return 0;
  }
  for (int32_t v = 0; v < n; ++v) {
    if (Rds[v]) T[v] = 1;
    if (!src[v]) continue;
    T[v] = 1;
    for (int64_t e = g->off[v]; e < g->off[v + 1]; ++e) T[g->col[e]] = 1;
  }
  int64_t cnt = 0;
  for (int32_t v = 0; v < n; ++v) cnt += T[v];
  size_t cc = (size_t)(cnt > 0 ? cnt : 1);
  s->s_ids = (int32_t*)malloc(sizeof(int32_t) * cc);
  s->s_X = (double*)malloc(sizeof(double) * ORC_FEATURES * cc);
  s->s_raw = (int64_t*)malloc(sizeof(int64_t) * ORC_FEATURES * cc);
  s->s_y = (uint8_t*)malloc(cc);
  if (!s->s_ids || !s->s_X || !s->s_raw || !s->s_y) {
    free(T);
    free(Cl);
    free(all);
    free_samples(s);
    return 0;
  }
  /* move labels: level 0 rerun from C_{t-1} with every vertex active */
  memcpy(Cl, C, sizeof(int32_t) * nn);
  memset(all, 1, nn);
  int64_t Tthr = s->opt.tau_den > 0 ? (two_m * two_m) / s->opt.tau_den : 0;
  int oom = 0;
  (void)level_sweeps(g, two_m, Tthr, Cl, all, &s->opt, 0, NULL, &oom, NULL, 0);
  if (oom) {
    free(T);
    free(Cl);
    free(all);
    free_samples(s);
    return 0;
  }
  int64_t q = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!T[i]) continue;
    int64_t* raw = s->s_raw + ORC_FEATURES * q;
    int32_t c = C[i];
    aggregate(g, C, i, ag);
    int64_t e_own = ag->seen[c] ? ag->acc[c] : 0;
    int64_t s_own = score(two_m, e_own, k[i], a[c], 1);
    /* best and second-best other communities: score desc, label asc */
    int32_t b1 = -1, b2 = -1;
    int64_t s1 = 0, s2 = 0;
    for (int32_t t = 0; t < ag->nt; ++t) {
      int32_t X = ag->touched[t];
      if (X == c) continue;
      int64_t sc = score(two_m, ag->acc[X], k[i], a[X], 0);
      if (b1 < 0 || sc > s1 || (sc == s1 && X < b1)) {
        b2 = b1;
        s2 = s1;
        b1 = X;
        s1 = sc;
      } else if (b2 < 0 || sc > s2 || (sc == s2 && X < b2)) {
        b2 = X;
        s2 = sc;
      }
    }
    agg_clear(ag);
    raw[0] = k[i];
    raw[1] = kprev[i];
    raw[2] = touch[i];
    raw[3] = e_own;
    raw[4] = b1 >= 0 ? s1 - s_own : ORC_NO_GAIN;
    raw[5] = b2 >= 0 ? s2 - s_own : ORC_NO_GAIN;
    raw[6] = a[c];
    raw[7] = Rds[i] ? 1 : 0;
    features_of(raw, two_m, s->s_X + ORC_FEATURES * q);
    s->s_ids[q] = i;
    s->s_y[q] = Cl[i] != c ? 1 : 0;
    ++q;
  }
  s->ns = cnt;
  free(T);
  free(Cl);
  free(all);
  return 1;
}

/* ------------------------------------------------------------------------ */
/* One time step (Sec. 3.4): stage (validate, update, screen), then finish   */
/* (levels over the active set, canonical labels).                           */

static void drop_stage(orc_state* s) {
  if (!s->staged) return;
  csr_free(&s->g);
  free(s->R);
  s->R = NULL;
  s->staged = 0;
}

int32_t orc_stage_batch(orc_state* s, int64_t na, const int32_t* au,
                        const int32_t* av, const int32_t* aw, int64_t nd,
                        const int32_t* du, const int32_t* dv) {
  if (!s || s->staged || na < 0 || nd < 0 || (na > 0 && (!au || !av || !aw)) ||
      (nd > 0 && (!du || !dv)))
    return ORC_E_ARG;
  int64_t two_m_new = 0;
  int32_t st = validate_batch(s, na, au, av, aw, nd, du, dv, &two_m_new);
  if (st != ORC_OK) return st;
  int32_t n = s->n;
  size_t nn = (size_t)(n > 0 ? n : 1);
  int mode = s->opt.mode;
  int collect = s->opt.collect || mode == ORC_MODE_LEARNED;
  int screen = mode == ORC_MODE_DELTA || mode == ORC_MODE_LEARNED || collect;
  int64_t* kprev = (int64_t*)malloc(sizeof(int64_t) * nn);
  if (!kprev) return ORC_E_OOM;
  for (int32_t v = 0; v < n; ++v) {
    int64_t t = 0;
    for (int32_t q = 0; q < s->rows[v].deg; ++q) t += s->rows[v].w[q];
    kprev[v] = t;
  }
  /* deletions first, then insertions (weights add; duplicates sum) */
  for (int64_t e = 0; e < nd; ++e) {
    row_remove(&s->rows[du[e]], dv[e]);
    row_remove(&s->rows[dv[e]], du[e]);
  }
  for (int64_t e = 0; e < na; ++e) {
    if (!row_add(&s->rows[au[e]], av[e], aw[e]) ||
        !row_add(&s->rows[av[e]], au[e], aw[e])) {
      free(kprev);
      return ORC_E_OOM;
    }
  }
  s->two_m = two_m_new;

  memset(&s->g, 0, sizeof(s->g));
  memset(&s->sinfo, 0, sizeof(s->sinfo));
  if (!snapshot(s, &s->g)) {
    free(kprev);
    return ORC_E_OOM;
  }
  s->R = (uint8_t*)calloc(nn, 1);
  uint8_t* cflag = (uint8_t*)calloc(nn, 1);
  int64_t* k = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* a = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* size = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* touch = (int64_t*)calloc(nn, sizeof(int64_t));
  uint8_t* src = (uint8_t*)calloc(nn, 1);
  uint8_t* acc = (uint8_t*)calloc(nn, 1);
  int64_t* pairs = (int64_t*)malloc(sizeof(int64_t) * (size_t)(na + nd + 1));
  agg_t ag;
  int have_ag = agg_alloc(&ag, n);
  int ok = s->R && cflag && k && a && size && touch && src && acc && pairs && have_ag;
  if (ok) {
    csr_degrees(&s->g, k);
    totals(&s->g, s->C, k, a, size);
    if (screen) {
      screen_additions(&s->g, s->C, k, a, s->two_m, na, au, av, s->R, cflag,
                       acc, &ag, &s->sinfo);
      if (s->opt.cascade_den > 0)
        screen_cascade(&s->g, s->C, k, a, s->two_m, acc, s->opt.cascade_num,
                       s->opt.cascade_den, s->R, &ag, &s->sinfo);
      screen_deletions(&s->g, s->C, k, a, size, s->two_m, nd, du, dv,
                       s->opt.del_rule, s->R, cflag, &ag, &s->sinfo);
      for (int32_t v = 0; v < n; ++v)
        if (cflag[s->C[v]]) s->R[v] = 1;
    }
    if (collect) {
      /* changed pairs (a pair deleted and re-added counts once) */
      int64_t np = 0;
      for (int64_t e = 0; e < nd; ++e) pairs[np++] = pair_key(du[e], dv[e]);
      for (int64_t e = 0; e < na; ++e) pairs[np++] = pair_key(au[e], av[e]);
      qsort(pairs, (size_t)np, sizeof(int64_t), cmp_i64);
      for (int64_t p = 0; p < np; ++p) {
        if (p > 0 && pairs[p] == pairs[p - 1]) continue;
        int32_t x = (int32_t)(pairs[p] >> 32), y = (int32_t)(pairs[p] & 0xffffffff);
        touch[x]++;
        touch[y]++;
        src[x] = 1;
        src[y] = 1;
      }
      ok = collect_samples(s, &s->g, k, kprev, a, touch, src, s->R, &ag);
    } else {
      free_samples(s);
    }
    if (mode == ORC_MODE_ALL || mode == ORC_MODE_STATIC) memset(s->R, 1, nn);
  }
  if (have_ag) agg_free(&ag);
  free(cflag);
  free(k);
  free(a);
  free(size);
  free(touch);
  free(src);
  free(acc);
  free(pairs);
  free(kprev);
  if (!ok) {
    csr_free(&s->g);
    free(s->R);
    s->R = NULL;
    return ORC_E_OOM;
  }
  s->staged = 1;
  return ORC_OK;
}

int32_t orc_finish_batch(orc_state* s, const uint8_t* R_override,
                         int32_t* C_out, uint8_t* R_out, orc_sweep_rec* sweeps,
                         int32_t cap, orc_step_info* info) {
  if (!s || !s->staged) return ORC_E_ARG;
  int32_t n = s->n;
  size_t nn = (size_t)n;
  if (R_override)
    for (int32_t v = 0; v < n; ++v) s->R[v] = R_override[v] ? 1 : 0;
  if (s->opt.mode == ORC_MODE_STATIC)
    for (int32_t v = 0; v < n; ++v) s->C[v] = v;
  int64_t Rsz = 0;
  for (int32_t v = 0; v < n; ++v) Rsz += s->R[v];
  if (R_out) memcpy(R_out, s->R, nn);
  trace_t tr = {sweeps, cap, 0};
  int32_t levels = 0;
  int64_t N = 0;
  int ok = run_levels(&s->g, s->C, s->R, &s->opt, &tr, &levels, &N);
  orc_step_info si = s->sinfo;
  drop_stage(s);
  if (!ok) return ORC_E_OOM;
  if (info) {
    *info = si;
    info->R_size = Rsz;
    fill_info(info, &tr, levels, N, s->two_m);
  }
  if (C_out) memcpy(C_out, s->C, sizeof(int32_t) * nn);
  return ORC_OK;
}

int32_t orc_apply_batch(orc_state* s, int64_t na, const int32_t* au,
                        const int32_t* av, const int32_t* aw, int64_t nd,
                        const int32_t* du, const int32_t* dv, int32_t* C_out,
                        uint8_t* R_out, orc_sweep_rec* sweeps, int32_t cap,
                        orc_step_info* info) {
  int32_t st = orc_stage_batch(s, na, au, av, aw, nd, du, dv);
  if (st != ORC_OK) return st;
  return orc_finish_batch(s, NULL, C_out, R_out, sweeps, cap, info);
}

int32_t orc_last_samples(const orc_state* s, int64_t* count, int32_t* ids,
                         double* X, int64_t* raw, uint8_t* y) {
  if (!s) return ORC_E_ARG;
  if (count) *count = s->ns;
  if (s->ns == 0) return ORC_OK;
  if (ids) memcpy(ids, s->s_ids, sizeof(int32_t) * (size_t)s->ns);
  if (X) memcpy(X, s->s_X, sizeof(double) * ORC_FEATURES * (size_t)s->ns);
  if (raw) memcpy(raw, s->s_raw, sizeof(int64_t) * ORC_FEATURES * (size_t)s->ns);
  if (y) memcpy(y, s->s_y, (size_t)s->ns);
  return ORC_OK;
}

int32_t orc_modularity(const orc_state* s, int64_t* N, int64_t* two_m,
                       double* q) {
  if (!s) return ORC_E_ARG;
  csr_t g;
  memset(&g, 0, sizeof(g));
  if (!snapshot(s, &g)) return ORC_E_OOM;
  size_t nn = (size_t)s->n;
  int64_t* k = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* a = (int64_t*)malloc(sizeof(int64_t) * nn);
  if (!k || !a) {
    free(k);
    free(a);
    csr_free(&g);
    return ORC_E_OOM;
  }
  csr_degrees(&g, k);
  int64_t tm = csr_two_m(&g);
  int64_t num = csr_numerator(&g, s->C, tm, k, a);
  free(k);
  free(a);
  csr_free(&g);
  if (N) *N = num;
  if (two_m) *two_m = tm;
  if (q) *q = tm == 0 ? 0.0 : (double)num / ((double)tm * (double)tm);
  return ORC_OK;
}

int32_t orc_communities(const orc_state* s, int32_t* out) {
  if (!s || !out) return ORC_E_ARG;
  memcpy(out, s->C, sizeof(int32_t) * (size_t)s->n);
  return ORC_OK;
}

int64_t orc_num_entries(const orc_state* s) {
  int64_t t = 0;
  for (int32_t u = 0; u < s->n; ++u) t += s->rows[u].deg;
  return t;
}

int32_t orc_export_csr(const orc_state* s, int64_t* off, int32_t* col,
                       int32_t* w) {
  if (!s || !off || !col || !w) return ORC_E_ARG;
  int64_t p = 0;
  for (int32_t u = 0; u < s->n; ++u) {
    off[u] = p;
    for (int32_t q = 0; q < s->rows[u].deg; ++q) {
      col[p] = s->rows[u].nb[q];
      w[p] = (int32_t)s->rows[u].w[q];
      ++p;
    }
  }
  off[s->n] = p;
  return ORC_OK;
}

void orc_destroy(orc_state* s) {
  if (!s) return;
  if (s->rows) {
    for (int32_t u = 0; u < s->n; ++u) {
      free(s->rows[u].nb);
      free(s->rows[u].w);
    }
    free(s->rows);
  }
  free(s->C);
  drop_stage(s);
  free_samples(s);
  free(s);
}

/* ------------------------------------------------------------------------ */
/* Stateless entry points for the pin tests.                                 */

static csr_t view(int32_t n, const int64_t* off, const int32_t* col,
                  const int64_t* w) {
  csr_t g;
  g.n = n;
  g.nnz = off[n];
  g.off = (int64_t*)off;
  g.col = (int32_t*)col;
  g.w = (int64_t*)w;
  return g;
}

int32_t orc_csr_modularity(int32_t n, const int64_t* off, const int32_t* col,
                           const int64_t* w, const int32_t* C, int64_t* N,
                           int64_t* two_m) {
  if (n < 1 || !off || !C) return ORC_E_ARG;
  csr_t g = view(n, off, col, w);
  int64_t* k = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* a = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!k || !a) {
    free(k);
    free(a);
    return ORC_E_OOM;
  }
  csr_degrees(&g, k);
  int64_t tm = csr_two_m(&g);
  if (N) *N = csr_numerator(&g, C, tm, k, a);
  if (two_m) *two_m = tm;
  free(k);
  free(a);
  return ORC_OK;
}

int64_t orc_csr_gain(int32_t n, const int64_t* off, const int32_t* col,
                     const int64_t* w, const int32_t* C, int32_t i,
                     int32_t D) {
  csr_t g = view(n, off, col, w);
  int64_t* k = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* a = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* size = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  agg_t ag;
  int64_t G = 0;
  if (k && a && size && agg_alloc(&ag, n)) {
    csr_degrees(&g, k);
    totals(&g, C, k, a, size);
    int64_t tm = csr_two_m(&g);
    int32_t c = C[i];
    if (D != c) {
      aggregate(&g, C, i, &ag);
      int64_t eD = ag.seen[D] ? ag.acc[D] : 0;
      int64_t ec = ag.seen[c] ? ag.acc[c] : 0;
      G = score(tm, eD, k[i], a[D], 0) - score(tm, ec, k[i], a[c], 1);
      agg_clear(&ag);
    }
    agg_free(&ag);
  }
  free(k);
  free(a);
  free(size);
  return G;
}

int32_t orc_csr_decide(int32_t n, const int64_t* off, const int32_t* col,
                       const int64_t* w, const int32_t* C, int32_t i,
                       int32_t guard, int64_t* best_gain) {
  csr_t g = view(n, off, col, w);
  int64_t* k = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* a = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* size = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  agg_t ag;
  int32_t d = -1;
  int64_t bg = 0;
  if (k && a && size && agg_alloc(&ag, n)) {
    csr_degrees(&g, k);
    totals(&g, C, k, a, size);
    d = decide(&g, C, a, size, k, csr_two_m(&g), i, guard, &ag, &bg);
    agg_free(&ag);
  }
  if (best_gain) *best_gain = bg;
  free(k);
  free(a);
  free(size);
  return d;
}

int32_t orc_csr_run_levels(int32_t n, const int64_t* off, const int32_t* col,
                           const int64_t* w, int32_t* C, const uint8_t* active,
                           const orc_options* opt, orc_sweep_rec* sweeps,
                           int32_t cap, int32_t* n_sweeps, int32_t* levels) {
  if (n < 1 || !off || !C || !active || !options_ok(opt)) return ORC_E_ARG;
  csr_t g = view(n, off, col, w);
  trace_t tr = {sweeps, cap, 0};
  int32_t lv = 0;
  int ok = run_levels(&g, C, active, opt, &tr, &lv, NULL);
  if (n_sweeps) *n_sweeps = tr.count;
  if (levels) *levels = lv;
  return ok ? ORC_OK : ORC_E_OOM;
}

int32_t orc_csr_coarsen(int32_t n, const int64_t* off, const int32_t* col,
                        const int64_t* w, const int32_t* C, int32_t* rank,
                        int32_t* n_out, int64_t* off_out, int32_t* col_out,
                        int64_t* w_out, int64_t* nnz_out) {
  if (n < 1 || !off || !C || !rank) return ORC_E_ARG;
  csr_t g = view(n, off, col, w);
  csr_t h;
  memset(&h, 0, sizeof(h));
  if (!coarsen(&g, C, rank, &h)) return ORC_E_OOM;
  if (n_out) *n_out = h.n;
  if (nnz_out) *nnz_out = h.nnz;
  if (off_out) memcpy(off_out, h.off, sizeof(int64_t) * ((size_t)h.n + 1));
  if (col_out) memcpy(col_out, h.col, sizeof(int32_t) * (size_t)h.nnz);
  if (w_out) memcpy(w_out, h.w, sizeof(int64_t) * (size_t)h.nnz);
  csr_free(&h);
  return ORC_OK;
}
