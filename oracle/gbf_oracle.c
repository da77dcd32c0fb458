/*
 * Plain, single-threaded CPU oracle for the generalized Bellman-Ford method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product path: only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * load this library.  It shares no code, header, table or helper with the
 * HIP library.
 *
 * What it computes (Weber, Kreuzer, Knoll, "A generalized Bellman-Ford
 * Algorithm for Application in Symbolic Optimal Control"):
 *   - Sect. III-C, dynamic programming operator
 *       P(W)(x) = min{ G(x), min_u max_{y in F(x,u)} g(x,y,u) + W(y) }
 *     with the running cost of a transition given as g(x,y,u) =
 *     g(x,u) + h(x,y,u): a per-pair part g and, optionally, a per-edge part
 *     h (one value per successor-list entry; absent = 0); the value
 *     function V is its maximal fixed point (Theorem on dynamic
 *     programming, Sect. III-C).
 *   - Sect. IV-A, Algorithm 1 (generalized Bellman-Ford-Yen): two state
 *     frontiers, the active one processed as F1 x U, in-place updates of W
 *     on strict improvement, predecessors of an improved state pushed into
 *     the upcoming frontier, and the round cap i < |X| that detects
 *     negative cycles.
 *   - Sect. IV-B: frontiers as FIFO queues whose length never exceeds |X|
 *     (a membership flag keeps every state at most once per frontier).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - Avoid cells are pinned to W = INF and never enter a frontier.
 *   - int32 costs: sums are formed in int64; a sum >= INT32_MAX means INF
 *     (no improvement); a sum below -INT32_MAX saturates to -INT32_MAX and
 *     is counted in `saturations`.
 *   - Per-edge costs h must be finite.  A pair's backup is
 *     g(x,u) + max_y (h(x,y,u) + W(y)): exact in int64 for int32; for
 *     single precision each h + W(y) is one IEEE addition and the pair cost
 *     one more (adding g after the max equals adding it per edge, since
 *     rounding is monotone).
 *   - Floating point: the definition is evaluated in double precision
 *     (oracle_solve_f64).  oracle_solve_f32 evaluates the same algorithm
 *     with one IEEE single-precision round-to-nearest-even addition per
 *     backup; it is the fp32 operator whose maximal fixed point the GPU
 *     reaches, and is used for the exact (bit-level) comparison.
 *   - Canonical policy (post-pass): for finite W(x), start from G(x) with
 *     "hand over", scan u ascending and keep the first u whose backup is
 *     strictly smaller; INF states get "none".  The first-improvement rule
 *     matches the paper's strict test d < W(x) and its worked example, where
 *     a state whose best input only ties G keeps mu(x) = U (hand over).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NEGCYCLE 1
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define OR_HANDOVER (-1)
#define OR_NONE (-2)

#define OR_INF_I32 ((int64_t)INT32_MAX)
#define OR_LOW_I32 (-(int64_t)INT32_MAX)

typedef struct {
    int64_t rounds;       /* while-loop iterations executed */
    int64_t pair_evals;   /* (x,u) in F1 x U whose successors were read */
    int64_t edge_relax;   /* sum of |F(x,u)| over those pairs */
    int64_t improvements; /* strict decreases of W */
    int64_t saturations;  /* int32 sums clamped at -INT32_MAX */
} oracle_counters;

/* ------------------------------------------------------------------ */
/* State-level predecessor lists: pred(y) = { x : y in F(x,u), some u }, */
/* each x listed once, ascending.                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t* ptr; /* n+1 */
    int32_t* idx;
} or_pred;

static void pred_free(or_pred* p) {
    free(p->ptr);
    free(p->idx);
    p->ptr = NULL;
    p->idx = NULL;
}

static int pred_build(int64_t n, int64_t K, const int64_t* sp, const int32_t* si, or_pred* out) {
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* last = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!cnt || !last) {
        free(cnt);
        free(last);
        return OR_ENOMEM;
    }
    for (int64_t y = 0; y < n; ++y) last[y] = -1;
    for (int64_t x = 0; x < n; ++x)
        for (int64_t u = 0; u < K; ++u) {
            int64_t p = x * K + u;
            for (int64_t e = sp[p]; e < sp[p + 1]; ++e) {
                int32_t y = si[e];
                if (last[y] != (int32_t)x) {
                    last[y] = (int32_t)x;
                    cnt[y + 1]++;
                }
            }
        }
    for (int64_t y = 0; y < n; ++y) cnt[y + 1] += cnt[y];
    int32_t* idx = (int32_t*)malloc((size_t)(cnt[n] > 0 ? cnt[n] : 1) * sizeof(int32_t));
    int64_t* fill = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!idx || !fill) {
        free(cnt);
        free(last);
        free(idx);
        free(fill);
        return OR_ENOMEM;
    }
    for (int64_t y = 0; y < n; ++y) {
        last[y] = -1;
        fill[y] = cnt[y];
    }
    for (int64_t x = 0; x < n; ++x)
        for (int64_t u = 0; u < K; ++u) {
            int64_t p = x * K + u;
            for (int64_t e = sp[p]; e < sp[p + 1]; ++e) {
                int32_t y = si[e];
                if (last[y] != (int32_t)x) {
                    last[y] = (int32_t)x;
                    idx[fill[y]++] = (int32_t)x;
                }
            }
        }
    free(last);
    free(fill);
    out->ptr = cnt;
    out->idx = idx;
    return OR_OK;
}

/* Validation shared by the entry points: strict F, indices in range. */
static int check_graph(int64_t n, int64_t K, const int64_t* sp, const int32_t* si) {
    if (n <= 0 || K <= 0 || sp[0] != 0) return OR_EINVAL;
    for (int64_t p = 0; p < n * K; ++p) {
        if (sp[p + 1] <= sp[p]) return OR_EINVAL; /* F(x,u) must be non-empty */
        for (int64_t e = sp[p]; e < sp[p + 1]; ++e)
            if (si[e] < 0 || si[e] >= n) return OR_EINVAL;
    }
    return OR_OK;
}

/* FIFO frontier with a membership flag. */
typedef struct {
    int32_t* q;
    int64_t len;
} or_fifo;

/* ------------------------------------------------------------------ */
/* Algorithm 1, one instantiation per value type.                      */
/* ------------------------------------------------------------------ */
#define OR_DEFINE_SOLVER(NAME, VT, GT, IS_INF, INFV, BACKUP, WT, EDGE, WINF, BACKUPW)                \
    int NAME(int64_t n, int64_t K, const int64_t* sp, const int32_t* si, const GT* g, const GT* h, \
             const GT* G, const uint8_t* avoid, int64_t max_rounds, VT* W, int32_t* mu,           \
             oracle_counters* c, int32_t* front_out, int64_t* front_len) {                         \
        oracle_counters cc;                                                                        \
        memset(&cc, 0, sizeof(cc));                                                                \
        int rc = check_graph(n, K, sp, si);                                                        \
        if (rc) return rc;                                                                         \
        or_pred pr;                                                                                \
        rc = pred_build(n, K, sp, si, &pr);                                                        \
        if (rc) return rc;                                                                         \
        or_fifo f1, f2;                                                                            \
        f1.q = (int32_t*)malloc((size_t)n * sizeof(int32_t));                                      \
        f2.q = (int32_t*)malloc((size_t)n * sizeof(int32_t));                                      \
        uint8_t* in2 = (uint8_t*)calloc((size_t)n, 1);                                             \
        if (!f1.q || !f2.q || !in2) {                                                              \
            free(f1.q);                                                                            \
            free(f2.q);                                                                            \
            free(in2);                                                                             \
            pred_free(&pr);                                                                        \
            return OR_ENOMEM;                                                                      \
        }                                                                                          \
        f1.len = f2.len = 0;                                                                       \
        /* initialisation: W <- G, mu <- U, F1 <- pred of every state with G < INF */             \
        for (int64_t x = 0; x < n; ++x) {                                                          \
            W[x] = (avoid && avoid[x]) ? INFV : (VT)G[x];                                          \
            mu[x] = OR_HANDOVER;                                                                   \
        }                                                                                          \
        for (int64_t y = 0; y < n; ++y) {                                                          \
            if (IS_INF(G[y]) || (avoid && avoid[y])) continue;                                     \
            for (int64_t e = pr.ptr[y]; e < pr.ptr[y + 1]; ++e) {                                  \
                int32_t x = pr.idx[e];                                                             \
                if ((avoid && avoid[x]) || in2[x]) continue;                                       \
                in2[x] = 1;                                                                        \
                f1.q[f1.len++] = x;                                                                \
            }                                                                                      \
        }                                                                                          \
        for (int64_t j = 0; j < f1.len; ++j) in2[f1.q[j]] = 0;                                     \
        if (max_rounds <= 0) max_rounds = n;                                                       \
        int64_t i = 0;                                                                             \
        while (f1.len > 0 && i < max_rounds) {                                                     \
            f2.len = 0;                                                                            \
            for (int64_t j = 0; j < f1.len; ++j) {                                                 \
                int32_t x = f1.q[j];                                                               \
                int improved = 0;                                                                  \
                for (int64_t u = 0; u < K; ++u) {                                                  \
                    int64_t p = x * K + u;                                                         \
                    if (IS_INF(g[p])) continue;                                                    \
                    cc.pair_evals++;                                                               \
                    cc.edge_relax += sp[p + 1] - sp[p];                                            \
                    VT d;                                                                          \
                    if (h) {                                                                       \
                        WT mw = EDGE(h[sp[p]], W[si[sp[p]]]);                                      \
                        for (int64_t e = sp[p] + 1; e < sp[p + 1]; ++e) {                          \
                            WT v = EDGE(h[e], W[si[e]]);                                           \
                            if (v > mw) mw = v;                                                    \
                        }                                                                          \
                        if (mw == WINF) continue;                                                  \
                        if (!BACKUPW(g[p], mw, &d, &cc)) continue;                                 \
                    } else {                                                                       \
                        VT mx = W[si[sp[p]]];                                                      \
                        for (int64_t e = sp[p] + 1; e < sp[p + 1]; ++e)                            \
                            if (W[si[e]] > mx) mx = W[si[e]];                                      \
                        if (mx == INFV) continue;                                                  \
                        if (!BACKUP(g[p], mx, &d, &cc)) continue;                                  \
                    }                                                                              \
                    if (d < W[x]) {                                                                \
                        W[x] = d;                                                                  \
                        mu[x] = (int32_t)u;                                                        \
                        improved = 1;                                                              \
                        cc.improvements++;                                                         \
                    }                                                                              \
                }                                                                                  \
                if (improved) {                                                                    \
                    for (int64_t e = pr.ptr[x]; e < pr.ptr[x + 1]; ++e) {                          \
                        int32_t xp = pr.idx[e];                                                    \
                        if ((avoid && avoid[xp]) || in2[xp]) continue;                             \
                        in2[xp] = 1;                                                               \
                        f2.q[f2.len++] = xp;                                                       \
                    }                                                                              \
                }                                                                                  \
            }                                                                                      \
            /* swap frontiers */                                                                   \
            int32_t* t = f1.q;                                                                     \
            f1.q = f2.q;                                                                           \
            f2.q = t;                                                                              \
            f1.len = f2.len;                                                                       \
            for (int64_t j = 0; j < f1.len; ++j) in2[f1.q[j]] = 0;                                 \
            ++i;                                                                                   \
        }                                                                                          \
        cc.rounds = i;                                                                             \
        int status = f1.len > 0 ? OR_NEGCYCLE : OR_OK;                                             \
        if (front_len) *front_len = f1.len;                                                        \
        if (front_out)                                                                             \
            for (int64_t j = 0; j < f1.len; ++j) front_out[j] = f1.q[j];                           \
        free(f1.q);                                                                                \
        free(f2.q);                                                                                \
        free(in2);                                                                                 \
        pred_free(&pr);                                                                            \
        if (c) *c = cc;                                                                            \
        return status;                                                                             \
    }

/* backup d = g + m; returns 0 if the result is INF (no improvement possible) */
static inline int backup_i32(int32_t g, int32_t m, int32_t* d, oracle_counters* c) {
    int64_t s = (int64_t)g + (int64_t)m;
    if (s >= OR_INF_I32) return 0;
    if (s < OR_LOW_I32) {
        s = OR_LOW_I32;
        c->saturations++;
    }
    *d = (int32_t)s;
    return 1;
}
static inline int backup_f64(float g, double m, double* d, oracle_counters* c) {
    (void)c;
    double s = (double)g + m;
    if (isinf(s) && s > 0) return 0;
    *d = s;
    return 1;
}
static inline int backup_f32(float g, float m, float* d, oracle_counters* c) {
    (void)c;
    volatile float s = g + m; /* one IEEE single addition, round to nearest even */
    if (isinf(s) && s > 0) return 0;
    *d = s;
    return 1;
}

/* per-edge term h + W(y); INF stays INF (a sentinel far above any finite
 * int32 sum, so that the max over a row is INF if any W(y) is) */
#define OR_EDGE_INF_I64 ((int64_t)1 << 62)
static inline int64_t edge_i32(int32_t h, int32_t w) {
    return (int64_t)w >= OR_INF_I32 ? OR_EDGE_INF_I64 : (int64_t)h + (int64_t)w;
}
static inline double edge_f64(float h, double w) { return (double)h + w; }
static inline float edge_f32(float h, float w) {
    volatile float s = h + w; /* one IEEE single addition */
    return s;
}
static inline int backupw_i32(int32_t g, int64_t m, int32_t* d, oracle_counters* c) {
    int64_t s = (int64_t)g + m;
    if (s >= OR_INF_I32) return 0;
    if (s < OR_LOW_I32) {
        s = OR_LOW_I32;
        c->saturations++;
    }
    *d = (int32_t)s;
    return 1;
}

#define IS_INF_I32(v) ((int64_t)(v) >= OR_INF_I32)
#define IS_INF_F(v) (isinf(v) && (v) > 0)

OR_DEFINE_SOLVER(oracle_solve_i32, int32_t, int32_t, IS_INF_I32, (int32_t)INT32_MAX, backup_i32, int64_t,
                 edge_i32, OR_EDGE_INF_I64, backupw_i32)
OR_DEFINE_SOLVER(oracle_solve_f64, double, float, IS_INF_F, (double)INFINITY, backup_f64, double, edge_f64,
                 (double)INFINITY, backup_f64)
OR_DEFINE_SOLVER(oracle_solve_f32, float, float, IS_INF_F, (float)INFINITY, backup_f32, float, edge_f32,
                 (float)INFINITY, backup_f32)

/* ------------------------------------------------------------------ */
/* Canonical policy + residual: one application of P to W.             */
/* Returns the number of non-avoid states with P(W)(x) != W(x).        */
/* ------------------------------------------------------------------ */
#define OR_DEFINE_POLICY(NAME, VT, GT, IS_INF, INFV, BACKUP, WT, EDGE, WINF, BACKUPW)                 \
    int64_t NAME(int64_t n, int64_t K, const int64_t* sp, const int32_t* si, const GT* g,           \
                 const GT* h, const GT* G, const uint8_t* avoid, const VT* W, int32_t* pol) {       \
        oracle_counters dummy;                                                                      \
        int64_t bad = 0;                                                                            \
        for (int64_t x = 0; x < n; ++x) {                                                           \
            if (avoid && avoid[x]) {                                                                \
                if (pol) pol[x] = OR_NONE;                                                          \
                if (W[x] != INFV) ++bad;                                                            \
                continue;                                                                           \
            }                                                                                       \
            VT best = IS_INF(G[x]) ? INFV : (VT)G[x];                                               \
            int32_t pu = OR_HANDOVER;                                                               \
            for (int64_t u = 0; u < K; ++u) {                                                       \
                int64_t p = x * K + u;                                                              \
                if (IS_INF(g[p])) continue;                                                         \
                VT d;                                                                               \
                if (h) {                                                                            \
                    WT mw = EDGE(h[sp[p]], W[si[sp[p]]]);                                           \
                    for (int64_t e = sp[p] + 1; e < sp[p + 1]; ++e) {                               \
                        WT v = EDGE(h[e], W[si[e]]);                                                \
                        if (v > mw) mw = v;                                                         \
                    }                                                                               \
                    if (mw == WINF) continue;                                                       \
                    if (!BACKUPW(g[p], mw, &d, &dummy)) continue;                                   \
                } else {                                                                            \
                    VT mx = W[si[sp[p]]];                                                           \
                    for (int64_t e = sp[p] + 1; e < sp[p + 1]; ++e)                                 \
                        if (W[si[e]] > mx) mx = W[si[e]];                                           \
                    if (mx == INFV) continue;                                                       \
                    if (!BACKUP(g[p], mx, &d, &dummy)) continue;                                    \
                }                                                                                   \
                if (d < best) {                                                                     \
                    best = d;                                                                       \
                    pu = (int32_t)u;                                                                \
                }                                                                                   \
            }                                                                                       \
            if (best == INFV) pu = OR_NONE;                                                         \
            if (pol) pol[x] = pu;                                                                   \
            if (best != W[x]) ++bad;                                                                \
        }                                                                                           \
        return bad;                                                                                 \
    }

OR_DEFINE_POLICY(oracle_policy_i32, int32_t, int32_t, IS_INF_I32, (int32_t)INT32_MAX, backup_i32, int64_t,
                 edge_i32, OR_EDGE_INF_I64, backupw_i32)
OR_DEFINE_POLICY(oracle_policy_f64, double, float, IS_INF_F, (double)INFINITY, backup_f64, double, edge_f64,
                 (double)INFINITY, backup_f64)
OR_DEFINE_POLICY(oracle_policy_f32, float, float, IS_INF_F, (float)INFINITY, backup_f32, float, edge_f32,
                 (float)INFINITY, backup_f32)

/* ------------------------------------------------------------------ */
/* Box decoding (the oracle's own): packed 8-byte box per pair, low    */
/* 32 bits = linear low corner, bytes 4..7 = extents per axis.  Cells  */
/* listed in ascending linear order.  Call with idx == NULL to size.   */
/* ------------------------------------------------------------------ */
int64_t oracle_box_to_csr(const int32_t* dims, int64_t npairs, const uint64_t* box, int64_t* ptr,
                          int32_t* idx) {
    int64_t s1 = dims[0], s2 = (int64_t)dims[0] * dims[1], s3 = (int64_t)dims[0] * dims[1] * dims[2];
    int64_t ncell = s3 * dims[3];
    int64_t pos = 0;
    if (ptr) ptr[0] = 0;
    for (int64_t p = 0; p < npairs; ++p) {
        uint64_t b = box[p];
        int64_t lo = (int64_t)(b & 0xffffffffu);
        int e[4];
        for (int a = 0; a < 4; ++a) e[a] = (int)((b >> (32 + 8 * a)) & 0xffu);
        int c[4];
        int64_t r = lo;
        c[0] = (int)(r % dims[0]);
        r /= dims[0];
        c[1] = (int)(r % dims[1]);
        r /= dims[1];
        c[2] = (int)(r % dims[2]);
        r /= dims[2];
        c[3] = (int)r;
        if (lo >= ncell) return OR_EINVAL;
        for (int a = 0; a < 4; ++a)
            if (c[a] + e[a] >= dims[a]) return OR_EINVAL;
        for (int j3 = 0; j3 <= e[3]; ++j3)
            for (int j2 = 0; j2 <= e[2]; ++j2)
                for (int j1 = 0; j1 <= e[1]; ++j1)
                    for (int j0 = 0; j0 <= e[0]; ++j0) {
                        if (idx) idx[pos] = (int32_t)(lo + j0 + j1 * s1 + j2 * s2 + j3 * s3);
                        ++pos;
                    }
        if (ptr) ptr[p + 1] = pos;
    }
    return pos;
}

/* ------------------------------------------------------------------ */
/* Sampled fixed-point check for problems too large for Algorithm 1 on  */
/* the CPU: one application of the operator P (Sect. III-C; the test   */
/* that certifies a fixed point) at the sampled states only, with the  */
/* oracle's own box decoding and the int32 reading of costs.  For each */
/* sampled state x (states[i], ascending or not) the caller passes its */
/* K boxes and costs (rows i*K .. i*K+K-1), G(x), and the full V and    */
/* avoid arrays.  An avoid state must have V = INF; otherwise           */
/*   P(V)(x) = min{ G(x), min_u g(x,u) + max_{y in F(x,u)} V(y) }      */
/* with INF for g = INF or any V(y) = INF (an avoid successor has       */
/* V = INF, which is the pruning of pairs that lead into the avoid set),*/
/* sums formed in 64 bits, >= INT32_MAX as INF and below -INT32_MAX     */
/* clamped.  Returns the number of sampled states with P(V)(x) != V(x)  */
/* (first offenders in bad_out, up to 16), or OR_EINVAL for a box that  */
/* leaves the grid.                                                    */
/* ------------------------------------------------------------------ */
int64_t oracle_residual_box_sample(const int32_t* dims, int64_t K, const int64_t* states, int64_t count,
                                   const uint64_t* box, const int32_t* g, const int32_t* G,
                                   const uint8_t* avoid, const int32_t* V, int64_t* bad_out) {
    int64_t s1 = dims[0], s2 = (int64_t)dims[0] * dims[1], s3 = (int64_t)dims[0] * dims[1] * dims[2];
    int64_t ncell = s3 * dims[3];
    int64_t bad = 0;
    oracle_counters dummy;
    memset(&dummy, 0, sizeof(dummy));
    for (int64_t i = 0; i < count; ++i) {
        int64_t x = states[i];
        int ok;
        if (avoid[x]) {
            ok = IS_INF_I32(V[x]);
        } else {
            int32_t best = G[i];
            for (int64_t u = 0; u < K; ++u) {
                uint64_t b = box[i * K + u];
                int32_t gu = g[i * K + u];
                int64_t lo = (int64_t)(b & 0xffffffffu);
                int e[4], c[4];
                for (int a = 0; a < 4; ++a) e[a] = (int)((b >> (32 + 8 * a)) & 0xffu);
                int64_t r = lo;
                c[0] = (int)(r % dims[0]);
                r /= dims[0];
                c[1] = (int)(r % dims[1]);
                r /= dims[1];
                c[2] = (int)(r % dims[2]);
                r /= dims[2];
                c[3] = (int)r;
                if (lo >= ncell) return OR_EINVAL;
                for (int a = 0; a < 4; ++a)
                    if (c[a] + e[a] >= dims[a]) return OR_EINVAL;
                if (IS_INF_I32(gu)) continue;
                int32_t mx = INT32_MIN;
                int inf = 0;
                for (int j3 = 0; j3 <= e[3] && !inf; ++j3)
                    for (int j2 = 0; j2 <= e[2] && !inf; ++j2)
                        for (int j1 = 0; j1 <= e[1] && !inf; ++j1)
                            for (int j0 = 0; j0 <= e[0]; ++j0) {
                                int32_t vy = V[lo + j0 + j1 * s1 + j2 * s2 + j3 * s3];
                                if (IS_INF_I32(vy)) {
                                    inf = 1;
                                    break;
                                }
                                if (vy > mx) mx = vy;
                            }
                if (inf) continue;
                int32_t d;
                if (backup_i32(gu, mx, &d, &dummy) && d < best) best = d;
            }
            ok = best == V[x];
        }
        if (!ok) {
            if (bad_out && bad < 16) bad_out[bad] = x;
            ++bad;
        }
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* Independent solver for non-negative running costs: a min-max        */
/* Dijkstra (Knuth's generalisation to superior functions, 1977).      */
/* States are settled in order of value; a pair becomes a candidate    */
/* when its last successor settles (without per-edge costs that one    */
/* holds the max).  int32 costs only; returns OR_EINVAL if some finite */
/* g < 0 or some per-edge cost is negative.                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t key;
    int32_t x;
} or_heap_item;

static void heap_push(or_heap_item* h, int64_t* len, int64_t key, int32_t x) {
    int64_t i = (*len)++;
    h[i].key = key;
    h[i].x = x;
    while (i > 0) {
        int64_t pa = (i - 1) / 2;
        if (h[pa].key <= h[i].key) break;
        or_heap_item t = h[pa];
        h[pa] = h[i];
        h[i] = t;
        i = pa;
    }
}

static or_heap_item heap_pop(or_heap_item* h, int64_t* len) {
    or_heap_item top = h[0];
    h[0] = h[--(*len)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *len && h[l].key < h[s].key) s = l;
        if (r < *len && h[r].key < h[s].key) s = r;
        if (s == i) break;
        or_heap_item t = h[s];
        h[s] = h[i];
        h[i] = t;
        i = s;
    }
    return top;
}

int oracle_dijkstra_i32(int64_t n, int64_t K, const int64_t* sp, const int32_t* si, const int32_t* g,
                        const int32_t* h, const int32_t* G, const uint8_t* avoid, int32_t* W) {
    int rc = check_graph(n, K, sp, si);
    if (rc) return rc;
    int64_t np = n * K;
    for (int64_t p = 0; p < np; ++p)
        if (!IS_INF_I32(g[p]) && g[p] < 0) return OR_EINVAL;
    if (h)
        for (int64_t e = 0; e < sp[np]; ++e)
            if (h[e] < 0 || IS_INF_I32(h[e])) return OR_EINVAL;
    /* reverse lists at pair level (with multiplicity) */
    int64_t m = sp[np];
    int64_t* rp = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* rv = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t* cnt = (int64_t*)malloc((size_t)np * sizeof(int64_t));
    int64_t* tent = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    uint8_t* done = (uint8_t*)calloc((size_t)n, 1);
    int64_t hcap = m + n + 1;
    or_heap_item* heap = (or_heap_item*)malloc((size_t)hcap * sizeof(or_heap_item));
    int64_t* fill = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!rp || !rv || !cnt || !tent || !done || !heap || !fill) {
        free(rp); free(rv); free(cnt); free(tent); free(done); free(heap); free(fill);
        return OR_ENOMEM;
    }
    for (int64_t e = 0; e < m; ++e) rp[si[e] + 1]++;
    for (int64_t y = 0; y < n; ++y) rp[y + 1] += rp[y];
    for (int64_t y = 0; y < n; ++y) fill[y] = rp[y];
    for (int64_t p = 0; p < np; ++p) {
        cnt[p] = sp[p + 1] - sp[p];
        for (int64_t e = sp[p]; e < sp[p + 1]; ++e) rv[fill[si[e]]++] = (int32_t)p;
    }
    int64_t hl = 0;
    for (int64_t x = 0; x < n; ++x) {
        tent[x] = (avoid && avoid[x]) ? OR_INF_I32 : (int64_t)G[x];
        if (tent[x] < OR_INF_I32) heap_push(heap, &hl, tent[x], (int32_t)x);
    }
    while (hl > 0) {
        or_heap_item it = heap_pop(heap, &hl);
        int32_t x = it.x;
        if (done[x] || it.key != tent[x]) continue;
        done[x] = 1;
        for (int64_t e = rp[x]; e < rp[x + 1]; ++e) {
            int64_t p = rv[e];
            if (--cnt[p] != 0) continue;
            int64_t xp = p / K;
            if ((avoid && avoid[xp]) || done[xp] || IS_INF_I32(g[p])) continue;
            /* all successors are settled: without h the last one has the
             * largest value; with h the max is taken over the row */
            int64_t mx = it.key;
            if (h) {
                mx = 0;
                for (int64_t e2 = sp[p]; e2 < sp[p + 1]; ++e2) {
                    int64_t v = (int64_t)h[e2] + tent[si[e2]];
                    if (e2 == sp[p] || v > mx) mx = v;
                }
            }
            int64_t d = (int64_t)g[p] + mx;
            if (d < tent[xp]) {
                tent[xp] = d;
                heap_push(heap, &hl, d, (int32_t)xp);
            }
        }
    }
    for (int64_t x = 0; x < n; ++x) W[x] = done[x] ? (int32_t)tent[x] : (int32_t)INT32_MAX;
    free(rp); free(rv); free(cnt); free(tent); free(done); free(heap); free(fill);
    return OR_OK;
}
