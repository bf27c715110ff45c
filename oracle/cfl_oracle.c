/*
 * Plain CPU oracle for context-free and regular path querying.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP
 * library: it computes the plain definitions, not the Kronecker method.
 *
 * 1. oracle_cfl: CFL-reachability by the textbook worklist over a grammar in
 *    the normal form  A -> eps | A -> t | A -> B | A -> B C.
 *    Definition followed: reachability semantics (Sec. 2.1, Def. of R) with a
 *    context-free language (Sec. 2.3, derivation and L(G)); Theorem 1 states
 *    that the index-creation algorithm reaches exactly this relation.
 *    A fact (A,u,v) means "some path u..v spells a word derivable from A".
 *      init:  (A,u,u) for every rule A -> eps and every vertex u;
 *             (A,u,v) for every edge (u,t,v) and rule A -> t.
 *      pop (B,u,v):
 *             A -> B      gives (A,u,v)
 *             A -> B C    joins with every known (C,v,w), gives (A,u,w)
 *             A -> C B    joins with every known (C,w,u), gives (A,w,v)
 *    Each fact is inserted into its row and column sets when discovered and
 *    pushed once; whichever fact of a joinable pair is popped second sees the
 *    other, so every derivation is found.  Terminates: finitely many facts.
 *
 * 2. oracle_rpq_rows: regular path query by breadth-first search over the
 *    product of the graph with an epsilon-NFA (Sec. 2.2: the graph read as an
 *    automaton whose states are all start and final, intersected with the
 *    query automaton).  One search per requested source vertex; a vertex v
 *    is in the source's row iff some product node (v, q) with q final is
 *    reachable from (source, q0).  Sources are independent, so they may run
 *    on several threads.
 *
 * 3. oracle_cfl_rounds: the relation of 1. as the least fixpoint of the
 *    normal-form grammar read as equations over relations, evaluated in
 *    semi-naive rounds on n x n bitsets (for graphs too large for the
 *    worklist's per-fact joins); see its own comment.
 *
 * 4. oracle_pairs_hash, oracle_groups_hash: pair count and the
 *    order-independent hash (sum of SplitMix64 over (u << 32) | v) of a pair
 *    set given as bitmap rows or as a union of squares G x G, for comparing
 *    relations too large to keep as bitmaps.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EMPTY_KEY 0xFFFFFFFFu

/* ------------------------------------------------------------------ */
/* A set of vertex ids: insertion-ordered list for iteration, plus a   */
/* hash table (small sets) or a bitset (large sets) for membership.    */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t count, cap;   /* list */
    uint32_t *list;
    uint32_t hcap;         /* power of two, 0 = no table */
    uint32_t *hash;
    uint64_t *bits;        /* non-NULL once upgraded */
} vset;

static uint32_t g_n;            /* vertex count of the current call */
static int g_oom;

static uint32_t mix32(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

static int vset_has(const vset *s, uint32_t v) {
    if (s->bits) return (int)((s->bits[v >> 6] >> (v & 63)) & 1u);
    if (!s->hcap) return 0;
    uint32_t m = s->hcap - 1, i = mix32(v) & m;
    for (;;) {
        uint32_t k = s->hash[i];
        if (k == v) return 1;
        if (k == EMPTY_KEY) return 0;
        i = (i + 1) & m;
    }
}

static void hash_put(uint32_t *tab, uint32_t cap, uint32_t v) {
    uint32_t m = cap - 1, i = mix32(v) & m;
    while (tab[i] != EMPTY_KEY) i = (i + 1) & m;
    tab[i] = v;
}

/* returns 1 if v was not in the set */
static int vset_add(vset *s, uint32_t v) {
    if (vset_has(s, v)) return 0;
    if (s->count == s->cap) {
        uint32_t nc = s->cap ? s->cap * 2 : 4;
        uint32_t *nl = (uint32_t *)realloc(s->list, (size_t)nc * sizeof(uint32_t));
        if (!nl) { g_oom = 1; return 0; }
        s->list = nl; s->cap = nc;
    }
    s->list[s->count++] = v;
    if (s->bits) {
        s->bits[v >> 6] |= 1ull << (v & 63);
        return 1;
    }
    uint32_t words = (g_n + 63) / 64;
    if (s->count > 16 && (uint64_t)s->count * 64 > (uint64_t)g_n) {
        /* large: switch membership to a bitset */
        s->bits = (uint64_t *)calloc(words, sizeof(uint64_t));
        if (!s->bits) { g_oom = 1; return 0; }
        for (uint32_t i = 0; i < s->count; i++) s->bits[s->list[i] >> 6] |= 1ull << (s->list[i] & 63);
        free(s->hash); s->hash = NULL; s->hcap = 0;
        return 1;
    }
    if ((uint64_t)s->count * 2 > s->hcap) {
        uint32_t nc = s->hcap ? s->hcap * 2 : 16;
        while ((uint64_t)s->count * 2 > nc) nc *= 2;
        uint32_t *nt = (uint32_t *)malloc((size_t)nc * sizeof(uint32_t));
        if (!nt) { g_oom = 1; return 0; }
        memset(nt, 0xFF, (size_t)nc * sizeof(uint32_t));
        for (uint32_t i = 0; i < s->count; i++) hash_put(nt, nc, s->list[i]);
        free(s->hash); s->hash = nt; s->hcap = nc;
    } else {
        hash_put(s->hash, s->hcap, v);
    }
    return 1;
}

static void vset_free(vset *s) { free(s->list); free(s->hash); free(s->bits); }

/* ------------------------------------------------------------------ */
/* worklist CFL-reachability                                          */
/* ------------------------------------------------------------------ */
enum { R_EPS = 0, R_TERM = 1, R_UNIT = 2, R_BIN = 3 };

typedef struct { uint32_t a, u, v; } fact;

typedef struct {
    fact *buf; size_t len, cap;
} fstack;

static void push(fstack *st, uint32_t a, uint32_t u, uint32_t v) {
    if (st->len == st->cap) {
        size_t nc = st->cap ? st->cap * 2 : 1024;
        fact *nb = (fact *)realloc(st->buf, nc * sizeof(fact));
        if (!nb) { g_oom = 1; return; }
        st->buf = nb; st->cap = nc;
    }
    st->buf[st->len].a = a; st->buf[st->len].u = u; st->buf[st->len].v = v;
    st->len++;
}

typedef struct {
    vset *rows;   /* [A*n + u] : {v : (A,u,v)} */
    vset *cols;   /* [A*n + v] : {u : (A,u,v)} */
    fstack st;
    uint64_t n_facts;
} kb;

static void add_fact(kb *k, uint32_t a, uint32_t u, uint32_t v) {
    size_t n = g_n;
    if (vset_add(&k->rows[(size_t)a * n + u], v)) {
        vset_add(&k->cols[(size_t)a * n + v], u);
        push(&k->st, a, u, v);
        k->n_facts++;
    }
}

/*
 * n vertices; m edges (src[i], lbl[i], dst[i]); duplicate edges allowed.
 * n_nt nonterminals; n_rules rules: kind[r], lhs[r], x[r], y[r]
 *   R_EPS : lhs -> eps            (x, y unused)
 *   R_TERM: lhs -> terminal x     (x is an edge label)
 *   R_UNIT: lhs -> nonterminal x
 *   R_BIN : lhs -> x y            (x, y nonterminals)
 * For each of the n_out nonterminals out_nt[k]: out_bits[k] receives the
 * row-major n x ceil(n/64) bitmap (bit v of row u, LSB first) when
 * out_bits != NULL, and out_count[k] the number of pairs.
 * Returns 0, or -1 on bad input, -2 when memory runs out.
 */
int oracle_cfl(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *lbl, const uint32_t *dst,
               uint32_t n_nt, uint32_t n_rules, const uint32_t *kind, const uint32_t *lhs,
               const uint32_t *x, const uint32_t *y,
               uint32_t n_out, const uint32_t *out_nt, uint64_t *out_bits, uint64_t *out_count,
               uint64_t *total_facts)
{
    g_n = n; g_oom = 0;
    for (uint32_t r = 0; r < n_rules; r++) {
        if (lhs[r] >= n_nt) return -1;
        if (kind[r] == R_UNIT && x[r] >= n_nt) return -1;
        if (kind[r] == R_BIN && (x[r] >= n_nt || y[r] >= n_nt)) return -1;
        if (kind[r] > R_BIN) return -1;
    }
    for (uint64_t i = 0; i < m; i++) if (src[i] >= n || dst[i] >= n) return -1;
    for (uint32_t k = 0; k < n_out; k++) if (out_nt[k] >= n_nt) return -1;

    kb k;
    memset(&k, 0, sizeof(k));
    size_t cells = (size_t)n_nt * n;
    k.rows = (vset *)calloc(cells ? cells : 1, sizeof(vset));
    k.cols = (vset *)calloc(cells ? cells : 1, sizeof(vset));
    if (!k.rows || !k.cols) { free(k.rows); free(k.cols); return -2; }

    /* rules indexed by the nonterminal that a popped fact carries */
    uint32_t *unit_cnt = (uint32_t *)calloc(n_nt + 1, sizeof(uint32_t));
    uint32_t *left_cnt = (uint32_t *)calloc(n_nt + 1, sizeof(uint32_t));
    uint32_t *right_cnt = (uint32_t *)calloc(n_nt + 1, sizeof(uint32_t));
    for (uint32_t r = 0; r < n_rules; r++) {
        if (kind[r] == R_UNIT) unit_cnt[x[r] + 1]++;
        if (kind[r] == R_BIN) { left_cnt[x[r] + 1]++; right_cnt[y[r] + 1]++; }
    }
    for (uint32_t a = 0; a < n_nt; a++) {
        unit_cnt[a + 1] += unit_cnt[a]; left_cnt[a + 1] += left_cnt[a]; right_cnt[a + 1] += right_cnt[a];
    }
    uint32_t *unit_r = (uint32_t *)malloc((unit_cnt[n_nt] + 1) * sizeof(uint32_t));
    uint32_t *left_r = (uint32_t *)malloc((left_cnt[n_nt] + 1) * sizeof(uint32_t));
    uint32_t *right_r = (uint32_t *)malloc((right_cnt[n_nt] + 1) * sizeof(uint32_t));
    uint32_t *fu = (uint32_t *)calloc(n_nt + 1, sizeof(uint32_t));
    uint32_t *fl = (uint32_t *)calloc(n_nt + 1, sizeof(uint32_t));
    uint32_t *fr = (uint32_t *)calloc(n_nt + 1, sizeof(uint32_t));
    for (uint32_t r = 0; r < n_rules; r++) {
        if (kind[r] == R_UNIT) unit_r[unit_cnt[x[r]] + fu[x[r]]++] = r;
        if (kind[r] == R_BIN) {
            left_r[left_cnt[x[r]] + fl[x[r]]++] = r;
            right_r[right_cnt[y[r]] + fr[y[r]]++] = r;
        }
    }

    /* initial facts */
    for (uint32_t r = 0; r < n_rules; r++) {
        if (kind[r] == R_EPS)
            for (uint32_t u = 0; u < n; u++) add_fact(&k, lhs[r], u, u);
        if (kind[r] == R_TERM)
            for (uint64_t i = 0; i < m; i++)
                if (lbl[i] == x[r]) add_fact(&k, lhs[r], src[i], dst[i]);
    }

    /* worklist */
    while (k.st.len && !g_oom) {
        fact f = k.st.buf[--k.st.len];
        uint32_t b = f.a, u = f.u, v = f.v;
        for (uint32_t i = unit_cnt[b]; i < unit_cnt[b + 1]; i++)
            add_fact(&k, lhs[unit_r[i]], u, v);
        /* A -> B C with this fact as B: join with row v of C */
        for (uint32_t i = left_cnt[b]; i < left_cnt[b + 1]; i++) {
            uint32_t r = left_r[i], a = lhs[r], c = y[r];
            vset *row = &k.rows[(size_t)c * n + v];
            uint32_t cnt = row->count;       /* later members are still on the stack */
            for (uint32_t j = 0; j < cnt; j++) add_fact(&k, a, u, row->list[j]);
        }
        /* A -> C B with this fact as B: join with column u of C */
        for (uint32_t i = right_cnt[b]; i < right_cnt[b + 1]; i++) {
            uint32_t r = right_r[i], a = lhs[r], c = x[r];
            vset *col = &k.cols[(size_t)c * n + u];
            uint32_t cnt = col->count;
            for (uint32_t j = 0; j < cnt; j++) add_fact(&k, a, col->list[j], v);
        }
    }

    int rc = g_oom ? -2 : 0;
    if (!rc) {
        uint64_t words = (n + 63) / 64;
        for (uint32_t o = 0; o < n_out; o++) {
            uint32_t a = out_nt[o];
            uint64_t cnt = 0;
            uint64_t *bm = out_bits ? out_bits + (size_t)o * n * words : NULL;
            if (bm) memset(bm, 0, (size_t)n * words * sizeof(uint64_t));
            for (uint32_t u = 0; u < n; u++) {
                vset *row = &k.rows[(size_t)a * n + u];
                cnt += row->count;
                if (bm)
                    for (uint32_t j = 0; j < row->count; j++) {
                        uint32_t v = row->list[j];
                        bm[(size_t)u * words + (v >> 6)] |= 1ull << (v & 63);
                    }
            }
            if (out_count) out_count[o] = cnt;
        }
        if (total_facts) *total_facts = k.n_facts;
    }

    for (size_t i = 0; i < cells; i++) { vset_free(&k.rows[i]); vset_free(&k.cols[i]); }
    free(k.rows); free(k.cols); free(k.st.buf);
    free(unit_cnt); free(left_cnt); free(right_cnt);
    free(unit_r); free(left_r); free(right_r); free(fu); free(fl); free(fr);
    return rc;
}

/* ------------------------------------------------------------------ */
/* product-automaton BFS for regular path queries                     */
/* ------------------------------------------------------------------ */
#define EPS_LABEL 0xFFFFFFFFu

/*
 * NFA: nq states, ntr transitions (tsrc, tlbl, tdst), tlbl == EPS_LABEL for an
 * epsilon move; start state q0; final[q] != 0 for accepting states.
 * For each source sources[i], out_rows[i] (ceil(n/64) words) receives the set
 * of v with (source, v) in the answer.  visits (optional) receives the number
 * of product nodes visited over all sources.
 */
int oracle_rpq_rows(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *lbl, const uint32_t *dst,
                    uint32_t n_labels, uint32_t nq, uint32_t ntr, const uint32_t *tsrc, const uint32_t *tlbl,
                    const uint32_t *tdst, uint32_t q0, const uint8_t *final, uint32_t n_sources,
                    const uint32_t *sources, uint64_t *out_rows, int threads, uint64_t *visits)
{
    if (q0 >= nq) return -1;
    for (uint64_t i = 0; i < m; i++)
        if (src[i] >= n || dst[i] >= n || lbl[i] >= n_labels) return -1;
    for (uint32_t t = 0; t < ntr; t++)
        if (tsrc[t] >= nq || tdst[t] >= nq || (tlbl[t] != EPS_LABEL && tlbl[t] >= n_labels)) return -1;
    for (uint32_t i = 0; i < n_sources; i++) if (sources[i] >= n) return -1;

    /* out-edges grouped by (vertex, label) */
    size_t keys = (size_t)n * n_labels;
    uint64_t *off = (uint64_t *)calloc(keys + 1, sizeof(uint64_t));
    uint32_t *adj = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint64_t *fill = (uint64_t *)calloc(keys + 1, sizeof(uint64_t));
    if (!off || !adj || !fill) { free(off); free(adj); free(fill); return -2; }
    for (uint64_t i = 0; i < m; i++) off[(size_t)src[i] * n_labels + lbl[i] + 1]++;
    for (size_t kk = 0; kk < keys; kk++) off[kk + 1] += off[kk];
    for (uint64_t i = 0; i < m; i++) {
        size_t key = (size_t)src[i] * n_labels + lbl[i];
        adj[off[key] + fill[key]++] = dst[i];
    }
    free(fill);
    /* NFA transitions grouped by source state */
    uint32_t *toff = (uint32_t *)calloc(nq + 1, sizeof(uint32_t));
    uint32_t *tord = (uint32_t *)malloc((ntr ? ntr : 1) * sizeof(uint32_t));
    uint32_t *tf = (uint32_t *)calloc(nq + 1, sizeof(uint32_t));
    for (uint32_t t = 0; t < ntr; t++) toff[tsrc[t] + 1]++;
    for (uint32_t q = 0; q < nq; q++) toff[q + 1] += toff[q];
    for (uint32_t t = 0; t < ntr; t++) tord[toff[tsrc[t]] + tf[tsrc[t]]++] = t;
    free(tf);

    uint64_t words = (n + 63) / 64;
    uint64_t total_visits = 0;
    int nthreads = threads > 0 ? threads : 1;

#pragma omp parallel num_threads(nthreads) reduction(+ : total_visits)
    {
        size_t pn = (size_t)n * nq;
        uint64_t *seen = (uint64_t *)calloc((pn + 63) / 64, sizeof(uint64_t));
        uint64_t *queue = (uint64_t *)malloc((pn ? pn : 1) * sizeof(uint64_t));
#pragma omp for schedule(dynamic, 4)
        for (uint32_t si = 0; si < n_sources; si++) {
            uint64_t *row = out_rows + (size_t)si * words;
            memset(row, 0, words * sizeof(uint64_t));
            size_t head = 0, tail = 0;
            /* product node id = v * nq + q */
            size_t start = (size_t)sources[si] * nq + q0;
            seen[start >> 6] |= 1ull << (start & 63);
            queue[tail++] = start;
            while (head < tail) {
                size_t node = queue[head++];
                uint32_t v = (uint32_t)(node / nq), q = (uint32_t)(node % nq);
                if (final[q]) row[v >> 6] |= 1ull << (v & 63);
                for (uint32_t j = toff[q]; j < toff[q + 1]; j++) {
                    uint32_t t = tord[j];
                    if (tlbl[t] == EPS_LABEL) {
                        size_t nx = (size_t)v * nq + tdst[t];
                        if (!((seen[nx >> 6] >> (nx & 63)) & 1)) {
                            seen[nx >> 6] |= 1ull << (nx & 63);
                            queue[tail++] = nx;
                        }
                    } else {
                        size_t key = (size_t)v * n_labels + tlbl[t];
                        for (uint64_t e = off[key]; e < off[key + 1]; e++) {
                            size_t nx = (size_t)adj[e] * nq + tdst[t];
                            if (!((seen[nx >> 6] >> (nx & 63)) & 1)) {
                                seen[nx >> 6] |= 1ull << (nx & 63);
                                queue[tail++] = nx;
                            }
                        }
                    }
                }
            }
            total_visits += tail;
            /* clear only what this search touched */
            for (size_t i = 0; i < tail; i++) {
                size_t nd = queue[i];
                seen[nd >> 6] &= ~(1ull << (nd & 63));
            }
        }
        free(seen); free(queue);
    }
    if (visits) *visits = total_visits;
    free(off); free(adj); free(toff); free(tord);
    return 0;
}

/* ------------------------------------------------------------------ */
/* semi-naive rounds over relation bitsets                             */
/* ------------------------------------------------------------------ */
/*
 * 3. oracle_cfl_rounds: the same relation as oracle_cfl (same normal form,
 *    same arguments), computed as the least fixpoint of the grammar read as
 *    equations over binary relations on the vertices:
 *        R_A  contains  the diagonal          for A -> eps
 *             contains  the edges of label t  for A -> t
 *             contains  R_B                   for A -> B
 *             contains  R_B ; R_C             for A -> B C
 *    (";" is relational composition: (u, w) with some v, (u,v) in R_B and
 *    (v,w) in R_C).  Round 0 holds the eps and terminal facts.  Round k+1
 *    adds what the unit and binary rules derive from facts of which at least
 *    one is new in round k (semi-naive evaluation: a pair of two older facts
 *    was already composed in an earlier round); it stops when a round adds
 *    nothing.  Every relation is an n x n bitset (row u: the v with (u, v)):
 *    3 n^2/8 bytes per nonterminal (the relation, last round's new facts,
 *    this round's derived facts).  Bookkeeping only, so that a round costs
 *    what its new facts cost: the rows holding new facts are listed, and the
 *    rows a round writes are flagged.  Rows of one composition are computed
 *    in parallel on `threads` threads.  rounds (optional) receives the number
 *    of rounds, the last (empty) one included.
 * Returns 0, -1 on bad input, -2 when memory runs out.
 */
typedef struct {
    uint64_t *rel, *cur, *nxt;   /* n * W words each */
    uint32_t *cur_rows;          /* rows of cur that hold a fact, cur_nrows of them */
    uint32_t cur_nrows;
    uint8_t *touched;            /* [n]: row of nxt written this round */
    uint64_t rel_count, cur_count;
} relset;

/* out |= X ; Y over the rows u in rows[0..nrows) (or all n rows if rows is
 * NULL): out[u] = OR of Y[v] over v in X[u].  When Y holds few pairs its rows
 * are walked as lists (built here), otherwise they are OR-ed word by word;
 * X[u] is first restricted to the v whose Y row is non-empty. */
static int compose_into(uint64_t *out, uint8_t *touched, const uint64_t *X, const uint32_t *rows, uint32_t nrows,
                        const uint64_t *Y, uint64_t y_count, uint32_t n, uint64_t W, int threads) {
    uint64_t *ynz = (uint64_t *)calloc(W ? W : 1, sizeof(uint64_t));
    if (!ynz) return -2;
    for (uint32_t v = 0; v < n; v++) {
        const uint64_t *row = Y + (uint64_t)v * W;
        for (uint64_t k = 0; k < W; k++)
            if (row[k]) { ynz[v >> 6] |= 1ull << (v & 63); break; }
    }
    /* lists when the average Y row has fewer than W/8 pairs */
    int lists = y_count * 8 < (uint64_t)n * W;
    uint64_t *yoff = NULL;
    uint32_t *ycol = NULL;
    if (lists) {
        yoff = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
        ycol = (uint32_t *)malloc((y_count ? y_count : 1) * sizeof(uint32_t));
        if (!yoff || !ycol) { free(yoff); free(ycol); free(ynz); return -2; }
        uint64_t at = 0;
        for (uint32_t v = 0; v < n; v++) {
            yoff[v] = at;
            const uint64_t *row = Y + (uint64_t)v * W;
            for (uint64_t k = 0; k < W; k++)
                for (uint64_t b = row[k]; b; b &= b - 1) ycol[at++] = (uint32_t)(k * 64 + __builtin_ctzll(b));
        }
        yoff[n] = at;
    }
    const int64_t count = rows ? (int64_t)nrows : (int64_t)n;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 64)
    for (int64_t i = 0; i < count; i++) {
        const uint32_t u = rows ? rows[i] : (uint32_t)i;
        const uint64_t *xr = X + (uint64_t)u * W;
        uint64_t *orow = out + (uint64_t)u * W;
        int wrote = 0;
        for (uint64_t k = 0; k < W; k++) {
            for (uint64_t b = xr[k] & ynz[k]; b; b &= b - 1) {
                uint32_t v = (uint32_t)(k * 64 + __builtin_ctzll(b));
                wrote = 1;
                if (lists) {
                    for (uint64_t e = yoff[v]; e < yoff[v + 1]; e++) {
                        uint32_t w = ycol[e];
                        orow[w >> 6] |= 1ull << (w & 63);
                    }
                } else {
                    const uint64_t *yr = Y + (uint64_t)v * W;
                    for (uint64_t j = 0; j < W; j++) orow[j] |= yr[j];
                }
            }
        }
        if (wrote) touched[u] = 1;
    }
    free(yoff); free(ycol); free(ynz);
    return 0;
}

int oracle_cfl_rounds(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *lbl, const uint32_t *dst,
                      uint32_t n_nt, uint32_t n_rules, const uint32_t *kind, const uint32_t *lhs,
                      const uint32_t *x, const uint32_t *y,
                      uint32_t n_out, const uint32_t *out_nt, uint64_t *out_bits, uint64_t *out_count,
                      int threads, uint32_t *rounds)
{
    for (uint32_t r = 0; r < n_rules; r++) {
        if (lhs[r] >= n_nt) return -1;
        if (kind[r] == R_UNIT && x[r] >= n_nt) return -1;
        if (kind[r] == R_BIN && (x[r] >= n_nt || y[r] >= n_nt)) return -1;
        if (kind[r] > R_BIN) return -1;
    }
    for (uint64_t i = 0; i < m; i++) if (src[i] >= n || dst[i] >= n) return -1;
    for (uint32_t k = 0; k < n_out; k++) if (out_nt[k] >= n_nt) return -1;
    if (threads < 1) threads = 1;

    const uint64_t W = (n + 63) / 64, words = (uint64_t)n * W;
    relset *R = (relset *)calloc(n_nt ? n_nt : 1, sizeof(relset));
    if (!R) return -2;
    int rc = 0;
    for (uint32_t a = 0; a < n_nt && !rc; a++) {
        R[a].rel = (uint64_t *)calloc(words ? words : 1, sizeof(uint64_t));
        R[a].cur = (uint64_t *)calloc(words ? words : 1, sizeof(uint64_t));
        R[a].nxt = (uint64_t *)calloc(words ? words : 1, sizeof(uint64_t));
        R[a].cur_rows = (uint32_t *)malloc(((size_t)n ? n : 1) * sizeof(uint32_t));
        R[a].touched = (uint8_t *)calloc((size_t)n ? n : 1, 1);
        if (!R[a].rel || !R[a].cur || !R[a].nxt || !R[a].cur_rows || !R[a].touched) rc = -2;
    }
    /* round 0: eps and terminal facts, all of them new; they are gathered in
     * nxt and enter like any round's derived facts */
    for (uint32_t r = 0; r < n_rules && !rc; r++) {
        relset *A = &R[lhs[r]];
        if (kind[r] == R_EPS)
            for (uint32_t u = 0; u < n; u++) {
                A->nxt[(uint64_t)u * W + (u >> 6)] |= 1ull << (u & 63);
                A->touched[u] = 1;
            }
        if (kind[r] == R_TERM)
            for (uint64_t i = 0; i < m; i++)
                if (lbl[i] == x[r]) {
                    A->nxt[(uint64_t)src[i] * W + (dst[i] >> 6)] |= 1ull << (dst[i] & 63);
                    A->touched[src[i]] = 1;
                }
    }
    uint32_t nr = 0;
    for (;;) {
        if (rc) break;
        /* merge: the derived facts not yet known are the new facts */
        int any_new = 0;
        for (uint32_t a = 0; a < n_nt; a++) {
            relset *A = &R[a];
            /* last round's new-fact rows are cleared; nxt becomes the new cur */
            for (uint32_t i = 0; i < A->cur_nrows; i++)
                memset(A->cur + (uint64_t)A->cur_rows[i] * W, 0, W * sizeof(uint64_t));
            uint32_t nrows = 0;
            uint64_t c = 0;
            for (uint32_t u = 0; u < n; u++) {
                if (!A->touched[u]) continue;
                A->touched[u] = 0;
                uint64_t *nx = A->nxt + (uint64_t)u * W, *rl = A->rel + (uint64_t)u * W;
                uint64_t cu = 0;
                for (uint64_t k = 0; k < W; k++) {
                    uint64_t nw = nx[k] & ~rl[k];
                    nx[k] = nw;
                    rl[k] |= nw;
                    cu += (uint64_t)__builtin_popcountll(nw);
                }
                if (cu) A->cur_rows[nrows++] = u;
                else memset(nx, 0, W * sizeof(uint64_t));
                c += cu;
            }
            uint64_t *t = A->cur; A->cur = A->nxt; A->nxt = t;
            A->cur_nrows = nrows;
            A->cur_count = c;
            A->rel_count += c;
            any_new |= c != 0;
        }
        nr++;
        if (!any_new) break;
        /* derive: every rule, reading rel and cur, writing nxt */
        for (uint32_t r = 0; r < n_rules && !rc; r++) {
            relset *A = &R[lhs[r]];
            if (kind[r] == R_UNIT) {
                const relset *B = &R[x[r]];
                for (uint32_t i = 0; i < B->cur_nrows; i++) {
                    const uint32_t u = B->cur_rows[i];
                    const uint64_t *bs = B->cur + (uint64_t)u * W;
                    uint64_t *ad = A->nxt + (uint64_t)u * W;
                    for (uint64_t k = 0; k < W; k++) ad[k] |= bs[k];
                    A->touched[u] = 1;
                }
            } else if (kind[r] == R_BIN) {
                const relset *B = &R[x[r]], *C = &R[y[r]];
                /* new ; all  and  all ; new */
                if (B->cur_count && C->rel_count)
                    rc = compose_into(A->nxt, A->touched, B->cur, B->cur_rows, B->cur_nrows, C->rel, C->rel_count, n,
                                      W, threads);
                if (!rc && B->rel_count && C->cur_count)
                    rc = compose_into(A->nxt, A->touched, B->rel, NULL, 0, C->cur, C->cur_count, n, W, threads);
            }
        }
    }
    if (!rc) {
        for (uint32_t o = 0; o < n_out; o++) {
            const relset *A = &R[out_nt[o]];
            if (out_bits) memcpy(out_bits + (uint64_t)o * words, A->rel, words * sizeof(uint64_t));
            if (out_count) out_count[o] = A->rel_count;
        }
        if (rounds) *rounds = nr;
    }
    for (uint32_t a = 0; a < n_nt; a++) {
        free(R[a].rel); free(R[a].cur); free(R[a].nxt); free(R[a].cur_rows); free(R[a].touched);
    }
    free(R);
    return rc;
}

/* ------------------------------------------------------------------ */
/* count and order-independent hash of a pair set                      */
/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014): the first output of the generator
 * seeded with z: z + golden gamma, then the two xor-shift-multiply steps
 * and a final xor-shift, as published. */
static uint64_t sm64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* rows of a row-major bitmap: row i is vertex row_ids[i] (or i if row_ids is
 * NULL); adds to *count the pairs and to *hash the sum of
 * splitmix64((u << 32) | v) over them (mod 2^64) */
void oracle_pairs_hash(uint32_t n, uint64_t n_rows, const uint32_t *row_ids, const uint64_t *bits, int threads,
                       uint64_t *count, uint64_t *hash)
{
    const uint64_t W = (n + 63) / 64;
    uint64_t c = 0, h = 0;
    if (threads < 1) threads = 1;
#pragma omp parallel for num_threads(threads) reduction(+ : c, h) schedule(static)
    for (uint64_t i = 0; i < n_rows; i++) {
        uint64_t u = row_ids ? row_ids[i] : i;
        const uint64_t *row = bits + i * W;
        for (uint64_t k = 0; k < W; k++)
            for (uint64_t b = row[k]; b; b &= b - 1) {
                uint64_t v = k * 64 + (uint64_t)__builtin_ctzll(b);
                c++;
                h += sm64((u << 32) | v);
            }
    }
    *count += c;
    *hash += h;
}

/* pairs of a union of full squares G x G over disjoint vertex groups: group g
 * is members[off[g] .. off[g+1]); count and hash as above */
void oracle_groups_hash(uint32_t n_groups, const uint64_t *off, const uint32_t *members, int threads,
                        uint64_t *count, uint64_t *hash)
{
    uint64_t c = 0, h = 0;
    if (threads < 1) threads = 1;
    for (uint32_t g = 0; g < n_groups; g++) {
        int64_t lo = (int64_t)off[g], hi = (int64_t)off[g + 1];
#pragma omp parallel for num_threads(threads) reduction(+ : c, h) schedule(dynamic, 16)
        for (int64_t i = lo; i < hi; i++) {
            uint64_t u = members[i];
            for (int64_t j = lo; j < hi; j++) {
                h += sm64((u << 32) | (uint64_t)members[j]);
                c++;
            }
        }
    }
    *count += c;
    *hash += h;
}
