/*
 * cfpq.h -- C ABI of the MI355X (gfx950) Kronecker-product path-query library.
 *
 * The library evaluates context-free and regular path queries with the
 * index-creation fixpoint of Shemetova et al., "One Algorithm to Evaluate
 * Them All" (Sec. 3.1, Listing 1): the Kronecker product of the query's
 * recursive-state-machine matrices with the graph's label matrices, the
 * incremental transitive closure of the product, and the write-back of new
 * nonterminal edges into the graph, repeated until no edge is added.
 *
 * Conventions for every call:
 *   - Every call returns cfpq_status; CFPQ_OK (0) on success.  No C++
 *     exception crosses this boundary.  cfpq_last_error() returns a
 *     thread-local text for the last non-OK status of the calling thread.
 *   - Inputs are caller-owned and copied during the call; the library keeps
 *     no pointer to caller memory.  Handles are library-owned until their
 *     destroy call.  Output buffers are caller-owned.
 *   - Vertex ids are 0..n-1, label ids 0..n_labels-1 (uint32).
 *   - A bitmap over pairs is row-major: row u holds ceil(n/64) uint64 words,
 *     bit (v % 64) of word (v / 64) set iff (u, v) is in the relation;
 *     bits at v >= n are zero.
 *   - Handles are immutable after creation: queries on different streams
 *     may share a graph and an RSM.  A result must not be destroyed while
 *     another thread uses it.
 *   - Device memory comes from the optional allocator (e.g. PyTorch's caching
 *     allocator), else from hipMalloc.  "stream" arguments are hipStream_t
 *     values passed as void* (NULL = the null stream).
 */
#ifndef CFPQ_H
#define CFPQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CFPQ_OK = 0,
    CFPQ_ERR_INVALID = -1,   /* an argument violates the rules stated below */
    CFPQ_ERR_OOM = -2,       /* device or host allocation failed */
    CFPQ_ERR_DEVICE = -3,    /* a HIP runtime call or kernel launch failed */
    CFPQ_ERR_NOT_FOUND = -4, /* extract_path: the pair is not in the relation */
    CFPQ_ERR_BUFFER = -5,    /* output buffer too small; required size returned */
    CFPQ_ERR_LIMIT = -6,     /* an iteration/size limit of the call was reached */
    CFPQ_ERR_REJECTED = -7   /* the request does not fit the resources given */
} cfpq_status;

typedef struct cfpq_graph_s *cfpq_graph;
typedef struct cfpq_rsm_s *cfpq_rsm;
typedef struct cfpq_result_s *cfpq_result;

/* Device-memory hooks.  alloc returns NULL on failure, else memory aligned
 * to 256 bytes (as hipMalloc's; a less aligned block is handed back to free
 * and the call fails with CFPQ_ERR_OOM); free receives the pointer and size
 * that alloc produced.  Both are called with the stream the memory is used
 * on.  cached may be NULL; otherwise it returns the bytes the allocator holds
 * unused and can hand out again (a caching allocator's free blocks, which
 * the device does not count as free): a query that sizes its buffers by the
 * device's free memory (the source tiles of CFPQ_STRATEGY_LEVELS) counts
 * them too.  Without it, memory such an allocator keeps from earlier calls
 * shrinks those tiles, down to one word. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, size_t bytes, void *stream, void *ctx);
    void *ctx;
    size_t (*cached)(void *ctx);
} cfpq_allocator;

/* ------------------------------------------------------------------------
 * Graph: an edge-labelled directed graph <V, E, L> (Sec. 2.1, definition of
 * an edge-labelled graph) held as its Boolean decomposition, one Boolean
 * matrix per label (Sec. 2.1, Boolean matrices decomposition).  On the
 * device each label matrix is stored by columns: for every vertex v the
 * sorted, duplicate-free list of its predecessors under that label.
 *
 * n_vertices >= 1; n_labels >= 1; src/label/dst: n_edges host arrays.
 * E is a set: duplicate edges collapse; self-loops are kept.
 * flags: CFPQ_ADD_INVERSES adds, for every label l, the inverse label
 *   n_labels + l carrying (v, u) for each (u, l, v) (the inverse relation of
 *   the same-generation and alias queries, Sec. 4.2); the graph then has
 *   2 * n_labels labels.  CFPQ_DEVICE_PTRS: src/label/dst are device
 *   pointers (read on the given stream before the call returns).
 * Errors: CFPQ_ERR_INVALID if n_vertices == 0, n_labels == 0, a vertex
 *   >= n_vertices, a label >= n_labels, a NULL array with n_edges > 0, or
 *   more than 2^32 - 1 distinct edges.
 * The graph stays resident on the current device until cfpq_graph_destroy.
 * ---------------------------------------------------------------------- */
#define CFPQ_ADD_INVERSES 1u
#define CFPQ_DEVICE_PTRS 2u

cfpq_status cfpq_graph_create(uint32_t n_vertices, uint32_t n_labels, const uint32_t *src,
                              const uint32_t *label, const uint32_t *dst, uint64_t n_edges,
                              uint32_t flags, const cfpq_allocator *alloc, void *stream,
                              cfpq_graph *out);
cfpq_status cfpq_graph_info(cfpq_graph g, uint32_t *n_vertices, uint32_t *n_labels,
                            uint64_t *n_edges);
void cfpq_graph_destroy(cfpq_graph g);

/* ------------------------------------------------------------------------
 * Recursive state machine (Sec. 2.3, definition of an RSM): boxes with
 * pairwise disjoint state sets, one initial state each, a set of final
 * states each, and transitions over terminals and box labels.  A regular
 * path query is a one-box RSM with no box-labelled transition (Sec. 3.1.2).
 *
 * n_states states 0..n_states-1; n_boxes boxes 0..n_boxes-1.
 * box_start[b]   : initial state of box b.
 * state_box[q]   : the box owning state q (state sets are disjoint).
 * is_final[q]    : nonzero iff q is a final state of its box.
 * transitions (t_src[i], t_sym[i], t_dst[i]), i < n_trans:
 *   t_sym <  n_terminals : terminal, matched against graph label t_sym;
 *   t_sym >= n_terminals : box label (nonterminal) t_sym - n_terminals.
 * start_box      : the box whose relation is "the answer" (the grammar's
 *                  start nonterminal); every box's relation is computed.
 * Errors: CFPQ_ERR_INVALID if a count is zero, an index is out of range, a
 *   box start is owned by another box, or a transition crosses boxes.
 * The RSM may be nondeterministic; the relation does not depend on that.
 * ---------------------------------------------------------------------- */
cfpq_status cfpq_rsm_create(uint32_t n_states, uint32_t n_terminals, uint32_t n_boxes,
                            const uint32_t *box_start, const uint32_t *state_box,
                            const uint8_t *is_final, const uint32_t *t_src, const uint32_t *t_sym,
                            const uint32_t *t_dst, uint32_t n_trans, uint32_t start_box,
                            cfpq_rsm *out);
void cfpq_rsm_destroy(cfpq_rsm r);

/* ------------------------------------------------------------------------
 * Query: the index-creation fixpoint (Sec. 3.1, Listing 1) on one GPU.
 *
 *   a. epsilon initialisation: every box whose initial state is final gets
 *      all loops (v, v) (Listing 1, before the loop); these loops also count
 *      as new edges of the first iteration;
 *   b. each iteration: Kronecker product of the RSM matrices with the NEW
 *      graph edges only (left-distributivity, Sec. 3.1.1), incremental
 *      transitive closure of the product restricted to the rows that start
 *      at a box's initial state, write-back of new nonterminal edges;
 *   c. stop after the first iteration that adds no nonterminal edge.
 *
 * Options (NULL = defaults):
 *   strategy   : CFPQ_STRATEGY_AUTO, _LEVELS (one launch per closure level,
 *                any size), _FUSED (one workgroup runs the whole fixpoint,
 *                in LDS when its working set fits the device's per-workgroup
 *                LDS and keep_blocks is off; small graphs only,
 *                CFPQ_ERR_LIMIT beyond its size limit),
 *                _CONDENSED (closure through the strongly connected
 *                components of the product graph, each component's row
 *                computed once in topological order; only for RSMs without
 *                box-labelled transitions, i.e. regular queries, else
 *                CFPQ_ERR_INVALID), _PEREDGE (the literal per-edge
 *                incremental closure of Sec. 3.1.1: the closure of the whole
 *                product graph kept as one bitset row per product node, every
 *                new product edge (i, j) added on its own -- each node that
 *                reaches i and not j takes in j's row and j -- in one
 *                workgroup; needs states * n <= 65536, else CFPQ_ERR_LIMIT;
 *                keep_rank and keep_blocks give CFPQ_ERR_INVALID; never
 *                picked by AUTO: it is the comparison arm of the method's
 *                complexity argument).  AUTO picks FUSED for graphs of at
 *                most 512 vertices (and at most 64 boxes), CONDENSED for
 *                other regular queries, LEVELS otherwise.
 *                A CONDENSED query on a graph that has run one before goes
 *                out in one piece, sized by the launch chains the previous
 *                one needed, with a single host read at the end (steps the
 *                sizes did not cover are finished synchronously; the
 *                answer does not depend on it).
 *   max_iters  : 0 = no limit beyond the natural bound; otherwise the query
 *                fails with CFPQ_ERR_LIMIT if the loop has not stopped after
 *                max_iters iterations.
 *   keep_rank  : keep, for every nonterminal pair, the iteration that added
 *                it (one byte per pair of every box, on the device: boxes *
 *                n^2 bytes, at most 64 GiB, else CFPQ_ERR_LIMIT); required by
 *                cfpq_extract_path when the RSM has box-labelled
 *                transitions.
 *   keep_blocks: keep the closure blocks, required by cfpq_result_block.
 *   tile_words : source-tile width in 64-bit words (levels strategy; the
 *                closure runs once per tile of sources).  0 = automatic:
 *                the widest tile whose frontier buffers fit in the free
 *                device memory left after the closure state, at most 1200
 *                words when box-labelled transitions use the sparse product
 *                (narrower tiles keep more frontier rows sparse), split
 *                into equal tiles.
 *   nt_mode    : how box-labelled transitions are multiplied (levels
 *                strategy): CFPQ_NT_AUTO = sparse rows (ELL lists + LDS
 *                accumulators) in the Kronecker seed, and in closure levels
 *                once a row tile spans 16 words or more (below that, whole-row
 *                OR per selector bit); CFPQ_NT_ROWS = whole-row OR
 *                everywhere; CFPQ_NT_MFMA = AUTO's seed plus the exact int8
 *                matrix-core product (v_mfma_i32_32x32x32_i8 on {0,1}
 *                operands, thresholded) in every closure level.  AUTO never
 *                picks the matrix cores: with sparse frontiers the dense
 *                product moves and multiplies far more than the bit-serial OR.
 *                The answer does not depend on the mode.
 *   recompute  : nonzero: every iteration of the levels strategy recomputes
 *                the closure from scratch over the whole M2 (the variant the
 *                paper evaluated, Sec. 6) instead of extending it from the
 *                new edges A2 only (Sec. 3.1.1).  Same answers, iterations
 *                and per-iteration counts; for comparison.
 *   profile    : record HIP events around the closure launches of the
 *                levels and condensed strategies and count the level
 *                kernel's words (see cfpq_result_profile); adds ~1 us per
 *                launch.
 *   stream     : hipStream_t for all work of the call (NULL = null stream).
 *   src_mask, dst_mask: host bitsets of ceil(n/64) words (bit v of word
 *                v / 64, LSB first; bits >= n ignored), NULL = every vertex.
 *                The start box's relation is restricted to sources in
 *                src_mask and targets in dst_mask (the multiple-source
 *                variant, Sec. 6): count, hash, bitmap, pairs and witness
 *                paths of that box see only those pairs.  For a query
 *                without box-labelled transitions only the masked sources
 *                are searched (work shrinks with the mask); for grammars
 *                the nonterminals still need every source, so the mask
 *                filters the answer.  Other boxes' relations, closure
 *                blocks and per-iteration counts are not masked.  Not
 *                accepted by cfpq_query_batch (graphs differ in size).
 * The call returns after the fixpoint has finished on the device.
 * Errors: CFPQ_ERR_INVALID if the RSM uses more terminals than the graph
 *   has labels; CFPQ_ERR_OOM; CFPQ_ERR_DEVICE; CFPQ_ERR_LIMIT.
 * ---------------------------------------------------------------------- */
enum { CFPQ_STRATEGY_AUTO = 0, CFPQ_STRATEGY_LEVELS = 1, CFPQ_STRATEGY_FUSED = 2, CFPQ_STRATEGY_CONDENSED = 3,
       CFPQ_STRATEGY_PEREDGE = 4 };
enum { CFPQ_NT_AUTO = 0, CFPQ_NT_ROWS = 1, CFPQ_NT_MFMA = 2 };

typedef struct {
    uint32_t strategy;
    uint32_t max_iters;
    uint32_t keep_rank;
    uint32_t keep_blocks;
    uint32_t tile_words;
    uint32_t profile;
    uint32_t nt_mode;
    uint32_t recompute;
    void *stream;
    const cfpq_allocator *alloc;
    const uint64_t *src_mask;
    const uint64_t *dst_mask;
} cfpq_query_opts;

cfpq_status cfpq_query(cfpq_graph g, cfpq_rsm r, const cfpq_query_opts *opts, cfpq_result *out);

/* Batched query: k (graph, RSM) pairs evaluated together; small queries
 * share launches (one workgroup per query), the others run one after the
 * other.  results[i] receives the result of pair i; on error every result
 * created so far is destroyed and all results[i] are NULL.  The answers are
 * identical to k separate cfpq_query calls. */
cfpq_status cfpq_query_batch(const cfpq_graph *graphs, const cfpq_rsm *rsms, uint32_t k,
                             const cfpq_query_opts *opts, cfpq_result *results);

/* ------------------------------------------------------------------------
 * Query that allocates no device memory.  For callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It runs the same fixpoint as cfpq_query with
 * CFPQ_STRATEGY_FUSED (one workgroup runs the whole loop) and writes box's
 * relation to dst; every buffer of the query (RSM tables, closure rows,
 * nonterminal matrices, frontiers, counters) lives in one static device array
 * of CFPQ_NOALLOC_SCRATCH_BYTES, which each device the library runs on holds
 * from the first call on it until the process ends.
 *
 * dst       : device pointer, row-major bitmap of n * ceil(n/64) words (see
 *             conventions), caller-owned; dst_words its size.
 * pairs, iterations: host pointers (may be NULL) receiving the number of
 *             pairs of box's relation and the iterations of the loop.
 * stream    : hipStream_t for the work (NULL = null stream); the call returns
 *             after the stream has finished it.
 * The array keeps the last call's contents; a call clears what it needs.
 * Calls share the device's array: the library holds a per-device lock for
 * the whole call, so calls from threads of one process run one at a time,
 * while calls that overlap on one GPU from anywhere else (another process's
 * copy of the library aside, which has its own array) would race.
 * Errors: CFPQ_ERR_INVALID (NULL handles or dst, box out of range, RSM uses
 *   more terminals than the graph has labels, graph on another device);
 *   CFPQ_ERR_BUFFER if dst_words < n * ceil(n/64); CFPQ_ERR_LIMIT if
 *   n > 2048, more than 64 boxes, or the query's working set exceeds
 *   CFPQ_NOALLOC_SCRATCH_BYTES (message states both sizes);
 *   CFPQ_ERR_DEVICE on a failed HIP call.
 * ---------------------------------------------------------------------- */
#define CFPQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

cfpq_status cfpq_query_noalloc(cfpq_graph g, cfpq_rsm r, uint32_t box, uint64_t *dst, uint64_t dst_words,
                               uint64_t *pairs, uint32_t *iterations, void *stream);

/* ------------------------------------------------------------------------
 * Result accessors.  "box" selects a nonterminal; its relation is the set
 * of (u, v) such that some path u..v spells a word the box derives
 * (Theorem 1).
 * ---------------------------------------------------------------------- */
/* number of pairs */
cfpq_status cfpq_result_count(cfpq_result res, uint32_t box, uint64_t *pairs);
/* order-independent hash: sum over pairs of splitmix64((u << 32) | v) mod 2^64
 * (SplitMix64 of Steele, Lea and Flood, 2014) */
cfpq_status cfpq_result_hash(cfpq_result res, uint32_t box, uint64_t *hash);
/* the relation as a row-major bitmap (see conventions); dst_words must be at
 * least n * ceil(n/64), else CFPQ_ERR_BUFFER.  dst_on_device != 0: dst is a
 * device pointer on the result's device. */
cfpq_status cfpq_result_bitmap(cfpq_result res, uint32_t box, uint64_t *dst, uint64_t dst_words,
                               int dst_on_device);
/* the relation as (u, v) pairs, sorted by u then v, into uv[2 * cap_pairs];
 * *n_pairs receives the count; CFPQ_ERR_BUFFER if cap_pairs is too small. */
cfpq_status cfpq_result_pairs(cfpq_result res, uint32_t box, uint32_t *uv, uint64_t cap_pairs,
                              uint64_t *n_pairs);
/* closure block between an initial state q_start and a state q_final of the
 * same box (for a regular query: the start/final state pair of the
 * automaton): bit (u, v) set iff (q_start, u) reaches (q_final, v) in the
 * product graph by a path of length >= 1, or (u == v and q_start ==
 * q_final).  Requires keep_blocks.  Row-major bitmap as above. */
cfpq_status cfpq_result_block(cfpq_result res, uint32_t q_start, uint32_t q_final, uint64_t *dst,
                              uint64_t dst_words);
/* iterations of the loop (including the last, unproductive one), new
 * nonterminal edges per iteration (first min(cap, iterations) entries), and
 * the device time of the fixpoint in milliseconds (events on the query
 * stream, from the first kernel to the last). */
cfpq_status cfpq_result_stats(cfpq_result res, uint32_t *iterations, uint64_t *delta_per_iter,
                              uint32_t cap, double *fixpoint_ms);

/* ------------------------------------------------------------------------
 * One witness path for (u, v) in box's relation (Sec. 3.2: a single path can
 * always be extracted).  Requires keep_rank if the RSM has box-labelled
 * transitions (a regular query needs no ranks).  The breadth-first search
 * over the product graph runs on the device, one launch per level; the
 * parent walk reads the parent entries back.  edges receives 3 * n_edges
 * uint32 values (src, label, dst) in path order; an empty path (u == v, box
 * nullable) has n_edges == 0.  Each nonterminal edge is expanded through
 * edges added in strictly earlier iterations, so the expansion terminates.
 * CFPQ_ERR_NOT_FOUND if (u, v) is not in the relation; CFPQ_ERR_BUFFER with
 * *n_edges set to the required count if cap_edges is too small;
 * CFPQ_ERR_LIMIT if the witness exceeds 2^26 edges.
 * ---------------------------------------------------------------------- */
cfpq_status cfpq_extract_path(cfpq_result res, uint32_t box, uint32_t u, uint32_t v,
                              uint32_t *edges, uint64_t cap_edges, uint64_t *n_edges);

/* ------------------------------------------------------------------------
 * All paths of bounded length (Sec. 3.2, paths extraction; Listing 2).  The
 * set of paths between two vertices can be infinite; this enumerates the
 * paths from u to v with at most max_edges edges whose words box derives,
 * each path once, in order of non-decreasing length, one length at a time
 * as cfpq_paths_next asks for them.  The empty path is included when
 * u == v and box derives the empty word.
 *
 * cfpq_paths_open: any result (ranks are not needed: membership of (u, v)
 * is read from the returned relation); the iterator shares the graph's host
 * edge lists and copies the RSM, so res may be destroyed afterwards.  If
 * (u, v) is not in box's relation (as returned, vertex masks included) the
 * iterator is empty.  Errors: CFPQ_ERR_INVALID (NULL arguments, box or
 * vertex out of range, max_edges above 4096).
 * cfpq_paths_next: the next path into edges (3 uint32 per edge: src, label,
 * dst).  CFPQ_ERR_NOT_FOUND when no path is left; CFPQ_ERR_BUFFER with
 * *n_edges set if cap_edges is too small (the path is kept for the next
 * call); CFPQ_ERR_LIMIT if the paths of one length exceed 2^24 edges.
 * Host computation: the RSM is taken as a grammar (a nonterminal per state
 * for the words leading from it to a final state), made free of epsilon and
 * unit rules, and expanded with every split pruned by memoised sets of
 * vertices reachable from (nonterminal, vertex) in exactly l edges.
 * ---------------------------------------------------------------------- */
typedef struct cfpq_paths_s *cfpq_paths;
cfpq_status cfpq_paths_open(cfpq_result res, uint32_t box, uint32_t u, uint32_t v, uint32_t max_edges,
                            cfpq_paths *out);
cfpq_status cfpq_paths_next(cfpq_paths it, uint32_t *edges, uint64_t cap_edges, uint64_t *n_edges);
void cfpq_paths_close(cfpq_paths it);

/* Per-kernel profile of a query run with opts.profile (levels and condensed
 * strategies).  Each kind is one kernel; every launch of it is bracketed by
 * HIP events of its own on the query stream.
 * launches: number of launches of that kernel; ms: their summed device time;
 * bytes: the bytes of the words the kernel's algorithm reads and writes:
 *   CFPQ_KERNEL_SEED: the Kronecker product with the new edges (the gather
 *     over seeds; no byte count);
 *   CFPQ_KERNEL_LEVEL: one frontier level of the incremental closure,
 *     8 * tile_words * (R_in + 3 * R_out), R_in the frontier rows read and
 *     R_out the target rows fed by them (read T, write T and the next
 *     frontier);
 *   CFPQ_KERNEL_WRITEBACK: 8 * (|F_N| + 3) per word of the rows of box N it
 *     processes (rows whose final-state closure rows changed in the
 *     iteration; from the second iteration on only the 64-word blocks where
 *     a final-state row gained bits or the A2^N row held bits);
 *   CFPQ_KERNEL_COND_LEVEL: one topological level of the component graph,
 *     8 bytes per word of component rows it writes (answer rows in full,
 *     other rows only in their non-empty chunks, a row cut into
 *     ceil(ceil(n/64) / 576) equal chunks) plus 8 bytes per word of
 *     predecessor rows it ORs in;
 *   CFPQ_KERNEL_COND_SCC: the component search and the condensation set-up
 *     (component in-degrees, links, level-0 roots), no byte count;
 *   CFPQ_KERNEL_NT_MFMA: matrix-core nonterminal products in closure levels;
 *     *bytes receives int8 operations, 2 per multiply-accumulate (65536 per
 *     v_mfma_i32_32x32x32_i8);
 *   CFPQ_KERNEL_NT_SPARSE: the sparse nonterminal products (seed and closure
 *     levels): 8 bytes per selector and source-activity word read, 4 per ELL
 *     count and entry read, 8 * tile_words per dense source row ORed and per
 *     product row written;
 *   CFPQ_KERNEL_ELL: the ELL lists the sparse products read (no byte count);
 *   CFPQ_KERNEL_NT_DENSE: the dense part of the nonterminal products (source
 *     rows with more than 32 bits in the tile), blocked through LDS: 8 bytes
 *     per selector word read, per source word staged, and 16 per product
 *     word updated.
 * CFPQ_ERR_INVALID if the query was not profiled. */
enum { CFPQ_KERNEL_SEED = 0, CFPQ_KERNEL_LEVEL = 1, CFPQ_KERNEL_WRITEBACK = 2, CFPQ_KERNEL_COND_LEVEL = 3,
       CFPQ_KERNEL_COND_SCC = 4, CFPQ_KERNEL_NT_MFMA = 5, CFPQ_KERNEL_NT_SPARSE = 6, CFPQ_KERNEL_ELL = 7,
       CFPQ_KERNEL_NT_DENSE = 8 };
cfpq_status cfpq_result_profile(cfpq_result res, uint32_t kind, uint64_t *launches, double *ms,
                                uint64_t *bytes);

void cfpq_result_destroy(cfpq_result res);

const char *cfpq_last_error(void);

/* Library version string. */
const char *cfpq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CFPQ_H */
