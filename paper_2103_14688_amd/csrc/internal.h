// Library-internal declarations shared by the host driver (api.hip) and the
// device kernels (kernels.hip).  Not part of the C ABI.
//
// Data layout on the device (HBM), for a query over a graph with n vertices
// and an RSM with nQ states and nB boxes:
//
//   The closure is kept "by columns of sources".  Row (q, v) of the state
//   array T is a bitset over source vertices u: bit u set iff the product
//   node (box_start(q), u) reaches (q, v) -- i.e. the box-start rows of the
//   closure C3 of Listing 1, transposed.  Box-start states also hold the
//   trivial bit u == v.  Words per row: P (padded), of which Pn = ceil(n/64)
//   carry vertices.
//
//     T   [nQ][n][P]   closure rows (monotone)
//     NT  [nB][n][P]   nonterminal matrices M2^N, transposed: row v = {u}
//     dNT [nB][n][P]   edges NT gained in the last write-back (A2 of Listing 1)
//     D,Dn[nQ][n][G]   frontier of the current closure level, restricted to
//                      one source tile of G words (bits over sources)
//     act[nQ][Pn]      bitset of frontier rows that are non-empty
//     tnz[nQ][Pn]      bitset of T rows that are non-empty
//
//   Graph label matrices are stored by columns: for vertex v and label l the
//   sorted predecessors gidx[goff[l*(n+1)+v] .. goff[l*(n+1)+v+1]).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cfpq {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr uint32_t kRingSlots = 1u << 16;   // device counter ring
constexpr uint32_t kSlotWords = 4;          // per slot: new bits, rows fed, rows gaining bits

struct InTrans {
    uint32_t src;   // source state
    uint32_t sym;   // < n_terms: graph label; else n_terms + box
};

// One closure launch: seeding from new edges (Kronecker product of the RSM
// with A2) or one frontier level of the incremental closure.
struct GatherArgs {
    uint32_t n, P, Pn, n_terms, nQ;
    uint32_t w0, gw, G;           // source tile [w0, w0+gw), frontier pitch G
    const uint32_t *goff, *gidx;
    const uint32_t *in_off;       // [nQ+1] incoming transitions per target state
    const InTrans *in_tr;
    uint64_t *T;
    const uint64_t *sel;          // nonterminal selectors: seed -> dNT, level -> NT
    const uint64_t *sel_act;      // seed: dnt_act bitset [nB][Pn]; level: null
    const uint64_t *src;          // rows OR-ed in: seed -> T, level -> D
    uint32_t src_pitch, src_off;
    const uint64_t *src_act;      // seed: tnz; level: act
    uint64_t *dn;                 // next frontier [nQ][n][G]
    uint64_t *actn;               // next frontier row bitset (pre-cleared)
    uint64_t *act_clear;          // bitset to clear for the launch after next (or null)
    uint32_t clear_words;
    uint64_t *tnz;
    unsigned long long *ctr;      // counter ring, kSlotWords per slot
    uint32_t slot_prev;           // kNoSlot: run unconditionally
    uint32_t slot_cur;            // counts of this launch
    uint32_t seed_terms;          // seed launch: terminal transitions take part
    const uint64_t *extra;        // seed: rows of the sparse nonterminal product [nQ][n][G] (or null:
    const uint64_t *extra_act;    //   nonterminal transitions OR whole rows), row bitset [nQ][Pn]
    const uint64_t *sel_sum;      // optional summary of the selector rows: bit w of row word w / 64
                                  // set iff selector word w may be non-zero, [rows][sum_pitch]
    uint32_t sum_pitch;
    // optional coarse activity of the source rows, [nQ][Pbs]: bit j % 64 of
    // word j / 64 set iff src_act word j may be non-zero, word Pbs - 1
    // non-zero iff the state may have an active row; actn_blk: the same for
    // the next frontier (cleared with actn); Pbs = sum_pitch + 1
    const uint64_t *src_blk;
    uint64_t *actn_blk;
    uint32_t Pbs;
    uint64_t *chg;                // optional: rows that gained bits in this iteration, [nQ][Pn]
    unsigned long long *bytes_ctr; // optional (profiling): bytes of the words the launch reads and writes
    // sparse product: source rows listed as dense (more than kEll bits) are
    // left to k_nt_dense; every target row with a selected source row is
    // still written and flagged (the dense product ORs into it afterwards)
    uint32_t dense_apart;
    // optional (seed): representative rows of the selector classes.  For a
    // target state f with exactly one box-labelled incoming transition (box
    // f_box[f], else kNoBox) and an active selector row (N, v), rep[N n + v]
    // is a row with the same selector contents; the product is computed for
    // representatives only, and (f, v) reads the row of (f, rep).  null = off
    const uint32_t *rep;
    const uint32_t *f_box;
    // optional: per row [nQ][n] a mask of the blocks of 2^blk_shift words of
    // T that gained bits in this iteration (bit b: words b 2^blk_shift ..)
    uint64_t *chgb;
    uint32_t blk_shift;
};
constexpr uint32_t kNoBox = 0xFFFFFFFFu;
// summary of the rows [nB][n][P] whose bit is set in act ([nB][Pn] bits;
// other rows' summaries are left as they are): bit w % 64 of summary word
// w / 64 set iff word w is non-zero
hipError_t launch_row_summary(const uint64_t *rows, uint32_t nB, uint32_t n, uint32_t P, uint32_t Pn,
                              const uint64_t *act, uint64_t *sum, uint32_t sum_pitch, hipStream_t s);

#ifndef CFPQ_ELL
#define CFPQ_ELL 32
#endif
constexpr uint32_t kEll = CFPQ_ELL;            // listed bits per source row in the sparse product (tuning)
constexpr uint32_t kEllDense = 0xFFFFFFFFu;    // row has more bits: OR it whole
constexpr uint32_t kEllBlocked = 0xFFFFFFFEu;  // row beyond a list, left to the LDS-blocked product
// (kEllDense rows are ORed whole by the sparse product itself: only where
// no dense product runs, the matrix-core and whole-row modes.  ORing rows
// of 33 to 1/8 of the tile's bits whole per target measured 2-4x slower
// than the blocked product on random dense grammars)
static_assert(kEll >= 2, "a dense row's list holds its 64-bit block mask");
// closure levels use the sparse product from this many words per row tile
// (narrower rows are ORed whole at no greater cost)
constexpr uint32_t kLevelSparseMinWords = 16;
// automatic source tiles of queries with box-labelled transitions: at most
// this many words (see run_levels; same generation n = 2e5: two tiles of
// 1563 words 760 ms, three of 1042 862 ms, one 794 ms; memory alias
// n = 1e5: one tile 10.71 s, two 10.47 s)
constexpr uint32_t kTileCapWords = 1600;
constexpr uint32_t kSparseMaxWords = 4096;     // LDS row accumulator limit (words per wavefront)

struct WritebackArgs {
    uint32_t n, P, Pn, nB;
    const uint32_t *fin_off, *fin; // final states per box
    const uint64_t *T;
    uint64_t *NT, *dNT, *dnt_act;  // dnt_act pre-cleared
    uint8_t *rank;                 // optional [nB][n][n]: rank[N][u][v] (source-major)
    uint32_t iter;
    unsigned long long *ctr;
    uint32_t slot_base;            // new edges of box N counted at slot_base + N
    const uint32_t *row_map;       // optional: T row of product node (f, v) is row_map[f*n+v]
    int fresh;                     // M2^N is known empty: write it without reading
    const uint8_t *row_nz;         // optional: per (T row, 512-word chunk) flag; 0 = the chunk is all zero
    const uint32_t *state_flags;   // optional (with multi): rows of single-member components of a
    const uint32_t *multi;         //   kAliasFinal state are already in NT; such rows are skipped
    const unsigned long long *skip_if[2];   // optional: the launch does nothing if either is nonzero
    // optional (levels strategy): only rows (N, v) with chg[f][v] set for a
    // final state f of N (its closure row gained bits in this iteration) or
    // with prev_act[N][v] set (their dNT row is not yet cleared) are visited;
    // every other row of NT and dNT is already what the write-back would leave
    const uint64_t *chg;
    const uint64_t *prev_act;
    unsigned long long *rows_ctr;  // optional (profiling): row words processed, per box [nB]
    // optional: summaries of the visited rows ([nB][n][sum_pitch], bit w % 64
    // of word w / 64 set iff word w is non-zero) of dNT and NT, written here
    // instead of by a separate pass over the rows
    uint64_t *dsum, *nsum;
    uint32_t sum_pitch;
    // optional: per row [nB][n] a 64-bit hash of its new edges (dNT row),
    // written for rows that gained edges (non-zero)
    uint64_t *dhash;
    // optional (levels strategy): chgb, the gathers' masks of the T blocks
    // that gained bits ([nQ][n], blocks of blk_words words), and dnb, per row
    // [nB][n] the blocks where dNT is non-zero (written here).  With chgb a
    // visited row is processed only in the blocks some final-state row
    // gained bits in or its dNT row held bits in: elsewhere NT cannot gain
    // and dNT, its summary and NT's summary are already what the write-back
    // would leave.  Without chgb rows are processed whole (dnb still written)
    const uint64_t *chgb;
    uint64_t *dnb;
    uint32_t blk_words;
};                                 // dNT / dnt_act may be null (no delta kept)

// kernels.hip
hipError_t launch_fill(uint64_t *p, uint64_t words, uint64_t value, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint64_t bytes, hipStream_t s);
// trivial bits of the box-start rows: (start, v) holds source bit v, for v in
// mask (null = every vertex)
hipError_t launch_seed_diag(uint64_t *T, uint64_t *tnz, uint32_t n, uint32_t P, uint32_t Pn,
                            const uint32_t *states, uint32_t n_states, const uint64_t *mask, hipStream_t s);
// vertex masks on one box's rows [n][P] (row v = sources): rows of targets
// outside dst lose every bit, the others keep the sources in src (either
// mask may be null)
hipError_t launch_mask_rows(uint64_t *rows, uint32_t n, uint32_t P, uint32_t Pn, const uint64_t *src,
                            const uint64_t *dst, hipStream_t s);
hipError_t launch_eps(uint64_t *NT, uint64_t *dNT, uint64_t *dnt_act, uint8_t *rank, uint32_t n,
                      uint32_t P, uint32_t Pn, const uint32_t *boxes, uint32_t nb, hipStream_t s);
hipError_t launch_gather(const GatherArgs &a, bool seed, uint32_t grid, hipStream_t s);
// ELL lists of the rows of the given states (act: skip rows whose activity
// bit is clear, may be null; ctr_prev: skip the launch when that count is 0)
hipError_t launch_ell_build(const uint64_t *rows, uint32_t pitch, uint32_t off, uint32_t gw, uint32_t n,
                            const uint32_t *states, uint32_t n_states, uint32_t *ell_cnt, uint32_t *ell_idx,
                            const uint64_t *act, uint32_t Pn, const unsigned long long *ctr_prev, hipStream_t s,
                            unsigned long long *bytes_ctr = nullptr);
hipError_t launch_nt_sparse(const GatherArgs &a, const uint32_t *ell_cnt, const uint32_t *ell_idx, uint64_t *extra,
                            uint64_t *extra_act, uint32_t grid, hipStream_t s);
// Dense part of the nonterminal product: the source rows the ELL build
// listed as dense (dns [nQ][Pn] bits, their coarse array dblk [nQ][Pbs]),
// blocked through LDS: a workgroup owns 128 target rows x 64 source words
// and ORs each staged block of 64 source rows into all of them.  Runs after
// k_nt_sparse (with dense_apart), ORing into the product rows it flagged.
struct DenseArgs {
    const uint64_t *dns, *dblk;
    const uint32_t *ell_idx;       // a dense row's list holds the 64-bit mask of its non-zero 64-word blocks
    const uint32_t *nt_dst;        // target states of box-labelled transitions
    uint32_t n_nt_dst;
    uint64_t *extra;               // product rows [nQ][n][G]
    const uint64_t *extra_act;     // [nQ][Pn], flagged by k_nt_sparse
};
hipError_t launch_nt_dense(const GatherArgs &a, const DenseArgs &d, hipStream_t s);
// ELL build also marks dense rows: dns bit and coarse dblk (both pre-cleared)
hipError_t launch_ell_build_dense(const uint64_t *rows, uint32_t pitch, uint32_t off, uint32_t gw, uint32_t n,
                                  const uint32_t *states, uint32_t n_states, uint32_t *ell_cnt, uint32_t *ell_idx,
                                  const uint64_t *act, uint32_t Pn, const unsigned long long *ctr_prev,
                                  uint64_t *dns, uint64_t *dblk, uint32_t Pbs, hipStream_t s,
                                  unsigned long long *bytes_ctr = nullptr);

// Dense nonterminal product of one transition (s, N, f) on the matrix cores.
struct MfmaArgs {
    uint32_t n, P, Pn, gw, G;
    const uint64_t *sel;          // selector rows of box N: [n][P], bits over x
    const uint64_t *src;          // source rows of state s (tile start), pitch src_pitch, bits over sources
    uint32_t src_pitch;
    const uint64_t *sact;         // live source rows of state s: [Pn]
    uint64_t *out;                // target state f rows: [n][G]
    uint64_t *out_act;            // target state f row bitset: [Pn]
    int first;                    // first transition into f this launch group: store, else OR
    const unsigned long long *ctr_prev;  // skip when the previous level added nothing (or null)
    unsigned long long *mfma_ctr; // optional: MFMA instructions issued
};
hipError_t launch_nt_mfma(const MfmaArgs &a, hipStream_t s);
hipError_t launch_writeback(const WritebackArgs &a, uint32_t grid, hipStream_t s);
// Seed deduplication: classes of equal dNT rows among the active ones (act
// [nB][Pn]), from the write-back's row hashes; keys/vals is an open-addressing
// table of mask + 1 >= 2 nB n slots (cleared here).  rep[N n + v] := a row of
// box N with the same contents (the least row index of its hash bucket when
// the rows compare equal word for word, else v itself).
hipError_t launch_dedup(uint32_t nB, uint32_t n, uint32_t P, uint32_t Pn, const uint64_t *act, const uint64_t *dhash,
                        const uint64_t *dNT, const uint64_t *dsum, uint32_t sum_pitch, unsigned long long *keys,
                        uint32_t *vals, uint64_t mask, uint32_t *rep, hipStream_t s);
hipError_t launch_popcount(const uint64_t *p, uint64_t rows, uint32_t pitch, uint32_t words,
                           unsigned long long *out, hipStream_t s);
hipError_t launch_hash(const uint64_t *NTb, uint32_t n, uint32_t P, unsigned long long *out,
                       hipStream_t s);
// dst[u][v-word] (row-major, pitch dst_pitch) from src[v][u-word] (pitch src_pitch)
hipError_t launch_transpose(const uint64_t *src, uint32_t src_pitch, uint64_t *dst,
                            uint32_t dst_pitch, uint32_t n, hipStream_t s);

// Implicit product graph of an RSM without box-labelled transitions.
struct ProdGraph {
    uint32_t n, nQ;
    const uint32_t *goff, *gidx;   // predecessors per label (columns)
    const uint32_t *soff, *sidx;   // successors per label (rows)
    const uint32_t *in_off, *out_off;
    const InTrans *in_tr;          // per target state: (source state, label)
    const InTrans *out_tr;         // per source state: (target state in .src, label)
    // the component search's transitions: those inside one strongly
    // connected component of the state graph (a cycle of the product graph
    // projects onto a cycle of states, so it uses no other), same layout
    const uint32_t *sin_off, *sout_off;
    const InTrans *sin_tr, *sout_tr;
    const uint64_t *src_mask;      // sources searched ([ceil(n/64)] bits), null = all
    // condensation links (written by k_cond_count, read by the level kernel;
    // null = not kept): per node up to kCondLinks components it is entered
    // from and stripe counters it retires, with counts (kCondLinks + 1 in
    // xin_cnt: more, walk the edges instead)
    uint32_t *xin_cnt, *xin, *xout_cnt, *xout;
    // trimming witnesses (null = none kept): per node, 1 + the live
    // predecessor and 1 + the live successor its last check found (0: none)
    uint32_t *trim_w;
};
constexpr uint32_t kCondLinks = 4;

// condense.hip
hipError_t launch_trim(const ProdGraph &g, uint8_t *alive, uint32_t *scc, const unsigned long long *prev,
                       unsigned long long *ctr, hipStream_t s);
hipError_t launch_pivot(const ProdGraph &g, const uint8_t *alive, unsigned long long *best, hipStream_t s);
// frontiers of the pivot searches: q[direction][parity] hold cap entries
// each (direction 0 forward, 1 backward); cnt[3 * direction + k] is a ring
// of three frontier sizes, zero before the first search launch
struct ReachQueues {
    uint32_t *q[2][2];
    unsigned long long *cnt;
    uint64_t cap;
};
// one level of forward/backward reachability from the pivot: expands the
// frontiers of launch `it` (0, 1, ... in order), marks in place and counts
// the nodes it claims into *ctr
hipError_t launch_reach(const ProdGraph &g, const uint8_t *alive, uint32_t *fw, uint32_t *bw, const ReachQueues &rq,
                        uint32_t it, unsigned long long *ctr, hipStream_t s);
// the pivot in *best (k_pivot's key; 0 = none) starts both searches as
// frontier 0
hipError_t launch_pivot_seed(const unsigned long long *best, uint32_t *fw, uint32_t *bw, const ReachQueues &rq,
                             hipStream_t s);
constexpr uint32_t kStripes = 16;           // in-degree counters per component
// per-state flags of the condensed strategy: bit 0 box start, bit 1 the only
// final state of its box (its single-member rows alias the answer), box id
// from bit 2 up
constexpr uint32_t kStartState = 1, kAliasFinal = 2, kFlagBoxShift = 2;
// counters of the condensed levels: kWave stripes of answer pairs per box,
// then (at kBytesSlot) kWave (words written, predecessor words requested) pairs
constexpr uint32_t kBytesSlot = 4096;
// open0/open1 (optional): the searches' next frontier sizes; nonzero means
// they are not complete and the launch does nothing
hipError_t launch_fwbw_assign(uint32_t N, uint8_t *alive, const uint32_t *fw, const uint32_t *bw,
                              const unsigned long long *best, uint32_t *scc, unsigned long long *ctr,
                              const unsigned long long *open0, const unsigned long long *open1, hipStream_t s);
hipError_t launch_color_init(uint32_t N, const uint8_t *alive, uint32_t *color, uint8_t *found, hipStream_t s);
hipError_t launch_color_prop(const ProdGraph &g, const uint8_t *alive, uint32_t *color,
                             const unsigned long long *prev, unsigned long long *ctr, hipStream_t s);
hipError_t launch_color_roots(uint32_t N, const uint8_t *alive, const uint32_t *color, uint8_t *found, uint32_t *scc,
                              hipStream_t s);
hipError_t launch_color_back(const ProdGraph &g, const uint8_t *alive, const uint32_t *color, uint8_t *found,
                             uint32_t *scc, const unsigned long long *prev, unsigned long long *ctr, hipStream_t s);
hipError_t launch_color_remove(uint32_t N, uint8_t *alive, const uint8_t *found, unsigned long long *ctr,
                               hipStream_t s);
// skip_if (optional, the condensation set-up kernels): the launch does
// nothing when *skip_if is nonzero (nodes still without a component)
hipError_t launch_cond_count(const ProdGraph &g, const uint32_t *scc, uint32_t *size, uint32_t *stripe,
                             const unsigned long long *skip_if, hipStream_t s);
hipError_t launch_cond_seed(uint32_t n, uint32_t P, uint32_t Pn, uint32_t nQ, const uint32_t *starts,
                            uint32_t n_starts, const uint32_t *scc, const uint32_t *multi, uint64_t *R, uint8_t *nz,
                            const uint64_t *mask, const unsigned long long *skip_if, hipStream_t s);
hipError_t launch_cond_roots(uint32_t N, const uint32_t *scc, const uint32_t *stripe, uint32_t *pending,
                             uint32_t *lev, unsigned long long *ctr, const unsigned long long *skip_if, hipStream_t s);
hipError_t launch_cond_level(const ProdGraph &g, uint32_t P, uint32_t Pn, const uint32_t *scc, const uint32_t *multi,
                             uint32_t *indeg, uint32_t *pending, uint32_t *lev, uint64_t *R, uint64_t *NT, uint8_t *nz,
                             const uint32_t *flags, uint32_t L, const unsigned long long *ctr_prev,
                             unsigned long long *ctr_next, unsigned long long *ctr_clear, unsigned long long *box_pairs,
                             unsigned long long *bytes_ctr, hipStream_t s);
hipError_t launch_cond_expand(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc, const uint8_t *nz, uint64_t *T,
                              hipStream_t s);
// A component row is cut into cond_chunks(Pn) equal chunks of at most
// kCondChunkWords words, each with its own non-empty flag: at most
// CFPQ_COND_LANE_WORDS words per lane of a wavefront (a compile-time tuning
// parameter, at most 16).  With the level kernel held to 128 VGPRs (four
// wavefronts per SIMD, CFPQ_COND_MIN_WAVES) 9 words measured fastest (three
// chunks at n = 10^5: 43.2 us per level launch, against 45.0 with 10, 45.1
// with 8 and 44.9 with 13 words uncapped, which takes 153 VGPRs and leaves
// room for three wavefronts per SIMD); 13 words under the cap spill.  Equal
// chunks avoid a short last chunk that costs a whole work item.
// The row phase moves CFPQ_COND_VEC words per lane access (1: 8-byte, 2:
// 16-byte loads and stores; with 2, chunks hold whole pairs of words, so a
// chunk starts 16-byte aligned, rows being 64-byte aligned).  A compile-time
// tuning parameter: 16-byte accesses (14 words per lane) measured slower,
// 65.5 against 54.5 us per level launch on the RPQ workload at n = 10^5.
#ifndef CFPQ_COND_VEC
#define CFPQ_COND_VEC 1
#endif
#ifndef CFPQ_COND_LANE_WORDS
#if CFPQ_COND_VEC == 2
#define CFPQ_COND_LANE_WORDS 14
#else
#define CFPQ_COND_LANE_WORDS 9
#endif
#endif
static_assert(CFPQ_COND_VEC == 1 || CFPQ_COND_VEC == 2, "8- or 16-byte row accesses");
static_assert(CFPQ_COND_LANE_WORDS % CFPQ_COND_VEC == 0, "whole vectors per lane");
constexpr uint32_t kCondChunkWords = CFPQ_COND_LANE_WORDS * 64;
static_assert(kCondChunkWords % CFPQ_COND_VEC == 0, "chunk capacity in whole vectors");
// equal widths, rounded up to whole vectors (never above the capacity); the
// count follows from the width, so the last chunk is never empty
// chunk width rounded to CFPQ_COND_CHUNK_ALIGN words (a multiple of
// CFPQ_COND_VEC dividing 64, so the rounded width stays within
// kCondChunkWords)
#ifndef CFPQ_COND_CHUNK_ALIGN
#define CFPQ_COND_CHUNK_ALIGN 16
#endif
static_assert(CFPQ_COND_CHUNK_ALIGN % CFPQ_COND_VEC == 0 && 64 % CFPQ_COND_CHUNK_ALIGN == 0, "chunk alignment");
__host__ __device__ inline uint32_t cond_chunk_words(uint32_t Pn) {
    if (Pn == 0) return kCondChunkWords;
    const uint32_t c = (Pn + kCondChunkWords - 1) / kCondChunkWords;
    const uint32_t w = (Pn + c - 1) / c;
    return (w + CFPQ_COND_CHUNK_ALIGN - 1) / CFPQ_COND_CHUNK_ALIGN * CFPQ_COND_CHUNK_ALIGN;
}
__host__ __device__ inline uint32_t cond_chunks(uint32_t Pn) {
    const uint32_t w = cond_chunk_words(Pn);
    return (Pn + w - 1) / w;
}

// Fused small-graph fixpoint: one workgroup runs a whole query.
#ifndef CFPQ_FUSED_LDS
#define CFPQ_FUSED_LDS 1
#endif
#ifndef CFPQ_FUSED_LDS_ODD
#define CFPQ_FUSED_LDS_ODD 1
#endif
struct FusedQuery {
    uint32_t n, P, Pn, n_terms, nQ, nB;
    const uint32_t *goff, *gidx;
    const uint32_t *in_off;
    const InTrans *in_tr;
    const uint32_t *starts;        // [nB] box start states
    const uint32_t *fin_off, *fin;
    const uint8_t *nullable;       // [nB]
    const uint8_t *box_used;       // [nB] box labels some transition
    uint64_t *T, *NT, *dNT, *D, *Dn;   // D/Dn: [nQ][n][P]
    uint64_t *act, *actn, *tnz, *dnt_act;
    uint8_t *rank;
    unsigned long long *stats;     // [0] iterations, [1] status, [2..] per-iteration deltas
    uint32_t max_iters, stats_cap;
    uint32_t lds_ok;               // the fixpoint may run in LDS (T is not kept)
};
// Words of a fused query's working set in LDS: T, D, Dn ([nQ][n] rows),
// M2^N and A2^N ([nB][n] rows), all at a pitch of `pitch` words, and the
// activity bitsets (act, actn, tnz: nQ rows, dnt_act: nB rows of Pn words).
__host__ __device__ inline uint64_t fused_lds_words(uint32_t n, uint32_t Pn, uint32_t pitch, uint32_t nQ,
                                                    uint32_t nB) {
    return (3ull * nQ + 2ull * nB) * n * pitch + (3ull * nQ + nB) * Pn;
}
// row pitch of a fused query's LDS working set: Pn, made odd (rows of
// consecutive threads then fall on different banks) where that still fits
__host__ __device__ inline uint32_t fused_lds_pitch(uint32_t n, uint32_t Pn, uint32_t nQ, uint32_t nB,
                                                    uint64_t lds_words) {
    const uint32_t odd = Pn | 1u;
    return (CFPQ_FUSED_LDS_ODD && fused_lds_words(n, Pn, odd, nQ, nB) <= lds_words) ? odd : Pn;
}
// lds_words: the launch's dynamic LDS in words (0: every query in global
// memory); a query whose working set fits runs there
hipError_t launch_fused(const FusedQuery *qs_dev, uint32_t n_queries, uint32_t *next_query, uint64_t lds_words,
                        hipStream_t s);
// dynamic LDS words a fused launch can take on the current device
uint64_t fused_lds_limit_words();

// One level of a breadth-first search over the product graph of a box (a
// frontier vector times the product's Boolean adjacency), recording parent
// pointers: the step of single-witness extraction (Sec. 3.2).  Terminal
// transitions follow graph edges; box-labelled transitions (M, x, y) are
// usable only where rank[M][x][y] < rk (pairs found in earlier iterations;
// no rank array: none usable).  Claims are exclusive (atomic on par), so
// every node enters one frontier once; a claimed (final state, v_target)
// node is reported in *hit.
struct WitnessBfs {
    uint32_t n, n_terms;
    const uint32_t *s_off;         // [nQ + 1] transitions by source state
    const InTrans *s_tr;           // .src = target state, .sym
    const uint32_t *final;         // [nQ] nonzero: final state
    const uint32_t *soff, *sidx;   // graph successors per label
    const uint8_t *rank;           // [nB][n][n] source-major, or null
    uint32_t rk;
    uint32_t v_target;
    const uint32_t *cur;           // frontier node ids (q * n + x)
    uint32_t ncur;
    uint32_t *next;                // next frontier; its size in ctr[0]
    uint32_t *par, *psym;          // per product node: parent node (kNoSlot = none), symbol
    unsigned int *ctr;             // [0] next size, [1] hit node (kNoSlot = none)
};
hipError_t launch_witness_bfs(const WitnessBfs &b, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s);

// Literal per-edge incremental closure (peredge.hip): the whole product
// graph's closure, one new edge at a time, in one workgroup.
struct PerEdgeQuery {
    uint32_t n, nQ, nB, n_terms, n_trans;
    uint32_t N, W, Wn;              // product nodes nQ * n, words per closure row, words per M row
    const uint32_t *soff, *sidx;    // graph successors per label
    const uint32_t *t_src, *t_sym, *t_dst;   // RSM transitions
    const uint32_t *starts, *fin_off, *fin;
    const uint8_t *nullable;
    uint64_t *C;                    // [N][W] closure rows (targets reachable by >= 1 edge)
    uint64_t *M, *dM;               // [nB][n][Wn] M2^N and its new edges, rows u (bits v)
    unsigned long long *stats;      // [0] iterations, [1] status, [2] rows grown, [3..] deltas
    uint32_t max_iters, stats_cap;
};
hipError_t launch_peredge(const PerEdgeQuery &q, hipStream_t s);

}  // namespace cfpq
