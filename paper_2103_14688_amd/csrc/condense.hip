// Closure of the product graph through its strongly connected components,
// for queries whose product has only terminal edges (regular path queries:
// one productive iteration, Sec. 3.1.2).
//
// The rows of all product nodes in one strongly connected component receive
// the same source bitset, so the closure is computed once per component, in
// topological order of the condensation:
//
//   R[c] = {u : (q_N^0, u) lies in c}  OR  OR_{c' -> c} R[c']
//
// Components are found on the device: iterated trimming (nodes without a
// live predecessor or successor are components of their own), forward and
// backward reachability from a high-degree pivot (its component is the
// intersection), then colouring (max-id propagation along edges; a root's
// component is what reaches the root inside its colour) for the rest.  The
// product graph is implicit: node p = q*n + v, edges (s, x) -> (f, y) for
// every transition (s, t, f) and graph edge (x, t, y).
//
// R[c] is stored in row c of T (c is the component's representative node),
// so no extra bitset memory is needed.
#include "internal.h"

#include <atomic>

namespace cfpq {

namespace {

constexpr int kCondChunks = CFPQ_COND_LANE_WORDS;   // words per lane of a chunk
constexpr uint32_t kCondNodes = 64;   // consecutive nodes per work item (ballot-selected)
static_assert(kCondChunks * kWave == kCondChunkWords, "chunk flags cover kCondChunks wavefront-widths");

__device__ __forceinline__ bool mask_bit(const uint64_t *bits, uint32_t i) { return (bits[i >> 6] >> (i & 63)) & 1ull; }

__device__ __forceinline__ unsigned long long wsum(unsigned long long x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// fn(pred) returns false to stop the walk
template <class F>
__device__ __forceinline__ void for_preds(const ProdGraph &g, uint32_t p, F &&fn) {
    const uint32_t q = p / g.n, v = p - q * g.n;
    for (uint32_t t = g.in_off[q]; t < g.in_off[q + 1]; ++t) {
        const InTrans tr = g.in_tr[t];
        const uint32_t *o = g.goff + (uint64_t)tr.sym * (g.n + 1) + v;
        const uint32_t base = tr.src * g.n;
        for (uint32_t e = o[0]; e < o[1]; ++e)
            if (!fn(base + g.gidx[e])) return;
    }
}

// Does some predecessor (successor) x of p pass test(x)?  Four edges per
// step: their index, flag and mark loads are independent, so they are in
// flight together instead of one edge's chain after another's.
template <bool SUCC, class F>
__device__ __forceinline__ bool any_adj(const ProdGraph &g, uint32_t p, F &&test) {
    const uint32_t q = p / g.n, v = p - q * g.n;
    const uint32_t tb = SUCC ? g.out_off[q] : g.in_off[q], te = SUCC ? g.out_off[q + 1] : g.in_off[q + 1];
    for (uint32_t t = tb; t < te; ++t) {
        const InTrans tr = SUCC ? g.out_tr[t] : g.in_tr[t];
        const uint32_t *o = (SUCC ? g.soff : g.goff) + (uint64_t)tr.sym * (g.n + 1) + v;
        const uint32_t *idx = SUCC ? g.sidx : g.gidx;
        const uint32_t b = o[0], e = o[1], base = tr.src * g.n;
        uint32_t i = b;
        for (; i + 4 <= e; i += 4) {
            const uint32_t x0 = base + idx[i], x1 = base + idx[i + 1], x2 = base + idx[i + 2], x3 = base + idx[i + 3];
            const bool h0 = test(x0), h1 = test(x1), h2 = test(x2), h3 = test(x3);
            if (h0 | h1 | h2 | h3) return true;
        }
        for (; i < e; ++i)
            if (test(base + idx[i])) return true;
    }
    return false;
}

// The first predecessor (successor) x of p that passes test(x), or
// kNoNode; the same four-edges-per-step walk as any_adj.
constexpr uint32_t kNoNode = 0xFFFFFFFFu;
template <bool SUCC, class F>
__device__ __forceinline__ uint32_t first_adj(const ProdGraph &g, uint32_t p, F &&test) {
    const uint32_t q = p / g.n, v = p - q * g.n;
    const uint32_t tb = SUCC ? g.out_off[q] : g.in_off[q], te = SUCC ? g.out_off[q + 1] : g.in_off[q + 1];
    for (uint32_t t = tb; t < te; ++t) {
        const InTrans tr = SUCC ? g.out_tr[t] : g.in_tr[t];
        const uint32_t *o = (SUCC ? g.soff : g.goff) + (uint64_t)tr.sym * (g.n + 1) + v;
        const uint32_t *idx = SUCC ? g.sidx : g.gidx;
        const uint32_t b = o[0], e = o[1], base = tr.src * g.n;
        uint32_t i = b;
        for (; i + 4 <= e; i += 4) {
            const uint32_t x0 = base + idx[i], x1 = base + idx[i + 1], x2 = base + idx[i + 2], x3 = base + idx[i + 3];
            const bool h0 = test(x0), h1 = test(x1), h2 = test(x2), h3 = test(x3);
            if (h0) return x0;
            if (h1) return x1;
            if (h2) return x2;
            if (h3) return x3;
        }
        for (; i < e; ++i)
            if (test(base + idx[i])) return base + idx[i];
    }
    return kNoNode;
}

template <class F>
__device__ __forceinline__ void for_succs(const ProdGraph &g, uint32_t p, F &&fn) {
    const uint32_t q = p / g.n, v = p - q * g.n;
    for (uint32_t t = g.out_off[q]; t < g.out_off[q + 1]; ++t) {
        const InTrans tr = g.out_tr[t];   // src field: destination state
        const uint32_t *o = g.soff + (uint64_t)tr.sym * (g.n + 1) + v;
        const uint32_t base = tr.src * g.n;
        for (uint32_t e = o[0]; e < o[1]; ++e)
            if (!fn(base + g.sidx[e])) return;
    }
}

// g with the component search's transitions (those inside one component
// of the state graph) in place of all of them
__device__ __forceinline__ ProdGraph search_view(const ProdGraph &g) {
    ProdGraph s = g;
    s.in_off = g.sin_off;
    s.in_tr = g.sin_tr;
    s.out_off = g.sout_off;
    s.out_tr = g.sout_tr;
    return s;
}

#define NODE_LOOP(N)                                                                        \
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < (N); p += gridDim.x * blockDim.x)

// *ctr += the sum of c over the workgroup (every thread of a kBlock-thread
// workgroup calls it): one atomic per workgroup, since atomics on one
// address from thousands of wavefronts serialise
__device__ __forceinline__ void count_add(unsigned long long *ctr, unsigned long long c) {
    __shared__ unsigned long long s_part[kBlock / kWave];
    c = wsum(c);
    if (__lane_id() == 0) s_part[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
#pragma unroll
        for (int k = 0; k < kBlock / kWave; ++k) t += s_part[k];
        if (t) atomicAdd(ctr, t);
    }
}

__device__ __forceinline__ uint32_t shfl_u32(uint32_t x, int src) { return (uint32_t)__shfl((int)x, src, kWave); }
__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src) {
    return (uint64_t)shfl_u32((uint32_t)x, src) | ((uint64_t)shfl_u32((uint32_t)(x >> 32), src) << 32);
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = __lane_id();
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, off, kWave);
        if (lane >= off) x += y;
    }
    return x;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t y = (uint32_t)__shfl_xor((int)x, off, kWave);
        x = y > x ? y : x;
    }
    return x;
}

// ----------------------------------------------------------------------------
// component search
// ----------------------------------------------------------------------------
__global__ void k_trim(ProdGraph g_all, uint8_t *alive, uint32_t *scc, const unsigned long long *prev,
                       unsigned long long *ctr) {
    if (prev && *prev == 0) return;  // the previous sweep removed nothing
    // a node without a live predecessor or successor over the search's
    // transitions lies on no cycle of live nodes
    const ProdGraph g = search_view(g_all);
    const uint32_t N = g.nQ * g.n;
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (!alive[p]) continue;
        auto live_other = [&](uint32_t x) { return x != p && alive[x] != 0; };
        bool in, out;
        if (g.trim_w) {
            // the live neighbours the last check found, if still live (a
            // witness is a neighbour other than p); else walk the edges
            const uint2 w = reinterpret_cast<const uint2 *>(g.trim_w)[p];
            in = w.x && alive[w.x - 1];
            out = w.y && alive[w.y - 1];
            if (!in) {
                const uint32_t x = first_adj<false>(g, p, live_other);
                in = x != kNoNode;
                if (in) g.trim_w[2 * (uint64_t)p] = x + 1;
            }
            if (in && !out) {
                const uint32_t x = first_adj<true>(g, p, live_other);
                out = x != kNoNode;
                if (out) g.trim_w[2 * (uint64_t)p + 1] = x + 1;
            }
        } else {
            in = any_adj<false>(g, p, live_other);
            out = in && any_adj<true>(g, p, live_other);
        }
        if (!in || !out) {
            alive[p] = 0;
            scc[p] = p;
            ++c;
        }
    }
    count_add(ctr, c);
}

__global__ void k_pivot(ProdGraph g_all, const uint8_t *alive, unsigned long long *best) {
    const ProdGraph g = search_view(g_all);   // degrees over the search's transitions
    const uint32_t N = g.nQ * g.n;
    unsigned long long mine = 0;
    NODE_LOOP(N) {
        if (!alive[p]) continue;
        // degrees from the offsets: no edge is read
        uint64_t din = 0, dout = 0;
        const uint32_t q = p / g.n, v = p - q * g.n;
        for (uint32_t t = g.in_off[q]; t < g.in_off[q + 1]; ++t) {
            const uint32_t *o = g.goff + (uint64_t)g.in_tr[t].sym * (g.n + 1) + v;
            din += o[1] - o[0];
        }
        for (uint32_t t = g.out_off[q]; t < g.out_off[q + 1]; ++t) {
            const uint32_t *o = g.soff + (uint64_t)g.out_tr[t].sym * (g.n + 1) + v;
            dout += o[1] - o[0];
        }
        uint64_t score = (din + 1) * (dout + 1);
        if (score > 0xFFFFFFFFull) score = 0xFFFFFFFFull;
        const unsigned long long key = (score << 32) | p;
        if (key > mine) mine = key;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(mine, off, kWave);
        mine = o > mine ? o : mine;
    }
    // one atomic per workgroup
    __shared__ unsigned long long s_best[kBlock / kWave];
    if (__lane_id() == 0) s_best[threadIdx.x / kWave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / kWave; ++k) mine = s_best[k] > mine ? s_best[k] : mine;
        if (mine) atomicMax(best, mine);
    }
}

constexpr uint32_t kReachStage = 256;   // claimed nodes staged per wavefront before an append
#ifndef CFPQ_REACH_PAIR
#define CFPQ_REACH_PAIR 2
#endif
static_assert(CFPQ_REACH_PAIR == 1 || CFPQ_REACH_PAIR == 2, "one or two transitions per expansion step");
static_assert(kReachStage >= kWave, "a step's claims fit the staging buffer");

// Forward and backward reachability from the pivot inside the live nodes,
// level by level: launch it expands frontier it of both directions (forward
// along successors, backward along predecessors), 64 edges per step per
// wavefront whatever the frontier nodes' degrees.  A live, unmarked neighbour
// is claimed with an atomic exchange of its mark and appended to frontier
// it + 1.  A node is claimed at most once per direction, so a frontier never
// holds more than N entries.  Frontier sizes live in a ring of three counters
// per direction: launch it reads slot it % 3, appends to slot (it + 1) % 3 and
// clears slot (it + 2) % 3, which launch it - 1 read and launch it + 1 fills.
__global__ __launch_bounds__(kBlock) void k_reach(ProdGraph g, const uint8_t *alive, uint32_t *fw, uint32_t *bw,
                                                  ReachQueues rq, uint32_t it, unsigned long long *ctr) {
    __shared__ uint32_t s_scan[kBlock / kWave][kWave];
    __shared__ uint32_t s_out[kBlock / kWave][kReachStage];   // claimed nodes, appended in one go
    const uint32_t r0 = it % 3, r1 = (it + 1) % 3, r2 = (it + 2) % 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rq.cnt[r2] = 0;
        rq.cnt[3 + r2] = 0;
    }
    const uint64_t nf = rq.cnt[r0], nb = rq.cnt[3 + r0];
    if (nf + nb == 0) return;  // both searches are complete
    const int lane = __lane_id();
    const uint32_t wib = threadIdx.x / kWave;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t itf = (nf + kWave - 1) / kWave, items = itf + (nb + kWave - 1) / kWave;
    const uint64_t below = (1ull << lane) - 1ull;
    unsigned long long claimed = 0;
    for (uint64_t w = wave; w < items; w += nwaves) {
        const bool fwd = w < itf;   // wave-uniform
        const uint64_t base = (fwd ? w : w - itf) * kWave;
        const uint64_t cnt = fwd ? nf : nb;
        const uint32_t d = fwd ? 0u : 1u;
        const uint32_t *cur = rq.q[d][it & 1];
        uint32_t *nxt = rq.q[d][(it + 1) & 1];
        uint32_t *mark = fwd ? fw : bw;
        unsigned long long *tail = rq.cnt + 3 * d + r1;
        const uint32_t *idx = fwd ? g.sidx : g.gidx;
        uint32_t v = 0, tb = 0, te = 0;
        if (base + lane < cnt) {
            const uint32_t y = cur[base + lane];
            const uint32_t q = y / g.n;
            v = y - q * g.n;
            tb = fwd ? g.sout_off[q] : g.sin_off[q];
            te = fwd ? g.sout_off[q + 1] : g.sin_off[q + 1];
        }
        // claimed nodes gather in s_out and go to the next frontier with one
        // atomic on its size per kReachStage - kWave of them
        uint32_t staged = 0;
        auto flush = [&]() {
            unsigned long long at = 0;
            if (lane == 0) at = atomicAdd(tail, (unsigned long long)staged);
            at = shfl_u64(at, 0);
            __builtin_amdgcn_wave_barrier();
            for (uint32_t i = (uint32_t)lane; i < staged; i += kWave)
                if (at + i < rq.cap) nxt[at + i] = s_out[wib][i];
            __builtin_amdgcn_wave_barrier();
            claimed += lane == 0 ? staged : 0u;
            staged = 0;
        };
        // CFPQ_REACH_PAIR transitions per step (1 or 2): their edge ranges go
        // through one scan and one expansion, so the edges of both are in
        // flight together
        constexpr uint32_t kTP = CFPQ_REACH_PAIR;
        const uint32_t ntr = wave_max_u32(te - tb);
        for (uint32_t k = 0; k < ntr; k += kTP) {
            uint32_t b[kTP], len[kTP], sb[kTP];
            uint32_t cnt_all = 0;
#pragma unroll
            for (uint32_t h = 0; h < kTP; ++h) {
                b[h] = 0;
                len[h] = 0;
                sb[h] = 0;
                if (tb + k + h < te) {
                    // in_tr: (source state, label); out_tr: (target state, label)
                    const InTrans tr = fwd ? g.sout_tr[tb + k + h] : g.sin_tr[tb + k + h];
                    const uint32_t *o = (fwd ? g.soff : g.goff) + (uint64_t)tr.sym * (g.n + 1) + v;
                    b[h] = o[0];
                    len[h] = o[1] - o[0];
                    sb[h] = tr.src * g.n;
                }
                cnt_all += len[h];
            }
            const uint32_t incl = wave_incl_scan(cnt_all);
            const uint32_t total = shfl_u32(incl, kWave - 1);
            if (total == 0) continue;
            s_scan[wib][lane] = incl;
            __builtin_amdgcn_wave_barrier();
            for (uint32_t f0 = 0; f0 < total; f0 += kWave) {
                const uint32_t f = f0 + (uint32_t)lane;
                uint32_t lo = 0, hi = kWave - 1;   // owner: first lane whose inclusive count exceeds f
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_scan[wib][mid] > f) hi = mid;
                    else lo = mid + 1;
                }
                const uint32_t startj = lo ? s_scan[wib][lo - 1] : 0u;
                uint32_t off = f - startj, bj = shfl_u32(b[0], (int)lo), sbj = shfl_u32(sb[0], (int)lo);
                if constexpr (kTP == 2) {
                    // past the owner's first range: its second
                    const uint32_t l0 = shfl_u32(len[0], (int)lo), b1 = shfl_u32(b[1], (int)lo),
                                   sb1 = shfl_u32(sb[1], (int)lo);
                    if (off >= l0) {
                        off -= l0;
                        bj = b1;
                        sbj = sb1;
                    }
                }
                uint32_t x = 0;
                bool got = false;
                if (f < total) {
                    x = sbj + idx[bj + off];
                    got = alive[x] && !mark[x] && atomicExch(&mark[x], 1u) == 0u;
                }
                const uint64_t m = __ballot(got);
                if (m) {
                    if (staged + kWave > kReachStage) flush();
                    if (got) s_out[wib][staged + (uint32_t)__popcll(m & below)] = x;
                    staged += (uint32_t)__popcll(m);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (staged) flush();
    }
    count_add(ctr, claimed);
}

// the pivot (from k_pivot's best key) starts both searches: it is marked and
// is frontier 0 of each direction (counter slot 0)
__global__ void k_pivot_seed(const unsigned long long *best, uint32_t *fw, uint32_t *bw, ReachQueues rq) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const unsigned long long b = *best;
    if (!b) return;
    const uint32_t p = (uint32_t)(b & 0xFFFFFFFFull);
    fw[p] = 1;
    bw[p] = 1;
    rq.q[0][0][0] = p;
    rq.q[1][0][0] = p;
    rq.cnt[0] = 1;
    rq.cnt[3] = 1;
}

__global__ void k_fwbw_assign(uint32_t N, uint8_t *alive, const uint32_t *fw, const uint32_t *bw,
                              const unsigned long long *best, uint32_t *scc, unsigned long long *ctr,
                              const unsigned long long *open0, const unsigned long long *open1) {
    if (open0 && (*open0 | *open1)) return;  // a search is not complete
    const unsigned long long b = *best;
    if (!b) return;
    const uint32_t pivot = (uint32_t)(b & 0xFFFFFFFFull);
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (alive[p] && fw[p] && bw[p]) {
            scc[p] = pivot;
            alive[p] = 0;
            ++c;
        }
    }
    count_add(ctr, c);
}

__global__ void k_color_init(uint32_t N, const uint8_t *alive, uint32_t *color, uint8_t *found) {
    NODE_LOOP(N) {
        color[p] = alive[p] ? p : 0u;
        found[p] = 0;
    }
}

__global__ void k_color_prop(ProdGraph g, const uint8_t *alive, uint32_t *color, const unsigned long long *prev,
                             unsigned long long *ctr) {
    if (prev && *prev == 0) return;
    const uint32_t N = g.nQ * g.n;
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (!alive[p]) continue;
        uint32_t m = color[p];
        const uint32_t old = m;
        for_preds(g, p, [&](uint32_t x) {
            if (alive[x]) {
                const uint32_t cx = color[x];
                if (cx > m) m = cx;
            }
            return true;
        });
        if (m > old) {
            color[p] = m;
            ++c;
        }
    }
    count_add(ctr, c);
}

__global__ void k_color_roots(uint32_t N, const uint8_t *alive, const uint32_t *color, uint8_t *found,
                              uint32_t *scc) {
    NODE_LOOP(N) {
        if (alive[p] && color[p] == p) {
            found[p] = 1;
            scc[p] = p;
        }
    }
}

__global__ void k_color_back(ProdGraph g, const uint8_t *alive, const uint32_t *color, uint8_t *found,
                             uint32_t *scc, const unsigned long long *prev, unsigned long long *ctr) {
    if (prev && *prev == 0) return;
    const uint32_t N = g.nQ * g.n;
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (!alive[p] || found[p]) continue;
        const uint32_t cp = color[p];
        if (any_adj<true>(g, p, [&](uint32_t x) { return alive[x] && found[x] && color[x] == cp; })) {
            found[p] = 1;
            scc[p] = cp;
            ++c;
        }
    }
    count_add(ctr, c);
}

__global__ void k_color_remove(uint32_t N, uint8_t *alive, const uint8_t *found, unsigned long long *ctr) {
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (alive[p]) {
            if (found[p]) alive[p] = 0;
            else ++c;
        }
    }
    count_add(ctr, c);
}

// ----------------------------------------------------------------------------
// condensation in topological order
// ----------------------------------------------------------------------------
// size[c] := 1 if component c has more than one member.  The edges entering c
// from other components are counted in kStripes counters, stripe chosen by
// the member node they enter, so that the many edges into one large
// component do not all meet on one address: stripe[c*kStripes + y % kStripes]
// counts edges x -> y with y in c and x outside it (one atomic per member
// node).  pending[c] := number of non-zero stripes (filled by k_cond_roots).
__global__ void k_cond_count(ProdGraph g, const uint32_t *scc, uint32_t *size, uint32_t *stripe,
                             const unsigned long long *skip_if) {
    if (skip_if && *skip_if) return;
    const uint32_t N = g.nQ * g.n;
    NODE_LOOP(N) {
        const uint32_t c = scc[p];
        if (c != p) size[c] = 1;  // a second member: the component is not a singleton
        // in-edges from other components, four per step (independent loads)
        uint32_t k = 0;
        const uint32_t q = p / g.n, v = p - q * g.n;
        // links: the distinct components p is entered from, and for every
        // entering edge x -> p the stripe it retires in x's list
        uint32_t lst[kCondLinks];
        uint32_t nl = 0;
        const uint32_t si = c * kStripes + p % kStripes;   // fits: N * kStripes < 2^32 when links are kept
        auto link = [&](uint32_t x, uint32_t cx) {
            if (!g.xin_cnt || cx == c) return;
            bool seen = false;
            for (uint32_t r = 0; r < nl && r < kCondLinks; ++r) seen |= lst[r] == cx;
            if (!seen) {
                if (nl < kCondLinks) lst[nl] = cx;
                ++nl;
            }
            const uint32_t slot = atomicAdd(&g.xout_cnt[x], 1u);
            if (slot < kCondLinks) g.xout[(uint64_t)x * kCondLinks + slot] = si;
        };
        for (uint32_t t = g.in_off[q]; t < g.in_off[q + 1]; ++t) {
            const InTrans tr = g.in_tr[t];
            const uint32_t *o = g.goff + (uint64_t)tr.sym * (g.n + 1) + v;
            const uint32_t b = o[0], e = o[1], base = tr.src * g.n;
            uint32_t i = b;
            for (; i + 4 <= e; i += 4) {
                const uint32_t x0 = base + g.gidx[i], x1 = base + g.gidx[i + 1], x2 = base + g.gidx[i + 2],
                               x3 = base + g.gidx[i + 3];
                const uint32_t c0 = scc[x0], c1 = scc[x1], c2 = scc[x2], c3 = scc[x3];
                k += (c0 != c) + (c1 != c) + (c2 != c) + (c3 != c);
                link(x0, c0);
                link(x1, c1);
                link(x2, c2);
                link(x3, c3);
            }
            for (; i < e; ++i) {
                const uint32_t x = base + g.gidx[i], cx = scc[x];
                k += cx != c;
                link(x, cx);
            }
        }
        if (k) atomicAdd(&stripe[(uint64_t)c * kStripes + p % kStripes], k);
        if (g.xin_cnt) {
            g.xin_cnt[p] = nl <= kCondLinks ? nl : kCondLinks + 1;
            for (uint32_t r = 0; r < nl && r < kCondLinks; ++r) g.xin[(uint64_t)p * kCondLinks + r] = lst[r];
        }
    }
}

// rows of components with several members are accumulated with atomics:
// clear them (one wavefront per representative)
__global__ __launch_bounds__(kBlock) void k_cond_zero_multi(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                                            const uint32_t *multi, uint64_t *R,
                                                            const unsigned long long *skip_if) {
    if (skip_if && *skip_if) return;
    // a lane per node finds the representatives (few), then the wavefront
    // clears their rows one after another
    const int lane = __lane_id();
    for (uint64_t p0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - (uint64_t)lane; p0 < N;
         p0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = p0 + (uint64_t)lane;
        uint64_t todo = __ballot(p < N && scc[p] == p && multi[p] != 0);
        while (todo) {
            const int j = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            uint64_t *row = R + (p0 + (uint64_t)j) * P;
            for (uint32_t w = lane; w < Pn; w += kWave) row[w] = 0;
        }
    }
}

// sources: (start, u) holds source bit u; only for several-member components
// (a single-member component's row is written whole, seed included, when its
// topological level is processed)
__global__ void k_cond_seed(uint32_t n, uint32_t P, const uint32_t *starts, uint32_t n_starts,
                            const uint32_t *scc, const uint32_t *multi, uint64_t *R, uint8_t *nz, uint32_t nch,
                            uint32_t cwds, const uint64_t *mask, const unsigned long long *skip_if) {
    if (skip_if && *skip_if) return;
    const int lane = __lane_id();
    const uint64_t total = (uint64_t)n_starts * n;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - (uint64_t)lane; i0 < total;
         i0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = i0 + (uint64_t)lane;
        uint32_t c = 0, u = 0;
        bool on = false;
        if (i < total) {
            const uint32_t s = starts[i / n];
            u = (uint32_t)(i % n);
            if (!mask || mask_bit(mask, u)) {
                c = scc[s * n + u];
                on = multi[c] != 0;
            }
        }
        const uint64_t act = __ballot(on);
        if (!act) continue;
        // the lanes that hit the first active lane's word (usually all of
        // them: the giant component's row) combine into one atomic
        const int l0 = __ffsll((unsigned long long)act) - 1;
        const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)c, l0);
        const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)(u >> 6), l0);
        const bool same = on && c == c0 && (u >> 6) == w0;
        uint64_t bits = same ? 1ull << (u & 63) : 0ull;
        for (int off = 32; off > 0; off >>= 1) bits |= shfl_u64(bits, lane ^ off);
        if (lane == l0) {
            atomicOr((unsigned long long *)&R[(uint64_t)c0 * P + w0], bits);
            nz[(uint64_t)c0 * nch + w0 / cwds] = 1;
        }
        if (on && !same) {
            atomicOr((unsigned long long *)&R[(uint64_t)c * P + (u >> 6)], 1ull << (u & 63));
            nz[(uint64_t)c * nch + (u >> 6) / cwds] = 1;
        }
    }
}

__global__ void k_cond_roots(uint32_t N, const uint32_t *scc, const uint32_t *stripe, uint32_t *pending,
                             uint32_t *lev, unsigned long long *ctr, const unsigned long long *skip_if) {
    if (skip_if && *skip_if) return;
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (scc[p] != p) continue;
        static_assert(kStripes % 4 == 0, "stripes read four at a time");
        const uint4 *st = reinterpret_cast<const uint4 *>(stripe + (uint64_t)p * kStripes);
        uint32_t nz = 0;
#pragma unroll
        for (uint32_t k = 0; k < kStripes / 4; ++k) {
            const uint4 w = st[k];
            nz += (w.x != 0) + (w.y != 0) + (w.z != 0) + (w.w != 0);
        }
        pending[p] = nz;
        if (nz == 0) {
            lev[p] = 0;
            ++c;
        } else {
            lev[p] = 0xFFFFFFFFu;
        }
    }
    count_add(ctr, c);
}

// Row of component c: single-member components of a state flagged
// kAliasFinal (the only final state of its box) keep their row in the answer
// matrix M2^N itself (row v of box N), all other components in R.
__device__ __forceinline__ uint64_t *comp_row(uint32_t c, uint32_t n, uint32_t P, const uint32_t *flags,
                                              const uint32_t *multi, uint64_t *R, uint64_t *NT) {
    const uint32_t f = flags[c / n];
    if ((f & kAliasFinal) && multi[c] == 0)
        return NT + ((uint64_t)(f >> kFlagBoxShift) * n + (c % n)) * P;
    return R + (uint64_t)c * P;
}

// predecessor rows listed per node; more take the whole-wavefront path (a
// compile-time tuning parameter: 2 and 4 measured slower, 12 and 16 even)
#ifndef CFPQ_COND_PRED_CAP
#define CFPQ_COND_PRED_CAP 8
#endif
constexpr uint32_t kCondPredCap = CFPQ_COND_PRED_CAP;
// lanes per node when OR-ing rows (kWave / kCondGroupLanes nodes at a time);
// a compile-time tuning parameter
// nodes per step of the row phase with a whole wavefront per node (their
// row loads in flight together); 0 selects the lane-group path instead.
// Compile-time tuning parameters: with 13-word lanes one node per step
// measured fastest (two cost the registers of a second accumulator; with
// 8-word lanes two were fastest), ahead of lane groups of 16 or 32 lanes
#ifndef CFPQ_COND_PAIR
#define CFPQ_COND_PAIR 1
#endif
#ifndef CFPQ_COND_GROUP_LANES
#define CFPQ_COND_GROUP_LANES 64
#endif
constexpr int kCondGroupLanes = CFPQ_COND_GROUP_LANES;
static_assert(kWave % kCondGroupLanes == 0 && kCondGroupLanes >= 16, "whole groups of at least 16 lanes");
constexpr int kCondGroupWords = (int)kCondChunkWords / kCondGroupLanes;
// words per lane and pass of the OR loop (register budget)
constexpr int kCondPassWords = kCondGroupWords < 16 ? kCondGroupWords : 16;
constexpr int kCondPasses = kCondGroupWords / kCondPassWords;
static_assert(kCondPasses * kCondPassWords == kCondGroupWords, "whole passes per chunk");
static_assert(CFPQ_COND_PAIR == 0 || kCondPasses == 1, "the paired row phase takes a chunk in one pass");
static_assert(kCondNodes == (uint32_t)kWave, "one node per lane in the edge-parallel phases");

// a single-member component's row word: written once, read by its
// successors in later launches (CFPQ_COND_NT = 1: streaming stores)
#ifndef CFPQ_COND_NT
#define CFPQ_COND_NT 1
#endif
__device__ __forceinline__ void store_row_word(uint64_t *dst, uint64_t x) {
#if CFPQ_COND_NT
    __builtin_nontemporal_store(x, dst);
#else
    *dst = x;
#endif
}

// Row-phase word layout: lane l's kk-th word of a chunk is word kk * 64 + l
// with 8-byte accesses, and words 2 (kk/2 * 64 + l) + {0, 1} (one 16-byte
// access per pair) with CFPQ_COND_VEC = 2.
constexpr int kCondVec = CFPQ_COND_VEC;
typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t cond_word(int kk, int lane) {
    return kCondVec == 1 ? (uint32_t)(kk * kWave + lane) : (uint32_t)(2 * ((kk >> 1) * kWave + lane));
}
// words w .. w + kCondVec - 1 of a chunk of cw words (zero past its end)
__device__ __forceinline__ void load_words(const uint64_t *src, uint32_t w, uint32_t cw, uint64_t *x) {
    if constexpr (kCondVec == 2) {
        if (w + 1 < cw) {
            const u64x2_t v = *reinterpret_cast<const u64x2_t *>(src + w);
            x[0] = v.x;
            x[1] = v.y;
        } else {
            x[0] = w < cw ? src[w] : 0ull;
            x[1] = 0;
        }
    } else {
        x[0] = w < cw ? src[w] : 0ull;
    }
}
__device__ __forceinline__ void store_words(uint64_t *row, uint32_t w, uint32_t cw, const uint64_t *x) {
    if constexpr (kCondVec == 2) {
        if (w + 1 < cw) {
            u64x2_t v;
            v.x = x[0];
            v.y = x[1];
#if CFPQ_COND_NT
            __builtin_nontemporal_store(v, reinterpret_cast<u64x2_t *>(row + w));
#else
            *reinterpret_cast<u64x2_t *>(row + w) = v;
#endif
        } else if (w < cw) {
            store_row_word(row + w, x[0]);
        }
    } else if (w < cw) {
        store_row_word(row + w, x[0]);
    }
}

// word offset of component c's row: in R, or (bit 63 set) in the answer
// matrix for an aliased answer row (see comp_row)
__device__ __forceinline__ uint64_t comp_off(uint32_t c, uint32_t n, uint32_t P, const uint32_t *flags,
                                             const uint32_t *multi) {
    const uint32_t f = flags[c / n];
    if ((f & kAliasFinal) && multi[c] == 0) return (1ull << 63) | (((uint64_t)(f >> kFlagBoxShift) * n + (c % n)) * P);
    return (uint64_t)c * P;
}
__device__ __forceinline__ uint64_t *off_ptr(uint64_t o, uint64_t *R, uint64_t *NT) {
    return (o >> 63) ? NT + (o & ~(1ull << 63)) : R + o;
}

// Edge-parallel walk over the edges of transition k of every lane's node
// (lane j owns node j of the work item; b/e/sb: its edge range and the base
// index of the transition's source (or target) state).  fn(j, e, sb_j, c_j)
// runs once per edge, 64 edges at a time whatever their owners' degrees.
template <class F>
__device__ __forceinline__ void edge_walk(uint32_t *scan, uint32_t b, uint32_t e, uint32_t sb, uint32_t cm, F &&fn) {
    const int lane = __lane_id();
    const uint32_t incl = wave_incl_scan(e - b);
    const uint32_t total = shfl_u32(incl, kWave - 1);
    if (total == 0) return;
    scan[lane] = incl;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t f0 = 0; f0 < total; f0 += kWave) {
        const uint32_t f = f0 + (uint32_t)lane;
        uint32_t lo = 0, hi = kWave - 1;   // owner: first node whose inclusive count exceeds f
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (scan[mid] > f) hi = mid;
            else lo = mid + 1;
        }
        const uint32_t bj = shfl_u32(b, (int)lo), sbj = shfl_u32(sb, (int)lo), cj = shfl_u32(cm, (int)lo);
        const uint32_t startj = lo ? scan[lo - 1] : 0u;
        if (f < total) fn(lo, bj + (f - startj), sbj, cj);
    }
    __builtin_amdgcn_wave_barrier();
}

// One node with the whole wavefront: OR the chunk of every predecessor row,
// add the seed bit, write (nodes with more than kCondPredCap listed rows).
__device__ void level_node_wave(const ProdGraph &g, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                const uint32_t *multi, uint64_t *R, uint64_t *NT, uint8_t *nz, const uint32_t *flags,
                                uint32_t p, uint32_t c, uint32_t ch, uint32_t nch,
                                unsigned long long *box_pairs, unsigned long long &pairs0,
                                unsigned long long &words_w, unsigned long long &words_r) {
    const int lane = __lane_id();
    const uint32_t cwds = cond_chunk_words(Pn);
    const uint32_t pass0 = ch * cwds;
    const uint32_t cw = (Pn - pass0 < cwds) ? Pn - pass0 : cwds;
    const bool single = multi[c] == 0;
    const uint32_t q = p / g.n, v = p - q * g.n;
    const uint32_t fq = flags[q];
    const bool alias = single && (fq & kAliasFinal);
    uint64_t *row = comp_row(c, g.n, P, flags, multi, R, NT) + pass0;
    const uint64_t seed_word =
        (single && (fq & kStartState) && (!g.src_mask || mask_bit(g.src_mask, v))) ? 1ull << (v & 63) : 0ull;
    const uint32_t seed_w = v >> 6;
    uint64_t acc[kCondChunks];
#pragma unroll
    for (int k = 0; k < kCondChunks; ++k) acc[k] = 0;
    uint32_t last = 0xFFFFFFFFu;
    for (uint32_t t = g.in_off[q]; t < g.in_off[q + 1]; ++t) {
        const InTrans tr = g.in_tr[t];
        const uint32_t *o = g.goff + (uint64_t)tr.sym * (g.n + 1) + v;
        const uint32_t b = o[0], e = o[1], sb = tr.src * g.n;
        for (uint32_t e0 = b; e0 < e; e0 += kWave) {
            uint32_t cx = c;
            bool use = false;
            if (e0 + lane < e) {
                cx = scc[sb + g.gidx[e0 + lane]];
                use = cx != c && nz[(uint64_t)cx * nch + ch];  // empty chunks hold no bits
            }
            uint64_t m = __ballot(use);
            while (m) {
                const int i = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                const uint32_t ci = (uint32_t)__builtin_amdgcn_readlane((int)cx, i);
                if (ci == last) continue;  // same row as the one just OR-ed
                last = ci;
                if (lane == 0) words_r += cw;
                const uint64_t *src = comp_row(ci, g.n, P, flags, multi, R, NT) + pass0;
#pragma unroll
                for (int k = 0; k < kCondChunks; ++k) {
                    const uint32_t w = pass0 + k * kWave + lane;
                    if (w < pass0 + cw) acc[k] |= src[k * kWave + lane];
                }
            }
        }
    }
    bool nonzero = false;
#pragma unroll
    for (int k = 0; k < kCondChunks; ++k) {
        const uint32_t w = pass0 + k * kWave + lane;
        if (w == seed_w && w < pass0 + cw) acc[k] |= seed_word;
        nonzero |= acc[k] != 0;
    }
    // a chunk that stays empty is neither written nor read later -- except
    // in an answer row, which must be complete
    const bool any_bits = __ballot(nonzero) != 0;
    if (any_bits || alias) {
        unsigned long long pc = 0;
#pragma unroll
        for (int k = 0; k < kCondChunks; ++k) {
            const uint32_t w = pass0 + k * kWave + lane;
            if (w < pass0 + cw) {
                if (single)
                    store_row_word(&row[k * kWave + lane], acc[k]);
                else if (acc[k])
                    atomicOr((unsigned long long *)&row[k * kWave + lane], acc[k]);
                if (alias) pc += (unsigned long long)__popcll(acc[k]);
            }
        }
        if (alias) {
            const uint32_t box = fq >> kFlagBoxShift;
            if (box == 0) pairs0 += pc;
            else if (pc) atomicAdd(&box_pairs[box * kWave], pc);
        }
        if (lane == 0) {
            if (any_bits) nz[(uint64_t)c * nch + ch] = 1;
            words_w += cw;
        }
    }
}

// One topological level L of the component graph: every component whose
// predecessors are all done gets its row (per 512-word chunk) as the OR of
// its predecessors' rows plus its seed bit, then releases its successors.
// A work item is 64 consecutive product nodes (one per lane) and one chunk:
//   A. edge-parallel over the items' in-edges: predecessor components with a
//      non-empty chunk go to a short LDS list per node (with their row
//      offsets, so the OR loop issues nothing but row loads);
//   B. the whole wavefront ORs a listed node's rows (8 words per lane), two
//      nodes per step with all their row loads in flight together, and
//      writes the chunk (CFPQ_COND_PAIR = 0 selects lane groups of
//      CFPQ_COND_GROUP_LANES lanes per node instead); nodes with longer
//      lists take the whole-wavefront path;
//   C. (first chunk only) edge-parallel over the out-edges: retire the
//      in-degree stripes of successor components and release them into
//      level L + 1.
// at least four wavefronts per SIMD: the kernel is held to 128 VGPRs, so all
// CFPQ_COND_BLOCKS_PER_CU = 4 workgroups of 4 wavefronts fit a compute unit
#ifndef CFPQ_COND_MIN_WAVES
#define CFPQ_COND_MIN_WAVES 4
#endif
#ifndef CFPQ_COND_ZERO16
#define CFPQ_COND_ZERO16 1
#endif
static_assert(!CFPQ_COND_ZERO16 || CFPQ_COND_CHUNK_ALIGN % 2 == 0, "16-byte stores need chunks on even words");
__global__ __launch_bounds__(kBlock, CFPQ_COND_MIN_WAVES) void k_cond_level(ProdGraph g, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                                       const uint32_t *multi, uint32_t *indeg, uint32_t *pending,
                                                       uint32_t *lev, uint64_t *R, uint64_t *NT, uint8_t *nz,
                                                       const uint32_t *flags, uint32_t L,
                                                       const unsigned long long *ctr_prev,
                                                       unsigned long long *ctr_next, unsigned long long *ctr_clear,
                                                       unsigned long long *box_pairs, unsigned long long *bytes_ctr) {
    __shared__ uint64_t s_pred[kBlock / kWave][kCondNodes][kCondPredCap];
    __shared__ uint32_t s_cnt[kBlock / kWave][kCondNodes];
    __shared__ uint32_t s_scan[kBlock / kWave][kCondNodes];
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_clear = 0;  // the counter level L + 2 will write
    if (*ctr_prev == 0) return;  // nothing reached level L
    const uint32_t N = g.nQ * g.n;
    const int lane = __lane_id();
    const uint32_t wib = threadIdx.x / kWave;
    [[maybe_unused]] const int grp = lane / kCondGroupLanes, gl = lane % kCondGroupLanes;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint32_t nch = cond_chunks(Pn), cwds = cond_chunk_words(Pn);
    const uint64_t items = (((uint64_t)N + kCondNodes - 1) / kCondNodes) * nch;
    unsigned long long released = 0, pairs0 = 0, words_w = 0, words_r = 0;
    for (uint64_t it = wave; it < items; it += nwaves) {
        const uint64_t base = (it / nch) * kCondNodes;
        const uint32_t ch = (uint32_t)(it % nch);
        const uint32_t pass0 = ch * cwds;
        const uint32_t cw = (Pn - pass0 < cwds) ? Pn - pass0 : cwds;  // words in chunk
        const uint32_t mine = (uint32_t)(base + lane);
        uint32_t cm = 0;
        bool at = false;
        if (mine < N) {
            cm = scc[mine];
            at = lev[cm] == L;
        }
        const uint64_t todo = __ballot(at);
        if (!todo) continue;
        // node metadata (lane j: node base + j)
        uint32_t q = 0, v = 0, fq = 0, tb = 0, te = 0, single = 0;
        uint64_t own = 0;
        if (at) {
            q = mine / g.n;
            v = mine - q * g.n;
            fq = flags[q];
            single = multi[cm] == 0;
            own = comp_off(cm, g.n, P, flags, multi);
            tb = g.in_off[q];
            te = g.in_off[q + 1];
        }
        // A. listed predecessor rows: from the node's links where it has
        // them (no edge walk), else edge-parallel over its in-edges
        s_cnt[wib][lane] = 0;
        bool walk_in = at;
        if (g.xin_cnt && at) {
            const uint32_t ic = g.xin_cnt[mine];
            if (ic <= kCondLinks) {
                walk_in = false;
                uint32_t cnt = 0;
                for (uint32_t r = 0; r < ic; ++r) {
                    const uint32_t cx = g.xin[(uint64_t)mine * kCondLinks + r];
                    if (nz[(uint64_t)cx * nch + ch]) s_pred[wib][lane][cnt++] = comp_off(cx, g.n, P, flags, multi);
                }
                s_cnt[wib][lane] = cnt;
            }
        }
        static_assert(kCondLinks <= kCondPredCap, "linked predecessors fit the LDS list");
        const uint32_t ntr = wave_max_u32(walk_in ? te - tb : 0u);
        for (uint32_t k = 0; k < ntr; ++k) {
            uint32_t b = 0, e = 0, sb = 0;
            if (walk_in && tb + k < te) {
                const InTrans tr = g.in_tr[tb + k];
                const uint32_t *o = g.goff + (uint64_t)tr.sym * (g.n + 1) + v;
                b = o[0];
                e = o[1];
                sb = tr.src * g.n;
            }
            edge_walk(s_scan[wib], b, e, sb, cm, [&](uint32_t j, uint32_t ei, uint32_t sbj, uint32_t cj) {
                const uint32_t cx = scc[sbj + g.gidx[ei]];
                if (cx == cj || !nz[(uint64_t)cx * nch + ch]) return;
                const uint64_t off = comp_off(cx, g.n, P, flags, multi);
                const uint32_t have = s_cnt[wib][j];
                for (uint32_t r = 0; r < have && r < kCondPredCap; ++r)
                    if (s_pred[wib][j][r] == off) return;   // listed already
                const uint32_t slot = atomicAdd(&s_cnt[wib][j], 1u);
                if (slot < kCondPredCap) s_pred[wib][j][slot] = off;
            });
        }
        __builtin_amdgcn_wave_barrier();
        const uint32_t my_cnt = s_cnt[wib][lane];
        const uint64_t over = __ballot(at && my_cnt > kCondPredCap);
        // B. the listed nodes' rows
        uint64_t pend = todo & ~over;
#if CFPQ_COND_PAIR
        // whole wavefront per node, kNS nodes per step: the row loads of all
        // of them are issued before any is waited for
        static_assert(kCondGroupLanes == kWave, "groups of whole-wavefront nodes");
        constexpr int kNS = CFPQ_COND_PAIR;
        while (pend) {
            int jn[kNS];
#pragma unroll
            for (int q = 0; q < kNS; ++q) {
                jn[q] = pend ? __ffsll((unsigned long long)pend) - 1 : -1;
                if (jn[q] >= 0) pend &= pend - 1;
            }
            uint32_t cN[kNS], vN[kNS], fqN[kNS], cntN[kNS], sgN[kNS];
            uint64_t ownN[kNS];
            bool doN[kNS], aliasN[kNS], seedN[kNS], anyN[kNS];
            uint32_t kmax = 0;
#pragma unroll
            for (int q = 0; q < kNS; ++q) {
                const int j = jn[q] < 0 ? jn[0] : jn[q];
                cN[q] = (uint32_t)__builtin_amdgcn_readlane((int)cm, j);
                vN[q] = (uint32_t)__builtin_amdgcn_readlane((int)v, j);
                fqN[q] = (uint32_t)__builtin_amdgcn_readlane((int)fq, j);
                cntN[q] = jn[q] < 0 ? 0u : (uint32_t)__builtin_amdgcn_readlane((int)my_cnt, j);
                sgN[q] = (uint32_t)__builtin_amdgcn_readlane((int)single, j);
                ownN[q] = shfl_u64(own, j);
                const bool seeded = sgN[q] && (fqN[q] & kStartState) && (!g.src_mask || mask_bit(g.src_mask, vN[q]));
                const uint32_t sw = vN[q] >> 6;
                seedN[q] = jn[q] >= 0 && seeded && sw >= pass0 && sw < pass0 + cw;
                anyN[q] = cntN[q] > 0 || seedN[q];
                aliasN[q] = jn[q] >= 0 && sgN[q] && (fqN[q] & kAliasFinal);
                doN[q] = jn[q] >= 0 && (anyN[q] || aliasN[q]);
                kmax = cntN[q] > kmax ? cntN[q] : kmax;
            }
            uint64_t acc[kNS][kCondPassWords];
#pragma unroll
            for (int q = 0; q < kNS; ++q)
#pragma unroll
                for (int kk = 0; kk < kCondPassWords; ++kk) acc[q][kk] = 0;
            for (uint32_t k = 0; k < kmax; ++k) {
                const uint64_t *src[kNS];
                uint64_t keep[kNS];
#pragma unroll
                for (int q = 0; q < kNS; ++q) {
                    // past a node's list: re-read the first node's row (k is
                    // inside the longest list, found first), masked off
                    const bool in = k < cntN[q];
                    int jj = jn[0];
#pragma unroll
                    for (int r = 0; r < kNS; ++r)
                        if (k < cntN[r]) { jj = jn[r]; break; }
                    if (in) jj = jn[q];
                    src[q] = off_ptr(s_pred[wib][jj][k], R, NT) + pass0;
                    keep[q] = in ? ~0ull : 0ull;
                }
                uint64_t x[kNS][kCondPassWords];
#pragma unroll
                for (int q = 0; q < kNS; ++q)
#pragma unroll
                    for (int kk = 0; kk < kCondPassWords; kk += kCondVec)
                        load_words(src[q], cond_word(kk, lane), cw, &x[q][kk]);
#pragma unroll
                for (int q = 0; q < kNS; ++q)
#pragma unroll
                    for (int kk = 0; kk < kCondPassWords; ++kk) acc[q][kk] |= x[q][kk] & keep[q];
            }
#pragma unroll
            for (int q = 0; q < kNS; ++q) {
                if (!doN[q]) continue;
                uint64_t *row = off_ptr(ownN[q], R, NT) + pass0;
#if CFPQ_COND_ZERO16
                if (!anyN[q]) {
                    // an empty answer-row chunk (nothing listed, no seed):
                    // zeros in 16-byte streaming stores (chunks and rows start
                    // on 16-word boundaries)
                    for (uint32_t w = 2 * (uint32_t)lane; w < cw; w += 2 * kWave) {
                        if (w + 1 < cw) {
                            u64x2_t z;
                            z.x = 0;
                            z.y = 0;
                            __builtin_nontemporal_store(z, reinterpret_cast<u64x2_t *>(row + w));
                        } else {
                            store_row_word(row + w, 0ull);
                        }
                    }
                    if (lane == 0) words_w += cw;
                    continue;
                }
#endif
                unsigned long long pc = 0;
#pragma unroll
                for (int kk = 0; kk < kCondPassWords; kk += kCondVec) {
                    const uint32_t w = cond_word(kk, lane);
#pragma unroll
                    for (int j = 0; j < kCondVec; ++j) {
                        if (seedN[q] && w + j == (vN[q] >> 6) - pass0) acc[q][kk + j] |= 1ull << (vN[q] & 63);
                        if (aliasN[q] && w + j < cw) pc += (unsigned long long)__popcll(acc[q][kk + j]);
                    }
                    if (sgN[q]) {
                        store_words(row, w, cw, &acc[q][kk]);
                    } else {
#pragma unroll
                        for (int j = 0; j < kCondVec; ++j)
                            if (w + j < cw && acc[q][kk + j])
                                atomicOr((unsigned long long *)&row[w + j], acc[q][kk + j]);
                    }
                }
                if (aliasN[q]) {
                    const uint32_t box = fqN[q] >> kFlagBoxShift;
                    if (box == 0) pairs0 += pc;
                    else if (pc) atomicAdd(&box_pairs[box * kWave], pc);
                }
                if (lane == 0) {
                    if (anyN[q]) nz[(uint64_t)cN[q] * nch + ch] = 1;
                    words_w += cw;
                    words_r += (unsigned long long)cntN[q] * cw;
                }
            }
        }
#else
        while (pend) {
            int jg = -1;
#pragma unroll
            for (int gi = 0; gi < kWave / kCondGroupLanes; ++gi) {
                if (pend) {
                    const int j = __ffsll((unsigned long long)pend) - 1;
                    pend &= pend - 1;
                    if (grp == gi) jg = j;
                }
            }
            const int js = jg < 0 ? 0 : jg;
            const uint32_t cj = shfl_u32(cm, js), vj = shfl_u32(v, js), fqj = shfl_u32(fq, js);
            const uint32_t cntj = shfl_u32(my_cnt, js), singlej = shfl_u32(single, js);
            const uint64_t ownj = shfl_u64(own, js);
            if (jg < 0) continue;
            const bool seeded = singlej && (fqj & kStartState) && (!g.src_mask || mask_bit(g.src_mask, vj));
            const uint32_t sw = vj >> 6;   // the seed: source vj begins at (start, vj)
            const bool seed_here = seeded && sw >= pass0 && sw < pass0 + cw;
            // every listed row has a non-empty chunk (its flag says so), so the
            // chunk is non-empty iff something is listed or the seed is in it
            const bool any_bits = cntj > 0 || seed_here;
            const bool alias = singlej && (fqj & kAliasFinal);
            if (!any_bits && !alias) continue;   // an empty chunk is neither written nor read later
            uint64_t *row = off_ptr(ownj, R, NT) + pass0;
            unsigned long long pc = 0;
#pragma unroll
            for (int h = 0; h < kCondPasses; ++h) {
                constexpr int kH = kCondPassWords;
                const uint32_t hw0 = (uint32_t)(h * kH * kCondGroupLanes);
                uint64_t acc[kH];
#pragma unroll
                for (int kk = 0; kk < kH; ++kk) acc[kk] = 0;
                for (uint32_t k = 0; k < cntj; ++k) {
                    const uint64_t *src = off_ptr(s_pred[wib][jg][k], R, NT) + pass0 + hw0;
#pragma unroll
                    for (int kk = 0; kk < kH; ++kk) {
                        const uint32_t w = hw0 + (uint32_t)(kk * kCondGroupLanes + gl);
                        if (w < cw) acc[kk] |= src[kk * kCondGroupLanes + gl];
                    }
                }
                if (seed_here) {
#pragma unroll
                    for (int kk = 0; kk < kH; ++kk)
                        if (hw0 + (uint32_t)(kk * kCondGroupLanes + gl) == sw - pass0) acc[kk] |= 1ull << (vj & 63);
                }
#pragma unroll
                for (int kk = 0; kk < kH; ++kk) {
                    const uint32_t w = hw0 + (uint32_t)(kk * kCondGroupLanes + gl);
                    if (w < cw) {
                        if (singlej)
                            store_row_word(&row[w], acc[kk]);
                        else if (acc[kk])
                            atomicOr((unsigned long long *)&row[w], acc[kk]);
                        if (alias) pc += (unsigned long long)__popcll(acc[kk]);
                    }
                }
            }
            if (alias) {
                const uint32_t box = fqj >> kFlagBoxShift;
                if (box == 0) pairs0 += pc;
                else if (pc) atomicAdd(&box_pairs[box * kWave], pc);
            }
            if (gl == 0) {
                if (any_bits) nz[(uint64_t)cj * nch + ch] = 1;
                words_w += cw;
                words_r += (unsigned long long)cntj * cw;
            }
        }
#endif
        for (uint64_t ov = over; ov;) {
            const int j = __ffsll((unsigned long long)ov) - 1;
            ov &= ov - 1;
            level_node_wave(g, P, Pn, scc, multi, R, NT, nz, flags, (uint32_t)base + (uint32_t)j,
                            (uint32_t)__builtin_amdgcn_readlane((int)cm, j), ch, nch, box_pairs, pairs0, words_w,
                            words_r);
        }
        // C. release successor components (once per node: first chunk)
        if (ch == 0) {
            // from the node's links where it has them, else edge-parallel
            // over its out-edges
            bool walk_out = at;
            if (g.xout_cnt && at) {
                const uint32_t oc = g.xout_cnt[mine];
                if (oc <= kCondLinks) {
                    walk_out = false;
                    for (uint32_t r = 0; r < oc; ++r) {
                        const uint32_t si = g.xout[(uint64_t)mine * kCondLinks + r];
                        const uint32_t cx = si / kStripes;
                        if (atomicSub(&indeg[si], 1u) == 1u && atomicSub(&pending[cx], 1u) == 1u) {
                            lev[cx] = L + 1;
                            ++released;
                        }
                    }
                }
            }
            uint32_t ob = 0, oe = 0;
            if (walk_out) {
                ob = g.out_off[q];
                oe = g.out_off[q + 1];
            }
            const uint32_t nout = wave_max_u32(oe - ob);
            for (uint32_t k = 0; k < nout; ++k) {
                uint32_t b = 0, e = 0, sb = 0;
                if (ob + k < oe) {
                    const InTrans tr = g.out_tr[ob + k];   // src field: destination state
                    const uint32_t *o = g.soff + (uint64_t)tr.sym * (g.n + 1) + v;
                    b = o[0];
                    e = o[1];
                    sb = tr.src * g.n;
                }
                edge_walk(s_scan[wib], b, e, sb, cm, [&](uint32_t j, uint32_t ei, uint32_t sbj, uint32_t cj) {
                    const uint32_t y = sbj + g.sidx[ei];
                    const uint32_t cx = scc[y];
                    // the last edge of a stripe retires the stripe, the last
                    // stripe releases the component
                    if (cx != cj && atomicSub(&indeg[(uint64_t)cx * kStripes + y % kStripes], 1u) == 1u &&
                        atomicSub(&pending[cx], 1u) == 1u) {
                        lev[cx] = L + 1;
                        ++released;
                    }
                });
            }
        }
    }
    count_add(ctr_next, released);
    // box 0's answer pairs: one striped atomic per wavefront
    pairs0 = wsum(pairs0);
    if (lane == 0 && pairs0) atomicAdd(&box_pairs[wave % kWave], pairs0);
    // words written and predecessor words requested (profiling only), striped
    // over kWave counter pairs
    if (bytes_ctr) {
        words_w = wsum(words_w);
        words_r = wsum(words_r);
        if (lane == 0 && (words_w | words_r)) {
            atomicAdd(&bytes_ctr[2 * (wave % kWave)], words_w);
            atomicAdd(&bytes_ctr[2 * (wave % kWave) + 1], words_r);
        }
    }
}

// copy each component's row to its other members (closure blocks on request)
__global__ __launch_bounds__(kBlock) void k_cond_expand(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                                        const uint8_t *nz, uint64_t *T) {
    const uint32_t nch = cond_chunks(Pn), cwds = cond_chunk_words(Pn);
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t pp = wave; pp < N; pp += nwaves) {
        const uint32_t c = scc[pp];
        const uint64_t *src = T + (uint64_t)c * P;
        uint64_t *dst = T + pp * P;
        for (uint32_t w = lane; w < Pn; w += kWave) {
            const bool live = nz[(uint64_t)c * nch + w / cwds] != 0;
            if (c != pp || !live) dst[w] = live ? src[w] : 0ull;
        }
    }
}

#ifndef CFPQ_COND_BLOCKS_PER_CU
#define CFPQ_COND_BLOCKS_PER_CU 4
#endif
// compute units of the current device (looked up once per device)
uint32_t device_cus() {
    static std::atomic<uint32_t> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    uint32_t c = cus[dev].load(std::memory_order_relaxed);
    if (!c) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        c = (uint32_t)v;
        cus[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

uint32_t node_grid(uint64_t N) {
    uint64_t g = (N + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    return (uint32_t)(g ? g : 1);
}

uint32_t wave_grid(uint64_t N) {
    uint64_t g = (N + (kBlock / kWave) - 1) / (kBlock / kWave);
    if (g > 4096) g = 4096;
    return (uint32_t)(g ? g : 1);
}

}  // namespace

hipError_t launch_trim(const ProdGraph &g, uint8_t *alive, uint32_t *scc, const unsigned long long *prev,
                       unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_trim, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, scc, prev, ctr);
    return hipGetLastError();
}

hipError_t launch_pivot(const ProdGraph &g, const uint8_t *alive, unsigned long long *best, hipStream_t s) {
    hipLaunchKernelGGL(k_pivot, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, best);
    return hipGetLastError();
}

hipError_t launch_reach(const ProdGraph &g, const uint8_t *alive, uint32_t *fw, uint32_t *bw, const ReachQueues &rq,
                        uint32_t it, unsigned long long *ctr, hipStream_t s) {
    // one wavefront per 64 frontier entries of either direction, at most
    // 2 * ceil(N / 64) items
    const uint64_t N = (uint64_t)g.nQ * g.n;
    hipLaunchKernelGGL(k_reach, dim3(wave_grid(2 * ((N + kWave - 1) / kWave))), dim3(kBlock), 0, s, g, alive, fw, bw,
                       rq, it, ctr);
    return hipGetLastError();
}

hipError_t launch_pivot_seed(const unsigned long long *best, uint32_t *fw, uint32_t *bw, const ReachQueues &rq,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_pivot_seed, dim3(1), dim3(64), 0, s, best, fw, bw, rq);
    return hipGetLastError();
}

hipError_t launch_fwbw_assign(uint32_t N, uint8_t *alive, const uint32_t *fw, const uint32_t *bw,
                              const unsigned long long *best, uint32_t *scc, unsigned long long *ctr,
                              const unsigned long long *open0, const unsigned long long *open1, hipStream_t s) {
    hipLaunchKernelGGL(k_fwbw_assign, dim3(node_grid(N)), dim3(kBlock), 0, s, N, alive, fw, bw, best, scc, ctr, open0,
                       open1);
    return hipGetLastError();
}

hipError_t launch_color_init(uint32_t N, const uint8_t *alive, uint32_t *color, uint8_t *found, hipStream_t s) {
    hipLaunchKernelGGL(k_color_init, dim3(node_grid(N)), dim3(kBlock), 0, s, N, alive, color, found);
    return hipGetLastError();
}

hipError_t launch_color_prop(const ProdGraph &g, const uint8_t *alive, uint32_t *color,
                             const unsigned long long *prev, unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_color_prop, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, color, prev,
                       ctr);
    return hipGetLastError();
}

hipError_t launch_color_roots(uint32_t N, const uint8_t *alive, const uint32_t *color, uint8_t *found, uint32_t *scc,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_color_roots, dim3(node_grid(N)), dim3(kBlock), 0, s, N, alive, color, found, scc);
    return hipGetLastError();
}

hipError_t launch_color_back(const ProdGraph &g, const uint8_t *alive, const uint32_t *color, uint8_t *found,
                             uint32_t *scc, const unsigned long long *prev, unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_color_back, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, color,
                       found, scc, prev, ctr);
    return hipGetLastError();
}

hipError_t launch_color_remove(uint32_t N, uint8_t *alive, const uint8_t *found, unsigned long long *ctr,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_color_remove, dim3(node_grid(N)), dim3(kBlock), 0, s, N, alive, found, ctr);
    return hipGetLastError();
}

hipError_t launch_cond_count(const ProdGraph &g, const uint32_t *scc, uint32_t *size, uint32_t *stripe,
                             const unsigned long long *skip_if, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_count, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, scc, size, stripe,
                       skip_if);
    return hipGetLastError();
}

hipError_t launch_cond_seed(uint32_t n, uint32_t P, uint32_t Pn, uint32_t nQ, const uint32_t *starts,
                            uint32_t n_starts, const uint32_t *scc, const uint32_t *multi, uint64_t *R, uint8_t *nz,
                            const uint64_t *mask, const unsigned long long *skip_if, hipStream_t s) {
    const uint64_t N = (uint64_t)nQ * n;
    const uint32_t nch = cond_chunks(Pn), cwds = cond_chunk_words(Pn);
    hipLaunchKernelGGL(k_cond_zero_multi, dim3(node_grid(N)), dim3(kBlock), 0, s, (uint32_t)N, P, Pn, scc, multi, R,
                       skip_if);
    hipLaunchKernelGGL(k_cond_seed, dim3(node_grid((uint64_t)n * n_starts)), dim3(kBlock), 0, s, n, P, starts,
                       n_starts, scc, multi, R, nz, nch, cwds, mask, skip_if);
    return hipGetLastError();
}

hipError_t launch_cond_roots(uint32_t N, const uint32_t *scc, const uint32_t *stripe, uint32_t *pending,
                             uint32_t *lev, unsigned long long *ctr, const unsigned long long *skip_if, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_roots, dim3(node_grid(N)), dim3(kBlock), 0, s, N, scc, stripe, pending, lev, ctr,
                       skip_if);
    return hipGetLastError();
}

hipError_t launch_cond_level(const ProdGraph &g, uint32_t P, uint32_t Pn, const uint32_t *scc, const uint32_t *multi,
                             uint32_t *indeg, uint32_t *pending, uint32_t *lev, uint64_t *R, uint64_t *NT, uint8_t *nz,
                             const uint32_t *flags, uint32_t L, const unsigned long long *ctr_prev,
                             unsigned long long *ctr_next, unsigned long long *ctr_clear, unsigned long long *box_pairs,
                             unsigned long long *bytes_ctr, hipStream_t s) {
    const uint64_t N = (uint64_t)g.nQ * g.n;
    const uint64_t nch = cond_chunks(Pn);
    // at most CFPQ_COND_BLOCKS_PER_CU workgroups per compute unit, striding
    // over the work items: all resident at once, no second partial round
    // (4 and 5 per CU measured even, ahead of 3, 6 and of one workgroup per
    // item)
    uint32_t grid = wave_grid((N + kCondNodes - 1) / kCondNodes * nch);
    const uint32_t cap = CFPQ_COND_BLOCKS_PER_CU * device_cus();
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(k_cond_level, dim3(grid), dim3(kBlock), 0, s, g, P, Pn, scc, multi, indeg, pending, lev, R, NT,
                       nz, flags, L, ctr_prev, ctr_next, ctr_clear, box_pairs, bytes_ctr);
    return hipGetLastError();
}

hipError_t launch_cond_expand(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc, const uint8_t *nz, uint64_t *T,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_cond_expand, dim3(wave_grid(N)), dim3(kBlock), 0, s, N, P, Pn, scc, nz, T);
    return hipGetLastError();
}

}  // namespace cfpq
