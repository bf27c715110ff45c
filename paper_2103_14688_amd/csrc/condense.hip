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

namespace cfpq {

namespace {

constexpr int kCondChunks = 8;
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

#define NODE_LOOP(N)                                                                        \
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < (N); p += gridDim.x * blockDim.x)

__device__ __forceinline__ void count_add(unsigned long long *ctr, unsigned long long c) {
    c = wsum(c);
    if (__lane_id() == 0 && c) atomicAdd(ctr, c);
}

// ----------------------------------------------------------------------------
// component search
// ----------------------------------------------------------------------------
__global__ void k_trim(ProdGraph g, uint8_t *alive, uint32_t *scc, const unsigned long long *prev,
                       unsigned long long *ctr) {
    if (prev && *prev == 0) return;  // the previous sweep removed nothing
    const uint32_t N = g.nQ * g.n;
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (!alive[p]) continue;
        bool in = false, out = false;
        for_preds(g, p, [&](uint32_t x) {
            if (x != p && alive[x]) { in = true; return false; }
            return true;
        });
        if (in)
            for_succs(g, p, [&](uint32_t x) {
                if (x != p && alive[x]) { out = true; return false; }
                return true;
            });
        if (!in || !out) {
            alive[p] = 0;
            scc[p] = p;
            ++c;
        }
    }
    count_add(ctr, c);
}

__global__ void k_pivot(ProdGraph g, const uint8_t *alive, unsigned long long *best) {
    const uint32_t N = g.nQ * g.n;
    unsigned long long mine = 0;
    NODE_LOOP(N) {
        if (!alive[p]) continue;
        uint64_t din = 0, dout = 0;
        for_preds(g, p, [&](uint32_t) { ++din; return true; });
        for_succs(g, p, [&](uint32_t) { ++dout; return true; });
        uint64_t score = (din + 1) * (dout + 1);
        if (score > 0xFFFFFFFFull) score = 0xFFFFFFFFull;
        const unsigned long long key = (score << 32) | p;
        if (key > mine) mine = key;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(mine, off, kWave);
        mine = o > mine ? o : mine;
    }
    if (__lane_id() == 0 && mine) atomicMax(best, mine);
}

// one sweep of forward and backward reachability from the pivot, restricted
// to live nodes, marking in place: a live node with a marked live predecessor
// joins fw, one with a marked live successor joins bw.  Sweeps repeat until
// one marks nothing.
__global__ void k_reach(ProdGraph g, const uint8_t *alive, uint32_t *fw, uint32_t *bw,
                        const unsigned long long *prev, unsigned long long *ctr) {
    if (prev && *prev == 0) return;  // the previous sweep marked nothing
    const uint32_t N = g.nQ * g.n;
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (!alive[p]) continue;
        if (!fw[p]) {
            bool hit = false;
            for_preds(g, p, [&](uint32_t x) {
                if (alive[x] && fw[x]) { hit = true; return false; }
                return true;
            });
            if (hit) {
                fw[p] = 1;
                ++c;
            }
        }
        if (!bw[p]) {
            bool hit = false;
            for_succs(g, p, [&](uint32_t x) {
                if (alive[x] && bw[x]) { hit = true; return false; }
                return true;
            });
            if (hit) {
                bw[p] = 1;
                ++c;
            }
        }
    }
    count_add(ctr, c);
}

__global__ void k_set_u32(uint32_t *a, uint32_t i, uint32_t v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a[i] = v;
}

// one level of a push breadth-first search restricted to live nodes: every
// node of the input frontier marks its unmarked live successors (forward) or
// predecessors (backward) and appends them to the output frontier
__global__ void k_push(ProdGraph g, const uint8_t *alive, uint32_t *mark, int backward, const uint32_t *fin,
                       const unsigned long long *n_in, uint32_t *fout, unsigned long long *n_out) {
    const unsigned long long cnt = *n_in;
    if (cnt == 0) return;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = fin[i];
        auto f = [&](uint32_t x) {
            if (alive[x] && mark[x] == 0 && atomicExch(&mark[x], 1u) == 0u) {
                const unsigned long long at = atomicAdd(n_out, 1ull);
                fout[at] = x;
            }
            return true;
        };
        if (backward) for_preds(g, p, f); else for_succs(g, p, f);
    }
}

__global__ void k_set_u64(unsigned long long *a, unsigned long long v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a = v;
}

__global__ void k_fwbw_assign(uint32_t N, uint8_t *alive, const uint32_t *fw, const uint32_t *bw,
                              uint32_t pivot, uint32_t *scc, unsigned long long *ctr) {
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
        bool hit = false;
        for_succs(g, p, [&](uint32_t x) {
            if (alive[x] && found[x] && color[x] == cp) { hit = true; return false; }
            return true;
        });
        if (hit) {
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
// the source node, so that the many edges into one large component do not
// all meet on one address: stripe[c*kStripes + x % kStripes] counts edges
// x -> c.  pending[c] := number of non-zero stripes (filled by k_cond_roots).
__global__ void k_cond_count(ProdGraph g, const uint32_t *scc, uint32_t *size, uint32_t *stripe) {
    const uint32_t N = g.nQ * g.n;
    NODE_LOOP(N) {
        const uint32_t c = scc[p];
        if (c != p) size[c] = 1;  // a second member: the component is not a singleton
        for_preds(g, p, [&](uint32_t x) {
            if (scc[x] != c) atomicAdd(&stripe[(uint64_t)c * kStripes + x % kStripes], 1u);
            return true;
        });
    }
}

// rows of components with several members are accumulated with atomics:
// clear them (one wavefront per representative)
__global__ __launch_bounds__(kBlock) void k_cond_zero_multi(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                                            const uint32_t *multi, uint64_t *R) {
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t p = wave; p < N; p += nwaves) {
        if (scc[p] != p || !multi[p]) continue;
        uint64_t *row = R + p * P;
        for (uint32_t w = lane; w < Pn; w += kWave) row[w] = 0;
    }
}

// sources: (start, u) holds source bit u; only for several-member components
// (a single-member component's row is written whole, seed included, when its
// topological level is processed)
__global__ void k_cond_seed(uint32_t n, uint32_t P, const uint32_t *starts, uint32_t n_starts,
                            const uint32_t *scc, const uint32_t *multi, uint64_t *R, uint8_t *nz, uint32_t nch,
                            const uint64_t *mask) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)n_starts * n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t s = starts[i / n], u = (uint32_t)(i % n);
        if (mask && !mask_bit(mask, u)) continue;
        const uint32_t c = scc[s * n + u];
        if (multi[c]) {
            atomicOr((unsigned long long *)&R[(uint64_t)c * P + (u >> 6)], 1ull << (u & 63));
            nz[(uint64_t)c * nch + (u >> 6) / (kCondChunks * kWave)] = 1;
        }
    }
}

__global__ void k_cond_roots(uint32_t N, const uint32_t *scc, const uint32_t *stripe, uint32_t *pending,
                             uint32_t *lev, unsigned long long *ctr) {
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (scc[p] != p) continue;
        uint32_t nz = 0;
        for (uint32_t k = 0; k < kStripes; ++k) nz += stripe[(uint64_t)p * kStripes + k] != 0;
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

// one topological level: every node whose component sits at level L ORs the
// rows of its predecessors' components (outside its own) into its
// component's row, then releases its successors' components.  Work items are
// (block of 64 consecutive nodes, 512-word chunk of the row): a wavefront
// selects the block's nodes at level L by ballot and handles them one at a
// time over its chunk; predecessors are filtered lane-parallel (component id,
// external, not a repeat of the last row OR-ed); the chunk-0 wavefront also
// releases the successors' components with lane-parallel atomics.
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

__global__ __launch_bounds__(kBlock) void k_cond_level(ProdGraph g, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                                       const uint32_t *multi, uint32_t *indeg, uint32_t *pending,
                                                       uint32_t *lev, uint64_t *R, uint64_t *NT, uint8_t *nz,
                                                       const uint32_t *flags, uint32_t L,
                                                       const unsigned long long *ctr_prev,
                                                       unsigned long long *ctr_next, unsigned long long *ctr_clear,
                                                       unsigned long long *box_pairs, unsigned long long *bytes_ctr) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_clear = 0;  // the counter level L + 2 will write
    if (*ctr_prev == 0) return;  // nothing reached level L
    const uint32_t N = g.nQ * g.n;
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint32_t nch = (Pn + kCondChunks * kWave - 1) / (kCondChunks * kWave);
    const uint64_t items = (((uint64_t)N + kCondNodes - 1) / kCondNodes) * nch;
    unsigned long long released = 0, pairs0 = 0, words_w = 0, words_r = 0;
    for (uint64_t it = wave; it < items; it += nwaves) {
        const uint64_t base = (it / nch) * kCondNodes;
        const uint32_t ch = (uint32_t)(it % nch);
        const uint32_t pass0 = ch * (kCondChunks * kWave);
        const uint32_t cw = (Pn - pass0 < kCondChunks * kWave) ? Pn - pass0 : kCondChunks * kWave;  // words in chunk
        const uint32_t mine = (uint32_t)(base + lane);
        uint32_t cm = 0;
        bool at = false;
        if ((uint32_t)lane < kCondNodes && mine < N) {
            cm = scc[mine];
            at = lev[cm] == L;
        }
        uint64_t todo = __ballot(at);
        while (todo) {
            const int j = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const uint32_t p = (uint32_t)base + (uint32_t)j;
            const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)cm, j);
            const bool single = multi[c] == 0;
            const uint32_t q = p / g.n, v = p - q * g.n;
            const uint32_t fq = flags[q];
            const bool alias = single && (fq & kAliasFinal);
            uint64_t *row = comp_row(c, g.n, P, flags, multi, R, NT) + pass0;
            // seed bit of a single-member component: (start, v) is where source v begins
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
                        words_r += cw;
                        const uint64_t *src = comp_row(ci, g.n, P, flags, multi, R, NT) + pass0;
#pragma unroll
                        for (int k = 0; k < kCondChunks; ++k) {
                            const uint32_t w = pass0 + k * kWave + lane;
                            if (w < Pn) acc[k] |= src[k * kWave + lane];
                        }
                    }
                }
            }
            bool nonzero = false;
#pragma unroll
            for (int k = 0; k < kCondChunks; ++k) {
                const uint32_t w = pass0 + k * kWave + lane;
                if (w == seed_w) acc[k] |= seed_word;
                nonzero |= acc[k] != 0;
            }
            // a chunk that stays empty is neither written nor read later --
            // except in an answer row, which must be complete
            const bool any_bits = __ballot(nonzero) != 0;
            if (any_bits || alias) {
#pragma unroll
                for (int k = 0; k < kCondChunks; ++k) {
                    const uint32_t w = pass0 + k * kWave + lane;
                    if (w < Pn) {
                        if (single)
                            row[k * kWave + lane] = acc[k];
                        else if (acc[k])
                            atomicOr((unsigned long long *)&row[k * kWave + lane], acc[k]);
                        if (alias) pairs0 += (unsigned long long)__popcll(acc[k]);
                    }
                }
                if (lane == 0 && any_bits) nz[(uint64_t)c * nch + ch] = 1;
                words_w += cw;
            }
            if (alias && (fq >> kFlagBoxShift) != 0) {
                // answer pairs of a box other than 0: count directly
                unsigned long long t = wsum(pairs0);
                if (lane == 0 && t) atomicAdd(&box_pairs[(fq >> kFlagBoxShift) * kWave], t);
                pairs0 = 0;
            }
            if (pass0 == 0) {
                // release successor components, lane-parallel
                for (uint32_t t = g.out_off[q]; t < g.out_off[q + 1]; ++t) {
                    const InTrans tr = g.out_tr[t];
                    const uint32_t *o = g.soff + (uint64_t)tr.sym * (g.n + 1) + v;
                    const uint32_t b = o[0], e = o[1], sb = tr.src * g.n;
                    for (uint32_t e0 = b; e0 < e; e0 += kWave) {
                        if (e0 + lane < e) {
                            const uint32_t cx = scc[sb + g.sidx[e0 + lane]];
                            // the last edge of a stripe retires the stripe, the
                            // last stripe releases the component
                            if (cx != c && atomicSub(&indeg[(uint64_t)cx * kStripes + p % kStripes], 1u) == 1u &&
                                atomicSub(&pending[cx], 1u) == 1u) {
                                lev[cx] = L + 1;
                                ++released;
                            }
                        }
                    }
                }
            }
        }
    }
    released = wsum(released);
    if (lane == 0 && released) atomicAdd(ctr_next, released);
    // box 0's answer pairs: one striped atomic per wavefront
    pairs0 = wsum(pairs0);
    if (lane == 0 && pairs0) atomicAdd(&box_pairs[wave % kWave], pairs0);
    // words written and predecessor words requested (profiling only), striped
    // over kWave counter pairs
    if (bytes_ctr && lane == 0 && (words_w | words_r)) {
        atomicAdd(&bytes_ctr[2 * (wave % kWave)], words_w);
        atomicAdd(&bytes_ctr[2 * (wave % kWave) + 1], words_r);
    }
}

// copy each component's row to its other members (closure blocks on request)
__global__ __launch_bounds__(kBlock) void k_cond_expand(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                                        const uint8_t *nz, uint64_t *T) {
    const uint32_t nch = (Pn + kCondChunks * kWave - 1) / (kCondChunks * kWave);
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t pp = wave; pp < N; pp += nwaves) {
        const uint32_t c = scc[pp];
        const uint64_t *src = T + (uint64_t)c * P;
        uint64_t *dst = T + pp * P;
        for (uint32_t w = lane; w < Pn; w += kWave) {
            const bool live = nz[(uint64_t)c * nch + w / (kCondChunks * kWave)] != 0;
            if (c != pp || !live) dst[w] = live ? src[w] : 0ull;
        }
    }
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

hipError_t launch_reach(const ProdGraph &g, const uint8_t *alive, uint32_t *fw, uint32_t *bw,
                        const unsigned long long *prev, unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_reach, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, fw, bw, prev, ctr);
    return hipGetLastError();
}

hipError_t launch_push(const ProdGraph &g, const uint8_t *alive, uint32_t *mark, int backward, const uint32_t *fin,
                       const unsigned long long *n_in, uint32_t *fout, unsigned long long *n_out, uint32_t grid,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_push, dim3(grid), dim3(kBlock), 0, s, g, alive, mark, backward, fin, n_in, fout, n_out);
    return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long *a, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, a, v);
    return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t *a, uint32_t i, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, s, a, i, v);
    return hipGetLastError();
}

hipError_t launch_fwbw_assign(uint32_t N, uint8_t *alive, const uint32_t *fw, const uint32_t *bw, uint32_t pivot,
                              uint32_t *scc, unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_fwbw_assign, dim3(node_grid(N)), dim3(kBlock), 0, s, N, alive, fw, bw, pivot, scc, ctr);
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
                             hipStream_t s) {
    hipLaunchKernelGGL(k_cond_count, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, scc, size, stripe);
    return hipGetLastError();
}

hipError_t launch_cond_seed(uint32_t n, uint32_t P, uint32_t Pn, uint32_t nQ, const uint32_t *starts,
                            uint32_t n_starts, const uint32_t *scc, const uint32_t *multi, uint64_t *R, uint8_t *nz,
                            const uint64_t *mask, hipStream_t s) {
    const uint64_t N = (uint64_t)nQ * n;
    const uint32_t nch = (Pn + kCondChunks * kWave - 1) / (kCondChunks * kWave);
    hipLaunchKernelGGL(k_cond_zero_multi, dim3(wave_grid(N)), dim3(kBlock), 0, s, (uint32_t)N, P, Pn, scc, multi, R);
    hipLaunchKernelGGL(k_cond_seed, dim3(node_grid((uint64_t)n * n_starts)), dim3(kBlock), 0, s, n, P, starts,
                       n_starts, scc, multi, R, nz, nch, mask);
    return hipGetLastError();
}

hipError_t launch_cond_roots(uint32_t N, const uint32_t *scc, const uint32_t *stripe, uint32_t *pending,
                             uint32_t *lev, unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_roots, dim3(node_grid(N)), dim3(kBlock), 0, s, N, scc, stripe, pending, lev, ctr);
    return hipGetLastError();
}

hipError_t launch_cond_level(const ProdGraph &g, uint32_t P, uint32_t Pn, const uint32_t *scc, const uint32_t *multi,
                             uint32_t *indeg, uint32_t *pending, uint32_t *lev, uint64_t *R, uint64_t *NT, uint8_t *nz,
                             const uint32_t *flags, uint32_t L, const unsigned long long *ctr_prev,
                             unsigned long long *ctr_next, unsigned long long *ctr_clear, unsigned long long *box_pairs,
                             unsigned long long *bytes_ctr, hipStream_t s) {
    const uint64_t N = (uint64_t)g.nQ * g.n;
    const uint64_t nch = (Pn + kCondChunks * kWave - 1) / (kCondChunks * kWave);
    hipLaunchKernelGGL(k_cond_level, dim3(wave_grid((N + kCondNodes - 1) / kCondNodes * nch)), dim3(kBlock), 0, s, g, P,
                       Pn, scc,
                       multi, indeg, pending, lev, R, NT, nz, flags, L, ctr_prev, ctr_next, ctr_clear, box_pairs,
                       bytes_ctr);
    return hipGetLastError();
}

hipError_t launch_cond_expand(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc, const uint8_t *nz, uint64_t *T,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_cond_expand, dim3(wave_grid(N)), dim3(kBlock), 0, s, N, P, Pn, scc, nz, T);
    return hipGetLastError();
}

}  // namespace cfpq
