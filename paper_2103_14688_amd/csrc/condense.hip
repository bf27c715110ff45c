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
__global__ void k_trim(ProdGraph g, uint8_t *alive, uint32_t *scc, unsigned long long *ctr) {
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

// one level of a pull breadth-first search restricted to live nodes:
// mark[p] = level + 1 if a live predecessor (forward) or successor
// (backward) carries mark == level
__global__ void k_reach(ProdGraph g, const uint8_t *alive, uint32_t *mark, uint32_t level, int backward,
                        unsigned long long *ctr) {
    const uint32_t N = g.nQ * g.n;
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (!alive[p] || mark[p]) continue;
        bool hit = false;
        auto f = [&](uint32_t x) {
            if (alive[x] && mark[x] == level) { hit = true; return false; }
            return true;
        };
        if (backward) for_succs(g, p, f); else for_preds(g, p, f);
        if (hit) {
            mark[p] = level + 1;
            ++c;
        }
    }
    count_add(ctr, c);
}

__global__ void k_set_u32(uint32_t *a, uint32_t i, uint32_t v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a[i] = v;
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

__global__ void k_color_prop(ProdGraph g, const uint8_t *alive, uint32_t *color, unsigned long long *ctr) {
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
                             uint32_t *scc, unsigned long long *ctr) {
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
// size[c] := 1 if component c has more than one member; indeg[c] := number of
// product edges entering c from other components
__global__ void k_cond_count(ProdGraph g, const uint32_t *scc, uint32_t *size, uint32_t *indeg) {
    const uint32_t N = g.nQ * g.n;
    NODE_LOOP(N) {
        const uint32_t c = scc[p];
        if (c != p) size[c] = 1;  // a second member: the component is not a singleton
        uint32_t ext = 0;
        for_preds(g, p, [&](uint32_t x) {
            ext += scc[x] != c;
            return true;
        });
        if (ext) atomicAdd(&indeg[c], ext);
    }
}

// sources: (start, u) holds source bit u
__global__ void k_cond_seed(uint32_t n, uint32_t P, const uint32_t *starts, uint32_t n_starts,
                            const uint32_t *scc, uint64_t *R) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)n_starts * n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t s = starts[i / n], u = (uint32_t)(i % n);
        const uint32_t c = scc[s * n + u];
        atomicOr((unsigned long long *)&R[(uint64_t)c * P + (u >> 6)], 1ull << (u & 63));
    }
}

__global__ void k_cond_roots(uint32_t N, const uint32_t *scc, const uint32_t *indeg, uint32_t *lev,
                             unsigned long long *ctr) {
    unsigned long long c = 0;
    NODE_LOOP(N) {
        if (scc[p] != p) continue;
        if (indeg[p] == 0) {
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
// component's row, then releases its successors' components
__global__ __launch_bounds__(kBlock) void k_cond_level(ProdGraph g, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                                       const uint32_t *size, uint32_t *indeg, uint32_t *lev,
                                                       uint64_t *R, uint32_t L, const unsigned long long *ctr_prev,
                                                       unsigned long long *ctr_next, unsigned long long *ctr_clear) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_clear = 0;  // the counter level L + 2 will write
    if (*ctr_prev == 0) return;  // nothing reached level L
    const uint32_t N = g.nQ * g.n;
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long released = 0;
    for (uint64_t pp = wave; pp < N; pp += nwaves) {
        const uint32_t p = (uint32_t)pp;
        const uint32_t c = scc[p];
        if (lev[c] != L) continue;
        const bool single = size[c] == 0;
        uint64_t *row = R + (uint64_t)c * P;
        for (uint32_t pass0 = 0; pass0 < Pn; pass0 += kCondChunks * kWave) {
            uint64_t acc[kCondChunks];
#pragma unroll
            for (int k = 0; k < kCondChunks; ++k) acc[k] = 0;
            bool any = false;
            for_preds(g, p, [&](uint32_t x) {
                const uint32_t cx = scc[x];
                if (cx != c) {
                    any = true;
                    const uint64_t *src = R + (uint64_t)cx * P + pass0;
#pragma unroll
                    for (int k = 0; k < kCondChunks; ++k) {
                        const uint32_t w = pass0 + k * kWave + lane;
                        if (w < Pn) acc[k] |= src[k * kWave + lane];
                    }
                }
                return true;
            });
            if (!any) break;
#pragma unroll
            for (int k = 0; k < kCondChunks; ++k) {
                const uint32_t w = pass0 + k * kWave + lane;
                if (w < Pn && acc[k]) {
                    if (single)
                        row[w] |= acc[k];
                    else
                        atomicOr((unsigned long long *)&row[w], acc[k]);
                }
            }
        }
        if (lane == 0)
            for_succs(g, p, [&](uint32_t x) {
                const uint32_t cx = scc[x];
                if (cx != c && atomicSub(&indeg[cx], 1u) == 1u) {
                    lev[cx] = L + 1;
                    ++released;
                }
                return true;
            });
    }
    if (lane == 0 && released) atomicAdd(ctr_next, released);
}

// copy each component's row to its other members (closure blocks on request)
__global__ __launch_bounds__(kBlock) void k_cond_expand(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc,
                                                        uint64_t *T) {
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t pp = wave; pp < N; pp += nwaves) {
        const uint32_t c = scc[pp];
        if (c == pp) continue;
        const uint64_t *src = T + (uint64_t)c * P;
        uint64_t *dst = T + pp * P;
        for (uint32_t w = lane; w < Pn; w += kWave) dst[w] = src[w];
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

hipError_t launch_trim(const ProdGraph &g, uint8_t *alive, uint32_t *scc, unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_trim, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, scc, ctr);
    return hipGetLastError();
}

hipError_t launch_pivot(const ProdGraph &g, const uint8_t *alive, unsigned long long *best, hipStream_t s) {
    hipLaunchKernelGGL(k_pivot, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, best);
    return hipGetLastError();
}

hipError_t launch_reach(const ProdGraph &g, const uint8_t *alive, uint32_t *mark, uint32_t level, int backward,
                        unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_reach, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, mark, level,
                       backward, ctr);
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

hipError_t launch_color_prop(const ProdGraph &g, const uint8_t *alive, uint32_t *color, unsigned long long *ctr,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_color_prop, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, color, ctr);
    return hipGetLastError();
}

hipError_t launch_color_roots(uint32_t N, const uint8_t *alive, const uint32_t *color, uint8_t *found, uint32_t *scc,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_color_roots, dim3(node_grid(N)), dim3(kBlock), 0, s, N, alive, color, found, scc);
    return hipGetLastError();
}

hipError_t launch_color_back(const ProdGraph &g, const uint8_t *alive, const uint32_t *color, uint8_t *found,
                             uint32_t *scc, unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_color_back, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, alive, color,
                       found, scc, ctr);
    return hipGetLastError();
}

hipError_t launch_color_remove(uint32_t N, uint8_t *alive, const uint8_t *found, unsigned long long *ctr,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_color_remove, dim3(node_grid(N)), dim3(kBlock), 0, s, N, alive, found, ctr);
    return hipGetLastError();
}

hipError_t launch_cond_count(const ProdGraph &g, const uint32_t *scc, uint32_t *size, uint32_t *indeg,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_cond_count, dim3(node_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, scc, size, indeg);
    return hipGetLastError();
}

hipError_t launch_cond_seed(uint32_t n, uint32_t P, const uint32_t *starts, uint32_t n_starts, const uint32_t *scc,
                            uint64_t *R, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_seed, dim3(node_grid((uint64_t)n * n_starts)), dim3(kBlock), 0, s, n, P, starts,
                       n_starts, scc, R);
    return hipGetLastError();
}

hipError_t launch_cond_roots(uint32_t N, const uint32_t *scc, const uint32_t *indeg, uint32_t *lev,
                             unsigned long long *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_roots, dim3(node_grid(N)), dim3(kBlock), 0, s, N, scc, indeg, lev, ctr);
    return hipGetLastError();
}

hipError_t launch_cond_level(const ProdGraph &g, uint32_t P, uint32_t Pn, const uint32_t *scc, const uint32_t *size,
                             uint32_t *indeg, uint32_t *lev, uint64_t *R, uint32_t L,
                             const unsigned long long *ctr_prev, unsigned long long *ctr_next,
                             unsigned long long *ctr_clear, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_level, dim3(wave_grid((uint64_t)g.nQ * g.n)), dim3(kBlock), 0, s, g, P, Pn, scc, size,
                       indeg, lev, R, L, ctr_prev, ctr_next, ctr_clear);
    return hipGetLastError();
}

hipError_t launch_cond_expand(uint32_t N, uint32_t P, uint32_t Pn, const uint32_t *scc, uint64_t *T, hipStream_t s) {
    hipLaunchKernelGGL(k_cond_expand, dim3(wave_grid(N)), dim3(kBlock), 0, s, N, P, Pn, scc, T);
    return hipGetLastError();
}

}  // namespace cfpq
