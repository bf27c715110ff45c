// Literal per-edge incremental closure (Sec. 3.1.1, application of the
// dynamic transitive closure): the closure C of the whole product graph is
// kept as one bitset row per product node, and every new product edge is
// added on its own, as in Ibaraki and Katoh's insertion:
//
//   add (i, j):  for every node u with u = i or C[u][i], and not C[u][j]:
//                    C[u] |= C*[j]          (C*[j] = C[j] with j itself)
//
// which is the paper's word-parallel "new bits" step (only 0 AND 1 gives 1)
// applied to whole rows.  Iterations follow Listing 1: the new product edges
// of an iteration are the Kronecker product of the RSM with the new graph
// edges (every terminal edge and the epsilon loops in the first iteration,
// the previous write-back's nonterminal edges after that), each added in
// turn; then the write-back takes every pair (u, v) with C[(q_N^0, u)] holding
// (f, v), f final in box N.
//
// One workgroup runs the whole query: the edges are sequential by the
// method's nature.  Product node p = q * n + v; N = nQ * n nodes, W words per
// closure row.  The nonterminal matrices are kept by rows (row u: bits over
// v) and transposed into the library's result layout at the end.
#include "internal.h"

namespace cfpq {

constexpr int kPeBlock = 1024;

__device__ __forceinline__ bool pe_bit(const uint64_t *row, uint32_t i) { return (row[i >> 6] >> (i & 63)) & 1ull; }

// C*[j] into LDS (the snapshot every updated row reads), then every row u that
// reaches i (or is i) and not j takes it in.  Row u is only ever read and
// written by the wavefront that owns it in this step.
__device__ void pe_add(const PerEdgeQuery &Q, uint32_t i, uint32_t j, uint64_t *s_row, unsigned long long *s_grow) {
    const int lane = __lane_id();
    const uint32_t wave = threadIdx.x / kWave;
    const uint64_t *cj = Q.C + (uint64_t)j * Q.W;
    for (uint32_t k = threadIdx.x; k < Q.W; k += blockDim.x)
        s_row[k] = cj[k] | (k == (j >> 6) ? 1ull << (j & 63) : 0ull);
    __syncthreads();
    unsigned long long grew = 0;
    for (uint32_t u0 = wave * kWave; u0 < Q.N; u0 += kPeBlock) {
        const uint32_t u = u0 + (uint32_t)lane;
        bool take = false;
        if (u < Q.N) {
            const uint64_t *cu = Q.C + (uint64_t)u * Q.W;
            take = (u == i || pe_bit(cu, i)) && !pe_bit(cu, j);
        }
        for (uint64_t m = __ballot(take); m; m &= m - 1) {
            const uint32_t t = u0 + (uint32_t)(__ffsll((unsigned long long)m) - 1);
            uint64_t *ct = Q.C + (uint64_t)t * Q.W;
            for (uint32_t k = lane; k < Q.W; k += kWave) ct[k] |= s_row[k];
            ++grew;
        }
    }
    if (lane == 0 && grew) atomicAdd(s_grow, grew);
    __syncthreads();   // s_row is rewritten by the next edge
}

__global__ __launch_bounds__(kPeBlock) void k_peredge(PerEdgeQuery Q) {
    extern __shared__ uint64_t s_row[];   // W words
    __shared__ unsigned long long s_cnt, s_grow;
    const uint32_t tid = threadIdx.x, n = Q.n;
    // C, M and dM arrive cleared
    if (tid == 0) s_grow = 0;
    __syncthreads();
    // epsilon initialisation: loops (v, v) of nullable boxes are edges of M2^N
    // and new edges of the first iteration
    for (uint32_t b = 0; b < Q.nB; ++b) {
        if (!Q.nullable[b]) continue;
        for (uint32_t v = tid; v < n; v += blockDim.x) {
            const uint64_t o = ((uint64_t)b * n + v) * Q.Wn + (v >> 6);
            Q.M[o] |= 1ull << (v & 63);
            Q.dM[o] |= 1ull << (v & 63);
        }
    }
    __syncthreads();
    uint32_t it = 0;
    unsigned long long status = 0;
    for (;;) {
        ++it;
        if (Q.max_iters && it > Q.max_iters) {
            status = 1;
            break;
        }
        // the new product edges of this iteration, one at a time, in a fixed
        // order (every thread walks the same lists, so the steps are uniform)
        for (uint32_t t = 0; t < Q.n_trans; ++t) {
            const uint32_t s = Q.t_src[t], sym = Q.t_sym[t], f = Q.t_dst[t];
            if (sym < Q.n_terms) {
                if (it != 1) continue;
                for (uint32_t a = 0; a < n; ++a) {
                    const uint32_t e0 = Q.soff[(uint64_t)sym * (n + 1) + a], e1 = Q.soff[(uint64_t)sym * (n + 1) + a + 1];
                    for (uint32_t e = e0; e < e1; ++e)
                        pe_add(Q, s * n + a, f * n + Q.sidx[e], s_row, &s_grow);
                }
            } else {
                const uint32_t b = sym - Q.n_terms;
                for (uint32_t a = 0; a < n; ++a) {
                    const uint64_t *dm = Q.dM + ((uint64_t)b * n + a) * Q.Wn;
                    for (uint32_t k = 0; k < Q.Wn; ++k) {
                        // every thread reads the same word: the edges are uniform
                        for (uint64_t bits = dm[k]; bits; bits &= bits - 1) {
                            const uint32_t v = k * 64 + (uint32_t)(__ffsll((unsigned long long)bits) - 1);
                            pe_add(Q, s * n + a, f * n + v, s_row, &s_grow);
                        }
                    }
                }
            }
        }
        // write-back: (u, v) with (q_N^0, u) reaching (f, v), f final in N
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        unsigned long long cnt = 0;
        for (uint64_t r = tid; r < (uint64_t)Q.nB * n; r += blockDim.x) {
            const uint32_t b = (uint32_t)(r / n), u = (uint32_t)(r % n);
            const uint64_t *cu = Q.C + ((uint64_t)Q.starts[b] * n + u) * Q.W;
            uint64_t *mrow = Q.M + r * Q.Wn, *drow = Q.dM + r * Q.Wn;
            for (uint32_t k = 0; k < Q.Wn; ++k) {
                uint64_t acc = 0;
                for (uint32_t fi = Q.fin_off[b]; fi < Q.fin_off[b + 1]; ++fi) {
                    // bits f * n + 64 k .. f * n + 64 k + 63 of the closure row
                    const uint64_t bit0 = (uint64_t)Q.fin[fi] * n + (uint64_t)k * 64;
                    const uint64_t w = bit0 >> 6, sh = bit0 & 63;
                    uint64_t x = cu[w] >> sh;
                    if (sh && w + 1 < Q.W) x |= cu[w + 1] << (64 - sh);
                    acc |= x;
                }
                const uint32_t hi = n - k * 64;
                if (hi < 64) acc &= (1ull << hi) - 1;
                const uint64_t nw = acc & ~mrow[k];
                mrow[k] |= nw;
                drow[k] = nw;
                cnt += (unsigned long long)__popcll(nw);
            }
        }
        if (cnt) atomicAdd(&s_cnt, cnt);
        __syncthreads();
        const unsigned long long delta = s_cnt;
        if (tid == 0 && it - 1 < Q.stats_cap) Q.stats[3 + it - 1] = delta;
        __syncthreads();
        if (delta == 0) break;
    }
    if (tid == 0) {
        Q.stats[0] = it;
        Q.stats[1] = status;
        Q.stats[2] = s_grow;
    }
}

hipError_t launch_peredge(const PerEdgeQuery &q, hipStream_t s) {
    hipLaunchKernelGGL(k_peredge, dim3(1), dim3(kPeBlock), (size_t)q.W * 8, s, q);
    return hipGetLastError();
}

}  // namespace cfpq
