// Device kernels of the Kronecker-product fixpoint (Sec. 3.1, Listing 1) for
// gfx950.  Layout and buffer roles are described in internal.h.
//
// The Kronecker product M1 (x) M2 is never materialised (Sec. 2.4: block
// (s, f) of the product is the OR of M2^x over the transitions (s, x, f)).
// A closure launch therefore walks, for every target product row (f, v),
// the incoming transitions (s, x, f) of state f and the predecessors y of v
// under x, and ORs the source bitsets of rows (s, y).  Because a row is a
// bitset over source vertices, one 64-bit word carries 64 closure rows of
// the paper's C3 at once, and a wavefront handles 64 consecutive words of a
// row with one coalesced 512-byte load per predecessor.
#include "internal.h"

namespace cfpq {

constexpr int kChunks = 8;   // 64-word chunks per pass over a source tile

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int j) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int o) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// ctr_k += the workgroup's sum of v_k, k < 3 (null counters are skipped;
// every thread of a kBlock-thread workgroup calls it): one atomic per counter
// and workgroup, since atomics on one address from thousands of wavefronts
// serialise
__device__ __forceinline__ void block_add(unsigned long long *c0, unsigned long long v0,
                                          unsigned long long *c1 = nullptr, unsigned long long v1 = 0,
                                          unsigned long long *c2 = nullptr, unsigned long long v2 = 0) {
    __shared__ unsigned long long s_part[3][kBlock / kWave];
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    v2 = wave_sum(v2);
    const uint32_t w = threadIdx.x / kWave;
    if (__lane_id() == 0) {
        s_part[0][w] = v0;
        s_part[1][w] = v1;
        s_part[2][w] = v2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long t = 0;
#pragma unroll
        for (int k = 0; k < kBlock / kWave; ++k) t += s_part[threadIdx.x][k];
        unsigned long long *c = threadIdx.x == 0 ? c0 : (threadIdx.x == 1 ? c1 : c2);
        if (t && c) atomicAdd(c, t);
    }
}

__device__ __forceinline__ bool test_bit(const uint64_t *bits, uint32_t i) {
    return (bits[i >> 6] >> (i & 63)) & 1ull;
}

// Row v of state f became active: its word's bit in the coarse activity
// array blk ([nQ][Pbs], see GatherArgs) and the state's any-word.  Each is
// read first and written only if not yet set, so the many rows of one block
// or state do not all meet on one address.
__device__ __forceinline__ void mark_blk(uint64_t *blk, uint32_t Pbs, uint32_t f, uint32_t v) {
    uint64_t *b = blk + (uint64_t)f * Pbs;
    const uint32_t w = v >> 6;
    const uint64_t bit = 1ull << (w & 63);
    if (!(__hip_atomic_load(&b[w >> 6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit))
        atomicOr((unsigned long long *)&b[w >> 6], bit);
    if (!__hip_atomic_load(&b[Pbs - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        __hip_atomic_store(&b[Pbs - 1], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whether state s may have an active source row (no coarse array: yes).
__device__ __forceinline__ bool state_live(const GatherArgs &a, uint32_t s) {
    return !a.src_blk || a.src_blk[(uint64_t)s * a.Pbs + a.Pbs - 1] != 0;
}

// SplitMix64 output function (Steele, Lea, Flood 2014): the generator's first
// output for seed x.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// simple fills / setup
// ---------------------------------------------------------------------------
__global__ void k_fill(uint64_t *p, uint64_t words, uint64_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_fill_u8(uint8_t *p, uint64_t bytes) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// minimum wavefronts per SIMD the closure kernels are compiled for (their
// VGPR budget: 512 / waves); 1 leaves the compiler's choice
#ifndef CFPQ_NT_SPARSE_MIN_WAVES
#define CFPQ_NT_SPARSE_MIN_WAVES 1
#endif
#ifndef CFPQ_GATHER_MIN_WAVES
#define CFPQ_GATHER_MIN_WAVES 1
#endif
#ifndef CFPQ_WB_MIN_WAVES
#define CFPQ_WB_MIN_WAVES 1
#endif

static uint32_t grid_for(uint64_t items, uint32_t block = kBlock, uint32_t cap = 8192) {
    uint64_t g = (items + block - 1) / block;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

hipError_t launch_fill(uint64_t *p, uint64_t words, uint64_t value, hipStream_t s) {
    if (!words) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(words)), dim3(kBlock), 0, s, p, words, value);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint64_t bytes, hipStream_t s) {
    if (!bytes) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(bytes)), dim3(kBlock), 0, s, p, bytes);
    return hipGetLastError();
}

// Box-start rows hold the trivial source bit: (q_N^0, v) is where the search
// from source v starts.  T rows of states[i] get bit v in row v.
__device__ void seed_diag_body(uint64_t *T, uint64_t *tnz, uint32_t n, uint32_t P, uint32_t Pn,
                               const uint32_t *states, uint32_t n_states, uint64_t tid,
                               uint64_t nthreads, const uint64_t *mask = nullptr) {
    for (uint64_t i = tid; i < (uint64_t)n_states * n; i += nthreads) {
        uint32_t s = states[i / n], v = (uint32_t)(i % n);
        if (mask && !test_bit(mask, v)) continue;
        T[((uint64_t)s * n + v) * P + (v >> 6)] |= 1ull << (v & 63);
    }
    for (uint64_t i = tid; i < (uint64_t)n_states * Pn; i += nthreads) {
        uint32_t s = states[i / Pn], k = (uint32_t)(i % Pn);
        uint32_t hi = n - k * 64;
        const uint64_t m = mask ? mask[k] : ~0ull;   // mask bits past n are clear
        tnz[(uint64_t)s * Pn + k] = (hi >= 64 ? ~0ull : ((1ull << hi) - 1)) & m;
    }
}

__global__ void k_seed_diag(uint64_t *T, uint64_t *tnz, uint32_t n, uint32_t P, uint32_t Pn,
                            const uint32_t *states, uint32_t n_states, const uint64_t *mask) {
    seed_diag_body(T, tnz, n, P, Pn, states, n_states,
                   (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                   (uint64_t)gridDim.x * blockDim.x, mask);
}

hipError_t launch_seed_diag(uint64_t *T, uint64_t *tnz, uint32_t n, uint32_t P, uint32_t Pn,
                            const uint32_t *states, uint32_t n_states, const uint64_t *mask, hipStream_t s) {
    if (!n_states) return hipSuccess;
    hipLaunchKernelGGL(k_seed_diag, dim3(grid_for((uint64_t)n_states * n)), dim3(kBlock), 0, s, T,
                       tnz, n, P, Pn, states, n_states, mask);
    return hipGetLastError();
}

__global__ void k_mask_rows(uint64_t *rows, uint32_t n, uint32_t P, uint32_t Pn, const uint64_t *src,
                            const uint64_t *dst) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)n * Pn;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)(i / Pn), w = (uint32_t)(i % Pn);
        uint64_t &x = rows[(uint64_t)v * P + w];
        if (dst && !test_bit(dst, v)) x = 0;
        else if (src) x &= src[w];
    }
}

__global__ __launch_bounds__(kBlock) void k_row_summary(const uint64_t *rows, uint32_t nB, uint32_t n, uint32_t P,
                                                        uint32_t Pn, const uint64_t *act, uint64_t *sum,
                                                        uint32_t sum_pitch) {
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t r = wave; r < (uint64_t)nB * n; r += nwaves) {
        const uint32_t N = (uint32_t)(r / n), v = (uint32_t)(r % n);
        if (!test_bit(act + (uint64_t)N * Pn, v)) continue;
        const uint64_t *row = rows + r * P;
        for (uint32_t k0 = 0; k0 < Pn; k0 += kWave) {
            const uint32_t k = k0 + (uint32_t)lane;
            const uint64_t m = __ballot(k < Pn && row[k] != 0);
            if (lane == 0) sum[r * sum_pitch + k0 / kWave] = m;
        }
    }
}

hipError_t launch_row_summary(const uint64_t *rows, uint32_t nB, uint32_t n, uint32_t P, uint32_t Pn,
                              const uint64_t *act, uint64_t *sum, uint32_t sum_pitch, hipStream_t s) {
    hipLaunchKernelGGL(k_row_summary, dim3(grid_for((uint64_t)nB * n * kWave)), dim3(kBlock), 0, s, rows, nB, n, P, Pn,
                       act, sum, sum_pitch);
    return hipGetLastError();
}

hipError_t launch_mask_rows(uint64_t *rows, uint32_t n, uint32_t P, uint32_t Pn, const uint64_t *src,
                            const uint64_t *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_rows, dim3(grid_for((uint64_t)n * Pn)), dim3(kBlock), 0, s, rows, n, P, Pn, src, dst);
    return hipGetLastError();
}

// Epsilon initialisation (Listing 1, before the loop): a box whose initial
// state is final derives the empty word, so M2^N gets every loop (v, v); the
// loops are also this iteration's new edges A2^N.
__device__ void eps_body(uint64_t *NT, uint64_t *dNT, uint64_t *dnt_act, uint8_t *rank,
                         uint32_t n, uint32_t P, uint32_t Pn, const uint32_t *boxes, uint32_t nb,
                         uint64_t tid, uint64_t nthreads) {
    for (uint64_t i = tid; i < (uint64_t)nb * n; i += nthreads) {
        uint32_t b = boxes[i / n], v = (uint32_t)(i % n);
        uint64_t off = ((uint64_t)b * n + v) * P + (v >> 6);
        NT[off] |= 1ull << (v & 63);
        dNT[off] |= 1ull << (v & 63);
        if (rank) rank[((uint64_t)b * n + v) * n + v] = 0;
    }
    for (uint64_t i = tid; i < (uint64_t)nb * Pn; i += nthreads) {
        uint32_t b = boxes[i / Pn], k = (uint32_t)(i % Pn);
        uint32_t hi = n - k * 64;
        dnt_act[(uint64_t)b * Pn + k] = hi >= 64 ? ~0ull : ((1ull << hi) - 1);
    }
}

__global__ void k_eps(uint64_t *NT, uint64_t *dNT, uint64_t *dnt_act, uint8_t *rank, uint32_t n,
                      uint32_t P, uint32_t Pn, const uint32_t *boxes, uint32_t nb) {
    eps_body(NT, dNT, dnt_act, rank, n, P, Pn, boxes, nb,
             (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x);
}

hipError_t launch_eps(uint64_t *NT, uint64_t *dNT, uint64_t *dnt_act, uint8_t *rank, uint32_t n,
                      uint32_t P, uint32_t Pn, const uint32_t *boxes, uint32_t nb, hipStream_t s) {
    if (!nb) return hipSuccess;
    hipLaunchKernelGGL(k_eps, dim3(grid_for((uint64_t)nb * n)), dim3(kBlock), 0, s, NT, dNT,
                       dnt_act, rank, n, P, Pn, boxes, nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// closure row: the core of both the Kronecker seeding and a closure level
// ---------------------------------------------------------------------------
// by: bytes this lane read (profiling count)
__device__ __forceinline__ void or_row(uint64_t (&acc)[kChunks], const uint64_t *row,
                                       uint32_t pass0, uint32_t gw, int lane, unsigned long long &by) {
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        uint32_t w = pass0 + c * kWave + lane;
        if (w < gw) {
            acc[c] |= row[c * kWave + lane];
            by += 8;
        }
    }
}

// One wavefront computes the new source bits of product row (f, v) over the
// source tile of a.  SEED: the OR runs over the new graph edges only (the
// Kronecker product with A2: every graph edge in the first iteration, the
// previous write-back's dNT afterwards) and takes whole closure rows T as
// the rows that now reach further.  LEVEL: the OR runs over all edges (the
// current M2) and takes the frontier rows D of the previous level.  Either
// way the result, masked by what T already holds, is the "custom AND" of
// Sec. 3.1.1 (0 AND 1 = 1, else 0): exactly the bits that are new.
// Returns (wave-uniformly) whether the row gained a bit; adds the number of
// new bits to cnt (per lane); fed tells whether any source row fed the row.
template <bool SEED>
__device__ bool gather_row(const GatherArgs &a, uint32_t f, uint32_t v, unsigned long long &cnt,
                           bool &fed, unsigned long long &by, uint64_t &blocks) {
    const int lane = __lane_id();
    const uint32_t tb = a.in_off[f], te = a.in_off[f + 1];
    fed = false;
    blocks = 0;   // the T blocks that gained bits (wave-uniform)
    if (tb == te) return false;
    bool row_new = false;
    for (uint32_t pass0 = 0; pass0 < a.gw; pass0 += kChunks * kWave) {
        uint64_t acc[kChunks];
#pragma unroll
        for (int c = 0; c < kChunks; ++c) acc[c] = 0;
        for (uint32_t t = tb; t < te; ++t) {
            const InTrans tr = a.in_tr[t];
            const uint64_t *rows = a.src + (uint64_t)tr.src * a.n * a.src_pitch + a.src_off + pass0;
            const uint64_t *sact = a.src_act + (uint64_t)tr.src * a.Pn;
            if (!state_live(a, tr.src)) continue;   // no active row in the source state
            if (tr.sym < a.n_terms) {
                if (SEED && !a.seed_terms) continue;
                const uint32_t *op = a.goff + (uint64_t)tr.sym * (a.n + 1) + v;
                const uint32_t b = op[0], e = op[1];
                for (uint32_t base = b; base < e; base += kWave) {
                    uint32_t x = 0;
                    bool ok = false;
                    if (base + lane < e) {
                        x = a.gidx[base + lane];
                        ok = test_bit(sact, x);
                    }
                    uint64_t m = __ballot(ok);
                    fed |= (m != 0);
                    while (m) {
                        const int j = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        const uint32_t xj = (uint32_t)__builtin_amdgcn_readlane((int)x, j);
                        or_row(acc, rows + (uint64_t)xj * a.src_pitch, pass0, a.gw, lane, by);
                    }
                }
            } else {
                if (a.extra) continue;  // done by the sparse or matrix-core product, OR-ed in below
                const uint32_t N = tr.sym - a.n_terms;
                if (SEED && !test_bit(a.sel_act + (uint64_t)N * a.Pn, v)) continue;
                const uint64_t *sel = a.sel + ((uint64_t)N * a.n + v) * a.P;
                const uint64_t *ssum = a.sel_sum ? a.sel_sum + ((uint64_t)N * a.n + v) * a.sum_pitch : nullptr;
                const uint64_t *sblk = a.src_blk ? a.src_blk + (uint64_t)tr.src * a.Pbs : nullptr;
                for (uint32_t k0 = 0; k0 < a.Pn; k0 += kWave) {
                    const uint32_t k = k0 + lane;
                    // 64 words at once: only where the selector row and the
                    // source activity may both be non-zero
                    uint64_t live = ssum ? ssum[k0 / kWave] : ~0ull;
                    if (sblk) live &= sblk[k0 / kWave];
                    if (!live) continue;
                    uint64_t wb = 0;
                    if (k < a.Pn && ((live >> lane) & 1ull)) {
                        // activity and selector words loaded together (one
                        // round trip; the summaries already say both may be
                        // non-zero)
                        const uint64_t sa = sact[k], sv = sel[k];
                        wb = sv & sa;
                    }
                    uint64_t m = __ballot(wb != 0);
                    fed |= (m != 0);
                    while (m) {
                        const int j = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        uint64_t bits = readlane64(wb, j);
                        while (bits) {
                            const int bb = __ffsll((unsigned long long)bits) - 1;
                            bits &= bits - 1;
                            const uint32_t xj = (k0 + (uint32_t)j) * 64u + (uint32_t)bb;
                            or_row(acc, rows + (uint64_t)xj * a.src_pitch, pass0, a.gw, lane, by);
                        }
                    }
                }
            }
        }
        // the product row of (f, v), or of its class representative
        uint32_t vx = v;
        if (SEED && a.rep) {
            const uint32_t Nf = a.f_box[f];
            if (Nf != kNoBox && test_bit(a.sel_act + (uint64_t)Nf * a.Pn, v)) vx = a.rep[(uint64_t)Nf * a.n + v];
        }
        if (a.extra && test_bit(a.extra_act + (uint64_t)f * a.Pn, vx)) {
            fed = true;
            or_row(acc, a.extra + ((uint64_t)f * a.n + vx) * a.G + pass0, pass0, a.gw, lane, by);
        }
        if (!fed) return false;  // no source row feeds (f, v): same in every pass
        uint64_t *trow = a.T + ((uint64_t)f * a.n + v) * a.P + a.w0 + pass0;
        uint64_t *drow = a.dn + ((uint64_t)f * a.n + v) * a.G + pass0;
        bool any = false;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const uint32_t w = pass0 + c * kWave + lane;
            uint64_t nw = 0;
            if (w < a.gw) {
                const uint64_t t = trow[c * kWave + lane];
                nw = acc[c] & ~t;
                if (nw) {
                    trow[c * kWave + lane] = t | nw;
                    any = true;
                    cnt += (unsigned long long)__popcll(nw);
                }
                drow[c * kWave + lane] = nw;
                by += nw ? 24 : 16;   // T read, frontier written, T written if it grew
            }
            if (a.chgb) {
                // the blocks of the chunk's words that grew (a chunk of 64
                // words meets at most two blocks): wave-uniform
                const uint64_t bal = __ballot(nw != 0);
                if (bal) {
                    const uint32_t base = a.w0 + pass0 + (uint32_t)c * kWave;
                    const uint32_t b0 = base >> a.blk_shift, b1 = (base + kWave - 1) >> a.blk_shift;
                    const uint64_t lo = b0 == b1 ? ~0ull : (1ull << ((b1 << a.blk_shift) - base)) - 1ull;
                    if (bal & lo) blocks |= 1ull << (b0 & 63u);
                    if (bal & ~lo) blocks |= 1ull << (b1 & 63u);
                }
            }
        }
        row_new |= (__ballot(any) != 0);
    }
    return row_new;
}

// ---------------------------------------------------------------------------
// sparse nonterminal product (Kronecker seed and closure levels): when the
// source rows hold few bits in the tile (closure rows after one inverse
// edge, frontier rows), OR-ing whole rows per selector bit wastes a row of
// loads per bit.  The rows are listed instead (ELL: up to kEll set-bit
// positions per row, denser rows flagged), and each target row gathers the
// listed bits of its selected predecessors into an LDS row accumulator.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x) {
    const int lane = __lane_id();
    uint32_t incl = x;
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += y;
    }
    return incl - x;
}

// one wavefront per (source state, row x): list the set bits of the tile
__global__ __launch_bounds__(kBlock) void k_ell_build(const uint64_t *rows, uint32_t pitch, uint32_t off, uint32_t gw,
                                                      uint32_t n, const uint32_t *states, uint32_t n_states,
                                                      uint32_t *ell_cnt, uint32_t *ell_idx, const uint64_t *act,
                                                      uint32_t Pn, const unsigned long long *ctr_prev,
                                                      unsigned long long *bytes_ctr, uint64_t *dns, uint64_t *dblk,
                                                      uint32_t Pbs) {
    if (ctr_prev && *ctr_prev == 0) return;  // the frontier ran dry
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long by = 0;   // profiling: bytes read and written by this lane
    for (uint64_t r = wave; r < (uint64_t)n_states * n; r += nwaves) {
        const uint32_t s = states[r / n], x = (uint32_t)(r % n);
        // rows marked inactive are never looked up (the product tests the
        // same activity bit first)
        if (act && !test_bit(act + (uint64_t)s * Pn, x)) continue;
        const uint64_t *row = rows + ((uint64_t)s * n + x) * pitch + off;
        uint32_t mine = 0;
        uint64_t bmask = 0;   // bit c: words [64 c, 64 c + 64) of the row's tile hold a bit
        for (uint32_t c = 0, w = lane; c * kWave < gw; ++c, w += kWave) {
            const uint64_t x_w = w < gw ? row[w] : 0ull;
            mine += (uint32_t)__popcll(x_w);
            if (__ballot(x_w != 0)) bmask |= 1ull << (c & 63);
            by += w < gw ? 8 : 0;
        }
        uint32_t total = mine;
        for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o, kWave);
        const uint64_t cell = (uint64_t)s * n + x;
        by += 4ull * mine + (lane == 0 ? 4 : 0);
        if (total > kEll) {
            if (lane == 0) {
                const bool blocked = dns != nullptr;
                ell_cnt[cell] = blocked ? kEllBlocked : kEllDense;
                if (blocked) {
                    atomicOr((unsigned long long *)&dns[(uint64_t)s * Pn + (x >> 6)], 1ull << (x & 63));
                    mark_blk(dblk, Pbs, s, x);
                    // a dense row's list holds its block mask instead (two
                    // 32-bit entries)
                    ell_idx[cell * kEll] = (uint32_t)bmask;
                    ell_idx[cell * kEll + 1] = (uint32_t)(bmask >> 32);
                }
            }
            continue;
        }
        uint32_t at = wave_excl_scan(mine);
        for (uint32_t w = lane; w < gw && mine; w += kWave) {
            uint64_t b = row[w];
            while (b) {
                const int i = __ffsll((unsigned long long)b) - 1;
                b &= b - 1;
                ell_idx[cell * kEll + at++] = w * 64 + (uint32_t)i;
                --mine;
            }
        }
        if (lane == 0) ell_cnt[cell] = total;
    }
    if (bytes_ctr) {
        by = wave_sum(by);
        if (lane == 0 && by) atomicAdd(bytes_ctr, by);
    }
}

// one wavefront per target row (f, v): OR over every nonterminal transition
// (s, N, f) and every selected edge (x, v) of N (seed: the new edges, dNT
// row v; levels: all of M2^N) of the live source row (s, x): listed rows bit
// by bit into an LDS accumulator of gw words, dense rows whole into
// registers; the result goes to extra[(f, v)]
__global__ __launch_bounds__(kBlock, CFPQ_NT_SPARSE_MIN_WAVES) void k_nt_sparse(GatherArgs a, const uint32_t *ell_cnt,
                                                       const uint32_t *ell_idx, uint64_t *extra,
                                                       uint64_t *extra_act) {
    if (a.slot_prev != kNoSlot && a.ctr[(uint64_t)a.slot_prev * kSlotWords] == 0) return;  // frontier ran dry
    extern __shared__ unsigned long long lds_acc[];
    const int lane = __lane_id();
    const uint32_t wib = threadIdx.x >> 6;
    unsigned long long *acc = lds_acc + (uint64_t)wib * a.gw;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    // dense rows (more set bits than an ELL list holds) are ORed into
    // registers, kDenseRegs words per lane (the first kDenseRegs * 64 words
    // of the tile; the rest through LDS), kDenseRows rows per step so that
    // their loads are in flight together
#ifndef CFPQ_DENSE_REGS
#define CFPQ_DENSE_REGS 8
#endif
    constexpr int kDenseRegs = CFPQ_DENSE_REGS;
#ifndef CFPQ_DENSE_ROWS
#define CFPQ_DENSE_ROWS 2
#endif
    constexpr int kDenseRows = CFPQ_DENSE_ROWS;   // rows in flight per step (tuning parameter)
    const uint32_t gw_reg = a.gw < kDenseRegs * kWave ? a.gw : kDenseRegs * kWave;
    // profiling: bytes of the words this wavefront reads and writes (per lane)
    unsigned long long by = 0;
    for (uint64_t r = wave; r < (uint64_t)a.nQ * a.n; r += nwaves) {
        const uint32_t f = (uint32_t)(r / a.n), v = (uint32_t)(r % a.n);
        bool cleared = false, any = false;
        uint64_t dacc[kDenseRegs];
#pragma unroll
        for (int q = 0; q < kDenseRegs; ++q) dacc[q] = 0;
        for (uint32_t t = a.in_off[f]; t < a.in_off[f + 1]; ++t) {
            const InTrans tr = a.in_tr[t];
            if (tr.sym < a.n_terms) continue;
            const uint32_t N = tr.sym - a.n_terms;
            if (!state_live(a, tr.src)) continue;   // no active row in the source state
            if (a.sel_act && !test_bit(a.sel_act + (uint64_t)N * a.Pn, v)) continue;
            // another row of the same selector class computes this product
            if (a.rep && a.f_box[f] == N && a.rep[(uint64_t)N * a.n + v] != v) continue;
            const uint64_t *sel = a.sel + ((uint64_t)N * a.n + v) * a.P;
            const uint64_t *sact = a.src_act + (uint64_t)tr.src * a.Pn;
            const uint64_t *ssum = a.sel_sum ? a.sel_sum + ((uint64_t)N * a.n + v) * a.sum_pitch : nullptr;
            const uint64_t *sblk = a.src_blk ? a.src_blk + (uint64_t)tr.src * a.Pbs : nullptr;
            for (uint32_t k0 = 0; k0 < a.Pn; k0 += kWave) {
                const uint32_t k = k0 + lane;
                // with a summary of the selector row and the coarse source
                // activity, only words where both may be non-zero are read
                uint64_t live = ssum ? ssum[k0 / kWave] : ~0ull;
                if (sblk) live &= sblk[k0 / kWave];
                if (!live) continue;
                uint64_t wb = 0;
                if (k < a.Pn && ((live >> lane) & 1ull)) {
                    // activity and selector words loaded together (one round
                    // trip; the summaries already say both may be non-zero)
                    const uint64_t sa = sact[k], sv = sel[k];
                    wb = sv & sa;
                    by += 16;
                }
                uint64_t m = __ballot(wb != 0);
                if (m && !cleared) {
                    for (uint32_t w = lane; w < a.gw; w += kWave) acc[w] = 0;
                    cleared = true;
                    __builtin_amdgcn_wave_barrier();
                }
                while (m) {
                    const int j = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1;
                    // the set bits of one selector word at once, lane i taking
                    // source row 64 (k0 + j) + i: its ELL entries go to the
                    // accumulator by LDS atomics; dense rows are ORed whole by
                    // the wave afterwards, one at a time
                    const uint64_t bits = readlane64(wb, j);
                    const uint32_t xb = (k0 + (uint32_t)j) * 64u;
                    const bool mine = (bits >> lane) & 1ull;
                    const uint64_t cell = (uint64_t)tr.src * a.n + xb + (uint32_t)lane;
                    // the count and the list's first four entries are loaded
                    // together (one memory round trip for short lists); the
                    // lists are 128-byte aligned, 16 bytes per load
                    const uint4 *idx4 = reinterpret_cast<const uint4 *>(ell_idx + cell * kEll);
                    uint32_t cnt = 0;
                    uint4 e0 = make_uint4(0, 0, 0, 0);
                    if (mine) {
                        cnt = ell_cnt[cell];
                        e0 = idx4[0];
                    }
                    // rows beyond an ELL list: ORed whole here, unless they are
                    // left to the blocked dense product
                    const bool dense = cnt == kEllDense || (cnt == kEllBlocked && !a.dense_apart);
                    const bool apart = cnt == kEllBlocked && a.dense_apart;
                    if (!dense && !apart && cnt) {
                        auto put = [&](uint32_t u) { atomicOr(&acc[u >> 6], 1ull << (u & 63)); };
                        put(e0.x);
                        if (cnt > 1) put(e0.y);
                        if (cnt > 2) put(e0.z);
                        if (cnt > 3) put(e0.w);
                        // the rest eight entries per step, both loads in flight
                        for (uint32_t e = 4; e < cnt; e += 8) {
                            const uint4 p = idx4[e / 4];
                            const uint4 q = e + 4 < cnt ? idx4[e / 4 + 1] : make_uint4(0, 0, 0, 0);
                            const uint32_t v8[8] = {p.x, p.y, p.z, p.w, q.x, q.y, q.z, q.w};
#pragma unroll
                            for (uint32_t i = 0; i < 8; ++i)
                                if (e + i < cnt) put(v8[i]);
                        }
                    }
                    if (mine) by += 4ull * (1 + (dense || apart ? 0u : cnt));
                    uint64_t dm = __ballot(dense);
                    if (lane == 0) by += 8ull * a.gw * (uint64_t)__popcll(dm);
                    const uint64_t *rbase = a.src + ((uint64_t)tr.src * a.n + xb) * a.src_pitch + a.src_off;
                    while (dm) {
                        const uint64_t *rr[kDenseRows];
#pragma unroll
                        for (int q = 0; q < kDenseRows; ++q) {
                            // fewer rows left: repeat the first (OR is idempotent)
                            const uint32_t d = dm ? (uint32_t)(__ffsll((unsigned long long)dm) - 1) : 0u;
                            rr[q] = dm ? rbase + (uint64_t)d * a.src_pitch : rr[0];
                            dm &= dm - 1;
                        }
#pragma unroll
                        for (int q = 0; q < kDenseRegs; ++q) {
                            const uint32_t w = (uint32_t)(q * kWave + lane);
                            if (w < gw_reg) {
                                uint64_t x = 0;
#pragma unroll
                                for (int i = 0; i < kDenseRows; ++i) x |= rr[i][w];
                                dacc[q] |= x;
                            }
                        }
                        for (uint32_t w = gw_reg + lane; w < a.gw; w += kWave) {
                            uint64_t x = 0;
#pragma unroll
                            for (int i = 0; i < kDenseRows; ++i) x |= rr[i][w];
                            acc[w] |= x;
                        }
                    }
                    any = true;
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
        if (!any) continue;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < kDenseRegs; ++q) {
            const uint32_t w = (uint32_t)(q * kWave + lane);
            if (w < gw_reg) acc[w] |= dacc[q];
        }
        __builtin_amdgcn_wave_barrier();
        uint64_t *out = extra + ((uint64_t)f * a.n + v) * a.G;
        bool nz = false;
        for (uint32_t w = lane; w < a.gw; w += kWave) {
            const uint64_t x = acc[w];
            out[w] = x;
            nz |= x != 0;
            by += 8;
        }
        // with dense rows apart the row is flagged even if still zero: the
        // dense product ORs into flagged rows only
        if ((a.dense_apart || __ballot(nz)) && lane == 0)
            atomicOr((unsigned long long *)&extra_act[(uint64_t)f * a.Pn + (v >> 6)], 1ull << (v & 63));
        __builtin_amdgcn_wave_barrier();
    }
    if (a.bytes_ctr) {
        by = wave_sum(by);
        if (lane == 0 && by) atomicAdd(a.bytes_ctr, by);
    }
}

hipError_t launch_ell_build(const uint64_t *rows, uint32_t pitch, uint32_t off, uint32_t gw, uint32_t n,
                            const uint32_t *states, uint32_t n_states, uint32_t *ell_cnt, uint32_t *ell_idx,
                            const uint64_t *act, uint32_t Pn, const unsigned long long *ctr_prev, hipStream_t s,
                            unsigned long long *bytes_ctr) {
    if (!n_states) return hipSuccess;
    hipLaunchKernelGGL(k_ell_build, dim3(grid_for((uint64_t)n_states * n * kWave)), dim3(kBlock), 0, s, rows, pitch,
                       off, gw, n, states, n_states, ell_cnt, ell_idx, act, Pn, ctr_prev, bytes_ctr, nullptr,
                       nullptr, 0u);
    return hipGetLastError();
}

hipError_t launch_ell_build_dense(const uint64_t *rows, uint32_t pitch, uint32_t off, uint32_t gw, uint32_t n,
                                  const uint32_t *states, uint32_t n_states, uint32_t *ell_cnt, uint32_t *ell_idx,
                                  const uint64_t *act, uint32_t Pn, const unsigned long long *ctr_prev,
                                  uint64_t *dns, uint64_t *dblk, uint32_t Pbs, hipStream_t s,
                                  unsigned long long *bytes_ctr) {
    if (!n_states) return hipSuccess;
    hipLaunchKernelGGL(k_ell_build, dim3(grid_for((uint64_t)n_states * n * kWave)), dim3(kBlock), 0, s, rows, pitch,
                       off, gw, n, states, n_states, ell_cnt, ell_idx, act, Pn, ctr_prev, bytes_ctr, dns, dblk, Pbs);
    return hipGetLastError();
}

hipError_t launch_nt_sparse(const GatherArgs &a, const uint32_t *ell_cnt, const uint32_t *ell_idx, uint64_t *extra,
                            uint64_t *extra_act, uint32_t grid, hipStream_t s) {
    const size_t lds = (size_t)(kBlock / kWave) * a.gw * 8;
    hipLaunchKernelGGL(k_nt_sparse, dim3(grid), dim3(kBlock), lds, s, a, ell_cnt, ell_idx, extra, extra_act);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dense nonterminal product, blocked through LDS.  For every transition
// (s, N, f) and target row (f, v):
//   extra[f][v] |= OR over dense source rows x of s with N(x, v): src[s][x]
// A workgroup owns a task (f, 128 consecutive targets v, 64 source words):
// wavefront w holds targets 32 w .. 32 w + 31 of the block, lane i the
// source word u0 + i, one accumulator word per target.  Per word xw of the
// selector (64 source rows x), if any of the block's targets selects one of
// the dense rows there, those rows' 64-word slices are staged in LDS once
// and ORed into every target that selects them: each source word read from
// memory serves up to 128 targets instead of one.
// ---------------------------------------------------------------------------
constexpr uint32_t kDenseTargets = 128;      // target rows per workgroup
constexpr uint32_t kDenseTPW = kDenseTargets / (kBlock / kWave);   // per wavefront

__device__ __forceinline__ bool dense_live(const uint64_t *dblk, uint32_t Pbs, uint32_t s) {
    return dblk[(uint64_t)s * Pbs + Pbs - 1] != 0;
}

__global__ __launch_bounds__(kBlock) void k_nt_dense(GatherArgs a, DenseArgs d) {
    if (a.slot_prev != kNoSlot && a.ctr[(uint64_t)a.slot_prev * kSlotWords] == 0) return;  // frontier ran dry
    __shared__ uint64_t tile[64][kWave];
    __shared__ uint64_t s_rows[kBlock / kWave];
    const int lane = __lane_id();
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t nvb = (a.n + kDenseTargets - 1) / kDenseTargets, nub = (a.gw + kWave - 1) / kWave;
    const uint64_t tasks = (uint64_t)d.n_nt_dst * nvb * nub;
    unsigned long long by = 0;
    for (uint64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
        // targets fastest: consecutive workgroups share the staged source slice
        const uint32_t vb = (uint32_t)(task % nvb), ub = (uint32_t)((task / nvb) % nub);
        const uint32_t f = d.nt_dst[task / ((uint64_t)nvb * nub)];
        const uint32_t v0 = vb * kDenseTargets + w * kDenseTPW, u = ub * kWave + (uint32_t)lane;
        uint64_t acc[kDenseTPW];
#pragma unroll
        for (uint32_t t = 0; t < kDenseTPW; ++t) acc[t] = 0;
        bool touched = false;
        for (uint32_t tr_i = a.in_off[f]; tr_i < a.in_off[f + 1]; ++tr_i) {
            const InTrans tr = a.in_tr[tr_i];
            if (tr.sym < a.n_terms) continue;
            const uint32_t sst = tr.src, N = tr.sym - a.n_terms;
            if (!dense_live(d.dblk, a.Pbs, sst)) continue;   // no dense source row in state s
            // lane t < 32 of each wavefront: selector row of its target v0 + t
            const uint32_t my_v = v0 + (uint32_t)(lane & 31);
            const bool v_ok = lane < (int)kDenseTPW && my_v < a.n &&
                              (!a.sel_act || test_bit(a.sel_act + (uint64_t)N * a.Pn, my_v));
            const uint64_t *sel = a.sel + ((uint64_t)N * a.n + my_v) * a.P;
            const uint64_t *ssum = a.sel_sum ? a.sel_sum + ((uint64_t)N * a.n + my_v) * a.sum_pitch : nullptr;
            const uint64_t *dbk = d.dblk + (uint64_t)sst * a.Pbs;
            const uint64_t *dn = d.dns + (uint64_t)sst * a.Pn;
            const uint64_t *rows = a.src + (uint64_t)sst * a.n * a.src_pitch + a.src_off;
            for (uint32_t xb = 0; xb + 1 < a.Pbs; ++xb) {
                uint64_t mwb = dbk[xb];   // x-words of this group holding dense rows
                if (!mwb) continue;
                if (ssum) {
                    // only x-words some target of the block may select (from the
                    // selector rows' summaries): one word per target per group
                    uint64_t us = v_ok ? ssum[xb] : 0ull;
                    by += v_ok ? 8 : 0;
                    for (int o = 32; o > 0; o >>= 1) us |= shfl_xor64(us, o);
                    if (lane == 0) s_rows[w] = us;
                    __syncthreads();
                    uint64_t u_all = 0;
#pragma unroll
                    for (uint32_t i = 0; i < kBlock / kWave; ++i) u_all |= s_rows[i];
                    __syncthreads();   // s_rows is reused below
                    mwb &= u_all;
                }
                for (uint64_t mw = mwb; mw; mw &= mw - 1) {
                    const uint32_t xw = xb * 64 + (uint32_t)(__ffsll((unsigned long long)mw) - 1);
                    const uint64_t mx = dn[xw];   // dense source rows x = 64 xw + j
                    if (!mx) continue;
                    const uint64_t sw = v_ok ? (sel[xw] & mx) : 0ull;
                    by += v_ok ? 8 : 0;
                    // rows some target of the block selects whose slice of
                    // this workgroup's 64 source words holds a bit (block
                    // masks from the ELL build)
                    uint64_t wu = sw;
                    for (int o = 32; o > 0; o >>= 1) wu |= shfl_xor64(wu, o);
                    uint64_t mine_rows = 0;
                    if (lane < 64) {
                        const uint32_t j = (uint32_t)lane;
                        if ((wu >> j) & 1ull) {
                            const uint32_t *li = d.ell_idx + ((uint64_t)sst * a.n + xw * 64 + j) * kEll;
                            const uint64_t bm = (uint64_t)li[0] | ((uint64_t)li[1] << 32);
                            if ((bm >> (ub & 63)) & 1ull) mine_rows = 1ull << j;
                        }
                    }
                    const uint64_t wave_rows = __ballot(mine_rows != 0);
                    if (lane == 0) s_rows[w] = wave_rows;
                    __syncthreads();
                    uint64_t staged = 0;
#pragma unroll
                    for (uint32_t i = 0; i < kBlock / kWave; ++i) staged |= s_rows[i];
                    if (staged) {
                        // wavefront w stages rows j (k-th set bit of staged) with k % 4 == w
                        uint64_t rem = staged;
                        for (uint32_t k = 0; rem; ++k, rem &= rem - 1) {
                            if ((k & 3) != w) continue;
                            const uint32_t j = (uint32_t)(__ffsll((unsigned long long)rem) - 1);
                            const uint64_t *row = rows + (uint64_t)(xw * 64 + j) * a.src_pitch;
                            tile[j][lane] = u < a.gw ? row[u] : 0ull;
                            by += u < a.gw ? 8 : 0;
                        }
                        __syncthreads();
#pragma unroll
                        for (uint32_t t = 0; t < kDenseTPW; ++t) {
                            uint64_t bits = readlane64(sw, (int)t) & staged;
                            while (bits) {
                                const int j = __ffsll((unsigned long long)bits) - 1;
                                bits &= bits - 1;
                                acc[t] |= tile[j][lane];
                            }
                        }
                        touched = true;
                    }
                    __syncthreads();   // s_rows and the tile are reused
                }
            }
        }
        if (touched && u < a.gw) {
#pragma unroll
            for (uint32_t t = 0; t < kDenseTPW; ++t) {
                const uint32_t v = v0 + t;
                if (v < a.n && acc[t] && test_bit(d.extra_act + (uint64_t)f * a.Pn, v)) {
                    uint64_t *o = d.extra + ((uint64_t)f * a.n + v) * a.G + u;
                    *o |= acc[t];
                    by += 16;
                }
            }
        }
    }
    if (a.bytes_ctr) {
        by = wave_sum(by);
        if (lane == 0 && by) atomicAdd(a.bytes_ctr, by);
    }
}

hipError_t launch_nt_dense(const GatherArgs &a, const DenseArgs &d, hipStream_t s) {
    const uint64_t tasks = (uint64_t)d.n_nt_dst * ((a.n + kDenseTargets - 1) / kDenseTargets) *
                           ((a.gw + kWave - 1) / kWave);
    if (!tasks) return hipSuccess;
    const uint64_t grid = tasks < 256 * 8 ? tasks : 256 * 8;
    hipLaunchKernelGGL(k_nt_dense, dim3((uint32_t)grid), dim3(kBlock), 0, s, a, d);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dense nonterminal product on the matrix cores: for one transition (s, N, f)
//   out[v][u] = OR_x sel[v][x] AND src[x][u]
// as an exact int8 product with int32 accumulation (v_mfma_i32_32x32x32_i8:
// {0,1} operands, sums <= n < 2^31), thresholded back to bits.  A wavefront
// owns 4 x 32 target rows and one 64-bit word of sources (64 columns); per
// 64-row step of x it transposes the 64 x 64 source block with ballots (B),
// expands the selector words of its rows (A) and issues 16 MFMAs.
// Any fixed assignment of the 32 k values of an MFMA to (lane group,
// element) serves, as long as A and B use the same one: the sum runs over k.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kMfmaTiles = 4;   // 32-row tiles per wavefront

// 16 bits -> 16 bytes in {0, 1}, byte e = bit e (copies of each nibble at
// bit offsets 0, 7, 14, 21 land one bit in each byte, without carries)
__device__ __forceinline__ v4i expand16(uint32_t b) {
    v4i r;
    r[0] = (int)(((b & 0xFu) * 0x00204081u) & 0x01010101u);
    r[1] = (int)((((b >> 4) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[2] = (int)((((b >> 8) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[3] = (int)((((b >> 12) & 0xFu) * 0x00204081u) & 0x01010101u);
    return r;
}

__global__ __launch_bounds__(kBlock) void k_nt_mfma(MfmaArgs a) {
    if (a.ctr_prev && *a.ctr_prev == 0) return;  // the frontier ran dry
    const int lane = __lane_id();
    const int g = lane >> 5, col = lane & 31;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint32_t rows_per = 32 * kMfmaTiles;
    const uint64_t tasks = (uint64_t)((a.n + rows_per - 1) / rows_per) * a.gw;
    unsigned long long mfmas = 0;
    for (uint64_t task = wave; task < tasks; task += nwaves) {
        const uint32_t vb = (uint32_t)(task / a.gw) * rows_per, w = (uint32_t)(task % a.gw);
        v16i C[kMfmaTiles][2];
#pragma unroll
        for (int t = 0; t < kMfmaTiles; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c) C[t][c] = (v16i){0};
        for (uint32_t xw = 0; xw < a.Pn; ++xw) {
            const uint32_t x = xw * 64 + (uint32_t)lane;
            uint64_t b = 0;
            if (x < a.n && test_bit(a.sact, x)) b = a.src[(uint64_t)x * a.src_pitch + w];
            if (__ballot(b != 0) == 0) continue;    // no live source row in this block
            uint64_t sw[kMfmaTiles];
            bool anysel = false;
#pragma unroll
            for (int t = 0; t < kMfmaTiles; ++t) {
                const uint32_t v = vb + t * 32 + col;
                sw[t] = v < a.n ? a.sel[(uint64_t)v * a.P + xw] : 0ull;
                anysel |= sw[t] != 0;
            }
            if (__ballot(anysel) == 0) continue;    // no selector bit in this block
            // B: column j of the 64 x 64 block = ballot of bit j over the rows
            uint64_t cm0 = 0, cm1 = 0;
#pragma unroll 8
            for (int j = 0; j < 64; ++j) {
                const uint64_t m = __ballot((b >> j) & 1ull);
                if (col == (j & 31)) {
                    if (j < 32) cm0 = m;
                    else cm1 = m;
                }
            }
            const int sh = 16 * g;
            const v4i B00 = expand16((uint32_t)(cm0 >> sh) & 0xFFFFu);
            const v4i B01 = expand16((uint32_t)(cm1 >> sh) & 0xFFFFu);
            const v4i B10 = expand16((uint32_t)(cm0 >> (32 + sh)) & 0xFFFFu);
            const v4i B11 = expand16((uint32_t)(cm1 >> (32 + sh)) & 0xFFFFu);
#pragma unroll
            for (int t = 0; t < kMfmaTiles; ++t) {
                const v4i A0 = expand16((uint32_t)(sw[t] >> sh) & 0xFFFFu);
                const v4i A1 = expand16((uint32_t)(sw[t] >> (32 + sh)) & 0xFFFFu);
                C[t][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B00, C[t][0], 0, 0, 0);
                C[t][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B10, C[t][0], 0, 0, 0);
                C[t][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B01, C[t][1], 0, 0, 0);
                C[t][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B11, C[t][1], 0, 0, 0);
            }
            mfmas += 4 * kMfmaTiles;
        }
        // threshold and pack: accumulator i of lane group g holds row
        // 8*(i/4) + 4*g + i%4 of the tile, column col (+32 for the second half)
#pragma unroll
        for (int t = 0; t < kMfmaTiles; ++t) {
            uint64_t mine = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint64_t b0 = __ballot(C[t][0][i] > 0), b1 = __ballot(C[t][1][i] > 0);
                const int r0 = 8 * (i / 4) + (i % 4), r1 = r0 + 4;
                const uint64_t w0 = (b0 & 0xFFFFFFFFull) | ((b1 & 0xFFFFFFFFull) << 32);
                const uint64_t w1 = (b0 >> 32) | ((b1 >> 32) << 32);
                if (lane == r0) mine = w0;
                if (lane == r1) mine = w1;
            }
            const uint32_t v = vb + t * 32 + (uint32_t)lane;
            if (lane < 32 && v < a.n) {
                uint64_t *o = a.out + (uint64_t)v * a.G + w;
                if (a.first)
                    *o = mine;
                else if (mine)
                    atomicOr((unsigned long long *)o, mine);
                if (mine) atomicOr((unsigned long long *)&a.out_act[v >> 6], 1ull << (v & 63));
            }
        }
    }
    if (a.mfma_ctr && lane == 0 && mfmas) atomicAdd(a.mfma_ctr, mfmas);   // wave-uniform count
}

hipError_t launch_nt_mfma(const MfmaArgs &a, hipStream_t s) {
    const uint64_t tasks = (uint64_t)((a.n + 32 * kMfmaTiles - 1) / (32 * kMfmaTiles)) * a.gw;
    hipLaunchKernelGGL(k_nt_mfma, dim3(grid_for(tasks * kWave)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <bool SEED>
__global__ __launch_bounds__(kBlock, CFPQ_GATHER_MIN_WAVES) void k_gather(GatherArgs a) {
    if (a.slot_prev != kNoSlot && a.ctr[(uint64_t)a.slot_prev * kSlotWords] == 0) return;  // frontier ran dry
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gthreads = (uint64_t)gridDim.x * blockDim.x;
    if (a.act_clear)
        for (uint64_t i = gtid; i < a.clear_words; i += gthreads) a.act_clear[i] = 0;
    const int lane = __lane_id();
    const uint64_t wave = gtid >> 6, nwaves = gthreads >> 6;
    unsigned long long cnt = 0, fed_rows = 0, new_rows = 0, by = 0;
    const uint64_t rows = (uint64_t)a.nQ * a.n;
    for (uint64_t r = wave; r < rows; r += nwaves) {
        const uint32_t f = (uint32_t)(r / a.n), v = (uint32_t)(r % a.n);
        bool fed = false;
        uint64_t blocks = 0;
        if (gather_row<SEED>(a, f, v, cnt, fed, by, blocks) && lane == 0) {
            if (a.chgb && blocks) atomicOr((unsigned long long *)&a.chgb[r], (unsigned long long)blocks);
            atomicOr((unsigned long long *)&a.actn[(uint64_t)f * a.Pn + (v >> 6)], 1ull << (v & 63));
            atomicOr((unsigned long long *)&a.tnz[(uint64_t)f * a.Pn + (v >> 6)], 1ull << (v & 63));
            if (a.actn_blk) mark_blk(a.actn_blk, a.Pbs, f, v);
            if (a.chg) atomicOr((unsigned long long *)&a.chg[(uint64_t)f * a.Pn + (v >> 6)], 1ull << (v & 63));
            ++new_rows;
        }
        fed_rows += fed ? 1 : 0;
    }
    // new bits per lane; rows fed and rows gaining bits once per wavefront
    unsigned long long *c = a.ctr + (uint64_t)a.slot_cur * kSlotWords;
    block_add(&c[0], cnt, &c[1], lane == 0 ? fed_rows : 0ull, &c[2], lane == 0 ? new_rows : 0ull);
    if (a.bytes_ctr) {
        by = wave_sum(by);
        if (lane == 0 && by) atomicAdd(a.bytes_ctr, by);
    }
}

hipError_t launch_gather(const GatherArgs &a, bool seed, uint32_t grid, hipStream_t s) {
    if (seed)
        hipLaunchKernelGGL(k_gather<true>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_gather<false>, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// write-back (Listing 1, after the closure): the pairs (u, v) with a new
// closure entry from (q_N^0, u) to (f, v), f final in box N, become edges of
// M2^N; those not already present form A2^N for the next iteration.
// ---------------------------------------------------------------------------
// returns the words of the row it processed (all Pn, or those of the blocks
// it visits)
__device__ __forceinline__ uint32_t writeback_row(const WritebackArgs &a, uint32_t N, uint32_t v,
                                                  unsigned long long &cnt_box, bool &any_row) {
    const int lane = __lane_id();
    const uint32_t fb = a.fin_off[N], fe = a.fin_off[N + 1];
    uint64_t *nt = a.NT + ((uint64_t)N * a.n + v) * a.P;
    uint64_t *dnt = a.dNT ? a.dNT + ((uint64_t)N * a.n + v) * a.P : nullptr;
    bool any = false;
    unsigned long long hs = 0;   // hash of the new edges: sum over non-zero words of a mix of (word, index)
    uint64_t dblocks = 0;        // blocks of the new dNT row holding bits
    const uint32_t nch = cond_chunks(a.Pn), cwds = cond_chunk_words(a.Pn);
    // word k of the row (lanes of one 64-word group together: lane l takes
    // word 64 i + l)
    auto word = [&](uint32_t k) {
        uint64_t acc = 0;
        for (uint32_t i = fb; i < fe; ++i) {
            const uint64_t node = (uint64_t)a.fin[i] * a.n + v;
            const uint64_t row = a.row_map ? (uint64_t)a.row_map[node] : node;
            if (a.row_nz && !a.row_nz[row * nch + k / cwds])
                continue;  // chunk never written: all zero
            acc |= a.T[row * a.P + k];
        }
        const uint64_t old = a.fresh ? 0ull : nt[k];
        const uint64_t nw = acc & ~old;
        if (a.fresh) nt[k] = nw;  // M2^N was empty: write without reading
        if (nw) {
            if (!a.fresh) nt[k] = old | nw;
            any = true;
            cnt_box += (unsigned long long)__popcll(nw);
            hs += splitmix64(nw ^ ((uint64_t)k * 0x9e3779b97f4a7c15ull));
            if (a.rank) {
                uint64_t bits = nw;
                while (bits) {
                    const int b = __ffsll((unsigned long long)bits) - 1;
                    bits &= bits - 1;
                    a.rank[((uint64_t)N * a.n + (uint64_t)k * 64 + b) * a.n + v] = (uint8_t)(a.iter > 255 ? 255 : a.iter);
                }
            }
        }
        if (dnt) dnt[k] = nw;
        const uint64_t dm = __ballot(nw != 0);
        const uint32_t g = (k - (uint32_t)lane) / kWave;   // the 64-word group
        if (a.dnb && dm) dblocks |= 1ull << (((uint64_t)g * kWave / a.blk_words) & 63u);
        if (a.dsum || a.nsum) {
            // one summary word per group
            const uint64_t nm = __ballot((old | nw) != 0);
            const uint64_t so = ((uint64_t)N * a.n + v) * a.sum_pitch + g;
            if (lane == 0) {
                if (a.dsum) a.dsum[so] = dm;
                if (a.nsum) a.nsum[so] = nm;
            }
        }
    };
    uint32_t words = a.Pn;
    if (a.chgb) {
        // the blocks where a final-state row gained bits or dNT held bits
        words = 0;
        uint64_t blocks = a.dnb ? a.dnb[(uint64_t)N * a.n + v] : 0ull;
        for (uint32_t i = fb; i < fe; ++i) blocks |= a.chgb[(uint64_t)a.fin[i] * a.n + v];
        while (blocks) {
            const uint32_t b = (uint32_t)__ffsll((unsigned long long)blocks) - 1;
            blocks &= blocks - 1;
            const uint32_t k1 = (b + 1) * a.blk_words < a.Pn ? (b + 1) * a.blk_words : a.Pn;
            words += k1 - b * a.blk_words;
            for (uint32_t k0 = b * a.blk_words; k0 < k1; k0 += kWave)
                if (k0 + (uint32_t)lane < k1) word(k0 + (uint32_t)lane);
        }
    } else {
        for (uint32_t k = lane; k < a.Pn; k += kWave) word(k);
    }
    if (a.dnb && lane == 0) a.dnb[(uint64_t)N * a.n + v] = dblocks;
    any_row = __ballot(any) != 0;
    if (a.dhash && any_row) {
        hs = wave_sum(hs);
        if (lane == 0) a.dhash[(uint64_t)N * a.n + v] = hs ? hs : 1ull;
    }
    return words;
}

constexpr uint32_t kWbLdsBoxes = 64;   // boxes whose new-edge counts gather in LDS first

__global__ __launch_bounds__(kBlock, CFPQ_WB_MIN_WAVES) void k_writeback(WritebackArgs a) {
    if ((a.skip_if[0] && *a.skip_if[0]) || (a.skip_if[1] && *a.skip_if[1])) return;
    // new edges per box: summed per workgroup in LDS (rows of one box meet
    // on one counter), flushed with one atomic per box and workgroup
    __shared__ unsigned long long s_box[kWbLdsBoxes], s_rows[kWbLdsBoxes];
    const bool lds_boxes = a.nB <= kWbLdsBoxes;
    if (lds_boxes)
        for (uint32_t i = threadIdx.x; i < a.nB; i += blockDim.x) s_box[i] = s_rows[i] = 0;
    __syncthreads();
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gthreads = (uint64_t)gridDim.x * blockDim.x;
    const int lane = __lane_id();
    const uint64_t wave = gtid >> 6, nwaves = gthreads >> 6;
    const uint64_t rows = (uint64_t)a.nB * a.n;
    auto one_row = [&](uint64_t r) {
        const uint32_t N = (uint32_t)(r / a.n), v = (uint32_t)(r % a.n);
        if (a.fin_off[N] == a.fin_off[N + 1]) {
            // a box without final states derives nothing: its relation is empty
            if (a.fresh)
                for (uint32_t k = lane; k < a.Pn; k += kWave) a.NT[((uint64_t)N * a.n + v) * a.P + k] = 0;
            return;
        }
        unsigned long long c = 0;
        bool any = false;
        const uint32_t words = writeback_row(a, N, v, c, any);
        c = wave_sum(c);
        if (a.rows_ctr && lane == 0) {   // profiling: row words processed
            if (lds_boxes)
                atomicAdd(&s_rows[N], (unsigned long long)words);
            else
                atomicAdd(&a.rows_ctr[N], (unsigned long long)words);
        }
        if (lane == 0 && any) {
            if (a.dnt_act)
                atomicOr((unsigned long long *)&a.dnt_act[(uint64_t)N * a.Pn + (v >> 6)], 1ull << (v & 63));
            if (lds_boxes)
                atomicAdd(&s_box[N], c);
            else
                atomicAdd(&a.ctr[(uint64_t)(a.slot_base + N) * kSlotWords], c);
        }
    };
    if (!a.state_flags && !a.chg)
        for (uint64_t r = wave; r < rows; r += nwaves) one_row(r);
    // levels strategy: a lane per row finds the rows whose final-state closure
    // rows gained bits in this iteration or whose dNT row still holds the
    // previous iteration's edges, 64 rows at a time
    for (uint64_t r0 = wave * kWave; !a.state_flags && a.chg && r0 < rows; r0 += nwaves * kWave) {
        const uint64_t r = r0 + (uint64_t)lane;
        bool need = false;
        if (r < rows) {
            const uint32_t N = (uint32_t)(r / a.n), v = (uint32_t)(r % a.n);
            need = a.prev_act && test_bit(a.prev_act + (uint64_t)N * a.Pn, v);
            for (uint32_t i = a.fin_off[N]; !need && i < a.fin_off[N + 1]; ++i)
                need = test_bit(a.chg + (uint64_t)a.fin[i] * a.Pn, v);
        }
        for (uint64_t todo = __ballot(need); todo; todo &= todo - 1)
            one_row(r0 + (uint64_t)(__ffsll((unsigned long long)todo) - 1));
    }
    // condensed closure: most answer rows were written (and counted) by the
    // closure itself; a lane per row finds the others, 64 rows at a time
    for (uint64_t r0 = wave * kWave; a.state_flags && r0 < rows; r0 += nwaves * kWave) {
        const uint64_t r = r0 + (uint64_t)lane;
        bool need = false;
        if (r < rows) {
            const uint32_t N = (uint32_t)(r / a.n), v = (uint32_t)(r % a.n);
            need = true;
            if (a.fin_off[N] != a.fin_off[N + 1]) {
                const uint32_t f = a.fin[a.fin_off[N]];
                if ((a.state_flags[f] & kAliasFinal) && a.multi[a.row_map[(uint64_t)f * a.n + v]] == 0) need = false;
            }
        }
        for (uint64_t todo = __ballot(need); todo; todo &= todo - 1)
            one_row(r0 + (uint64_t)(__ffsll((unsigned long long)todo) - 1));
    }
    if (lds_boxes) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < a.nB; i += blockDim.x) {
            if (s_box[i]) atomicAdd(&a.ctr[(uint64_t)(a.slot_base + i) * kSlotWords], s_box[i]);
            if (a.rows_ctr && s_rows[i]) atomicAdd(&a.rows_ctr[i], s_rows[i]);
        }
    }
}

hipError_t launch_writeback(const WritebackArgs &a, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_writeback, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// seed deduplication: equal dNT rows select the same rows, so their seed
// products are equal; one representative per class computes it
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long dedup_key(uint64_t h, uint32_t N) {
    const uint64_t k = splitmix64(h + N);
    return k ? k : 1ull;   // 0 marks an empty slot
}

// a thread per row: insert the active rows' keys, each bucket keeping its
// least row index (row ids N n + v)
__global__ void k_dedup_insert(uint32_t nB, uint32_t n, uint32_t Pn, const uint64_t *act, const uint64_t *dhash,
                               unsigned long long *keys, uint32_t *vals, uint64_t mask) {
    const uint64_t rows = (uint64_t)nB * n;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t N = (uint32_t)(r / n), v = (uint32_t)(r % n);
        if (!test_bit(act + (uint64_t)N * Pn, v)) continue;
        const unsigned long long key = dedup_key(dhash[r], N);
        // linear probing; the table has at least twice as many slots as rows,
        // so an empty or matching slot is always found
        for (uint64_t slot = key & mask;; slot = (slot + 1) & mask) {
            const unsigned long long prev = atomicCAS(&keys[slot], 0ull, key);
            if (prev == 0ull || prev == key) {
                atomicMin(&vals[slot], (uint32_t)r);
                break;
            }
        }
    }
}

// a wavefront per active row: its bucket's least row, kept as representative
// only if the two rows are equal (summaries, then the words they flag)
__global__ __launch_bounds__(kBlock) void k_dedup_rep(uint32_t nB, uint32_t n, uint32_t P, uint32_t Pn,
                                                      const uint64_t *act, const uint64_t *dhash, const uint64_t *dNT,
                                                      const uint64_t *dsum, uint32_t sum_pitch,
                                                      const unsigned long long *keys, const uint32_t *vals,
                                                      uint64_t mask, uint32_t *rep) {
    const int lane = __lane_id();
    const uint64_t rows = (uint64_t)nB * n;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t r = wave; r < rows; r += nwaves) {
        const uint32_t N = (uint32_t)(r / n), v = (uint32_t)(r % n);
        if (!test_bit(act + (uint64_t)N * Pn, v)) continue;
        const unsigned long long key = dedup_key(dhash[r], N);
        uint64_t slot = key & mask;
        while (keys[slot] != key) slot = (slot + 1) & mask;   // inserted above: found
        const uint32_t c = vals[slot];
        uint32_t out = v;
        if (c != (uint32_t)r && c / n == N) {
            const uint64_t rc = c;
            bool diff = false;
            for (uint32_t k = lane; k < sum_pitch; k += kWave)
                diff |= dsum[r * sum_pitch + k] != dsum[rc * sum_pitch + k];
            if (!__ballot(diff)) {
                for (uint32_t k = lane; k < Pn; k += kWave) {
                    const uint64_t sw = dsum[r * sum_pitch + k / kWave];
                    if ((sw >> (k & 63)) & 1ull) diff |= dNT[r * P + k] != dNT[rc * P + k];
                }
            }
            if (!__ballot(diff)) out = c % n;
        }
        if (lane == 0) rep[r] = out;
    }
}

hipError_t launch_dedup(uint32_t nB, uint32_t n, uint32_t P, uint32_t Pn, const uint64_t *act, const uint64_t *dhash,
                        const uint64_t *dNT, const uint64_t *dsum, uint32_t sum_pitch, unsigned long long *keys,
                        uint32_t *vals, uint64_t mask, uint32_t *rep, hipStream_t s) {
    const uint64_t rows = (uint64_t)nB * n;
    hipError_t e = launch_fill((uint64_t *)keys, mask + 1, 0, s);
    if (e == hipSuccess) e = launch_fill((uint64_t *)vals, (mask + 1) / 2, ~0ull, s);   // u32 slots, pairs per word
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dedup_insert, dim3(grid_for(rows)), dim3(kBlock), 0, s, nB, n, Pn, act, dhash, keys, vals,
                       mask);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dedup_rep, dim3(grid_for(rows * kWave)), dim3(kBlock), 0, s, nB, n, P, Pn, act, dhash, dNT,
                       dsum, sum_pitch, keys, vals, mask, rep);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// result kernels
// ---------------------------------------------------------------------------
__global__ void k_popcount(const uint64_t *p, uint64_t rows, uint32_t pitch, uint32_t words,
                           unsigned long long *out) {
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gthreads = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long c = 0;
    for (uint64_t i = gtid; i < rows * words; i += gthreads)
        c += (unsigned long long)__popcll(p[(i / words) * pitch + (i % words)]);
    block_add(out, c);
}

hipError_t launch_popcount(const uint64_t *p, uint64_t rows, uint32_t pitch, uint32_t words,
                           unsigned long long *out, hipStream_t s) {
    hipLaunchKernelGGL(k_popcount, dim3(grid_for(rows * words)), dim3(kBlock), 0, s, p, rows, pitch,
                       words, out);
    return hipGetLastError();
}

// NTb: one box's transposed matrix, row v = bits over u.
__global__ void k_hash(const uint64_t *NTb, uint32_t n, uint32_t P, unsigned long long *out) {
    const uint32_t Pn = (n + 63) / 64;
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gthreads = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long h = 0;
    for (uint64_t i = gtid; i < (uint64_t)n * Pn; i += gthreads) {
        const uint32_t v = (uint32_t)(i / Pn), k = (uint32_t)(i % Pn);
        uint64_t bits = NTb[(uint64_t)v * P + k];
        while (bits) {
            const int b = __ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            const uint64_t u = (uint64_t)k * 64 + b;
            h += splitmix64((u << 32) | v);
        }
    }
    block_add(out, h);
}

hipError_t launch_hash(const uint64_t *NTb, uint32_t n, uint32_t P, unsigned long long *out,
                       hipStream_t s) {
    const uint64_t items = (uint64_t)n * ((n + 63) / 64);
    hipLaunchKernelGGL(k_hash, dim3(grid_for(items)), dim3(kBlock), 0, s, NTb, n, P, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// witness search: one breadth-first level over a box's product graph
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bfs_claim(const WitnessBfs &b, uint32_t id, uint32_t from, uint32_t sym) {
    if (atomicCAS(&b.par[id], kNoSlot, from) != kNoSlot) return;   // already reached
    b.psym[id] = sym;
    b.next[atomicAdd(&b.ctr[0], 1u)] = id;
    if (id % b.n == b.v_target && b.final[id / b.n]) atomicCAS(&b.ctr[1], kNoSlot, id);
}

__global__ __launch_bounds__(kBlock) void k_witness_bfs(WitnessBfs b) {
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t i = wave; i < b.ncur; i += nwaves) {
        const uint32_t node = b.cur[i], q = node / b.n, x = node % b.n;
        for (uint32_t t = b.s_off[q]; t < b.s_off[q + 1]; ++t) {
            const InTrans tr = b.s_tr[t];
            const uint32_t f = tr.src;
            if (tr.sym < b.n_terms) {
                const uint32_t e0 = b.soff[(uint64_t)tr.sym * (b.n + 1) + x], e1 = b.soff[(uint64_t)tr.sym * (b.n + 1) + x + 1];
                for (uint32_t e = e0 + (uint32_t)lane; e < e1; e += kWave) bfs_claim(b, f * b.n + b.sidx[e], node, tr.sym);
            } else if (b.rank) {
                const uint8_t *row = b.rank + ((uint64_t)(tr.sym - b.n_terms) * b.n + x) * b.n;
                for (uint32_t y = (uint32_t)lane; y < b.n; y += kWave)
                    if (row[y] < b.rk) bfs_claim(b, f * b.n + y, node, tr.sym);
            }
        }
    }
}

hipError_t launch_witness_bfs(const WitnessBfs &b, hipStream_t s) {
    if (!b.ncur) return hipSuccess;
    hipLaunchKernelGGL(k_witness_bfs, dim3(grid_for((uint64_t)b.ncur * kWave)), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, value);
    return hipGetLastError();
}

// 64x64 bit-block transpose, one wavefront per block: lane i holds source
// row (64*vb + i), word ub; ballot of bit j across lanes is destination row
// (64*ub + j), word vb.
__global__ __launch_bounds__(kBlock) void k_transpose(const uint64_t *src, uint32_t src_pitch,
                                                      uint64_t *dst, uint32_t dst_pitch, uint32_t n) {
    const uint32_t Pn = (n + 63) / 64;
    const int lane = __lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t blk = wave; blk < (uint64_t)Pn * Pn; blk += nwaves) {
        const uint32_t vb = (uint32_t)(blk / Pn), ub = (uint32_t)(blk % Pn);
        const uint32_t v = vb * 64 + lane;
        const uint64_t word = v < n ? src[(uint64_t)v * src_pitch + ub] : 0ull;
        uint64_t mine = 0;
        for (int j = 0; j < 64; ++j) {
            const uint64_t col = __ballot((word >> j) & 1ull);
            if (lane == j) mine = col;
        }
        const uint32_t u = ub * 64 + lane;
        if (u < n) dst[(uint64_t)u * dst_pitch + vb] = mine;
    }
}

hipError_t launch_transpose(const uint64_t *src, uint32_t src_pitch, uint64_t *dst,
                            uint32_t dst_pitch, uint32_t n, hipStream_t s) {
    const uint64_t Pn = (n + 63) / 64;
    hipLaunchKernelGGL(k_transpose, dim3(grid_for(Pn * Pn * 64)), dim3(kBlock), 0, s, src, src_pitch,
                       dst, dst_pitch, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused small-graph fixpoint: one workgroup runs the whole loop of Listing 1
// for one query, with workgroup barriers in place of kernel boundaries.  A
// persistent grid drains a device queue of queries, so many small queries
// share one launch.
// ---------------------------------------------------------------------------
constexpr int kFusedBlock = 1024;
constexpr int kFusedMaxBoxes = 64;

__device__ void block_fill(uint64_t *p, uint64_t words) {
    for (uint64_t i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0;
}

// Rows of at most kNarrowWords words (n <= 512): one thread per row instead
// of one wavefront, which would leave all but a few lanes idle; the fused
// kernel walks its rows this way.
constexpr uint32_t kNarrowWords = 8;

template <bool SEED>
__device__ bool gather_row_thread(const GatherArgs &a, uint32_t f, uint32_t v, unsigned long long &cnt) {
    const uint32_t tb = a.in_off[f], te = a.in_off[f + 1];
    if (tb == te) return false;
    uint64_t acc[kNarrowWords];
#pragma unroll
    for (uint32_t w = 0; w < kNarrowWords; ++w) acc[w] = 0;
    bool fed = false;
    auto take = [&](const uint64_t *r) {
#pragma unroll
        for (uint32_t w = 0; w < kNarrowWords; ++w)
            if (w < a.gw) acc[w] |= r[w];
        fed = true;
    };
    for (uint32_t t = tb; t < te; ++t) {
        const InTrans tr = a.in_tr[t];
        const uint64_t *rows = a.src + (uint64_t)tr.src * a.n * a.src_pitch + a.src_off;
        const uint64_t *sact = a.src_act + (uint64_t)tr.src * a.Pn;
        if (tr.sym < a.n_terms) {
            if (SEED && !a.seed_terms) continue;
            const uint32_t *op = a.goff + (uint64_t)tr.sym * (a.n + 1) + v;
            for (uint32_t e = op[0]; e < op[1]; ++e) {
                const uint32_t x = a.gidx[e];
                if (test_bit(sact, x)) take(rows + (uint64_t)x * a.src_pitch);
            }
        } else {
            const uint32_t N = tr.sym - a.n_terms;
            if (SEED && !test_bit(a.sel_act + (uint64_t)N * a.Pn, v)) continue;
            const uint64_t *sel = a.sel + ((uint64_t)N * a.n + v) * a.P;
            for (uint32_t k = 0; k < a.Pn; ++k)
                for (uint64_t b = sel[k] & sact[k]; b; b &= b - 1)
                    take(rows + (uint64_t)(k * 64 + (uint32_t)__builtin_ctzll(b)) * a.src_pitch);
        }
    }
    if (!fed) return false;
    uint64_t *trow = a.T + ((uint64_t)f * a.n + v) * a.P + a.w0;
    uint64_t *drow = a.dn + ((uint64_t)f * a.n + v) * a.G;
    bool any = false;
#pragma unroll
    for (uint32_t w = 0; w < kNarrowWords; ++w) {
        if (w < a.gw) {
            const uint64_t t = trow[w];
            const uint64_t nw = acc[w] & ~t;
            if (nw) {
                trow[w] = t | nw;
                any = true;
                cnt += (unsigned long long)__popcll(nw);
            }
            drow[w] = nw;
        }
    }
    return any;
}

// write-back of one row (N, v) by one thread (narrow rows; see writeback_row)
__device__ bool writeback_row_thread(const WritebackArgs &a, uint32_t N, uint32_t v, unsigned long long &cnt_box) {
    const uint32_t fb = a.fin_off[N], fe = a.fin_off[N + 1];
    uint64_t *nt = a.NT + ((uint64_t)N * a.n + v) * a.P;
    uint64_t *dnt = a.dNT + ((uint64_t)N * a.n + v) * a.P;
    bool any = false;
    for (uint32_t k = 0; k < a.Pn; ++k) {
        uint64_t acc = 0;
        for (uint32_t i = fb; i < fe; ++i) acc |= a.T[((uint64_t)a.fin[i] * a.n + v) * a.P + k];
        const uint64_t old = nt[k];
        const uint64_t nw = acc & ~old;
        if (nw) {
            nt[k] = old | nw;
            any = true;
            cnt_box += (unsigned long long)__popcll(nw);
            if (a.rank)
                for (uint64_t bits = nw; bits; bits &= bits - 1)
                    a.rank[((uint64_t)N * a.n + (uint64_t)k * 64 + __builtin_ctzll(bits)) * a.n + v] =
                        (uint8_t)(a.iter > 255 ? 255 : a.iter);
        }
        dnt[k] = nw;
    }
    return any;
}

__device__ void run_fused(const FusedQuery &Q, unsigned long long *s_cnt,
                          unsigned long long *s_box) {
    const int lane = __lane_id();
    const uint32_t wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const uint64_t qwords = (uint64_t)Q.nQ * Q.n * Q.P, bwords = (uint64_t)Q.nB * Q.n * Q.P;
    block_fill(Q.T, qwords);
    block_fill(Q.NT, bwords);
    block_fill(Q.dNT, bwords);
    block_fill(Q.tnz, (uint64_t)Q.nQ * Q.Pn);
    block_fill(Q.act, (uint64_t)Q.nQ * Q.Pn);
    block_fill(Q.actn, (uint64_t)Q.nQ * Q.Pn);
    block_fill(Q.dnt_act, (uint64_t)Q.nB * Q.Pn);
    if (threadIdx.x == 0) {
        Q.stats[0] = 0;
        Q.stats[1] = 0;
    }
    __syncthreads();
    seed_diag_body(Q.T, Q.tnz, Q.n, Q.P, Q.Pn, Q.starts, Q.nB, threadIdx.x, blockDim.x);
    __syncthreads();
    // epsilon initialisation for nullable boxes
    if (threadIdx.x < Q.nB) s_box[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t b = 0; b < Q.nB; ++b) {
        if (!Q.nullable[b]) continue;
        for (uint64_t i = threadIdx.x; i < Q.n; i += blockDim.x) {
            const uint32_t v = (uint32_t)i;
            const uint64_t off = ((uint64_t)b * Q.n + v) * Q.P + (v >> 6);
            Q.NT[off] |= 1ull << (v & 63);
            Q.dNT[off] |= 1ull << (v & 63);
            if (Q.rank) Q.rank[((uint64_t)b * Q.n + v) * Q.n + v] = 0;
        }
        for (uint64_t k = threadIdx.x; k < Q.Pn; k += blockDim.x) {
            const uint32_t hi = Q.n - (uint32_t)k * 64;
            Q.dnt_act[(uint64_t)b * Q.Pn + k] = hi >= 64 ? ~0ull : ((1ull << hi) - 1);
        }
        if (threadIdx.x == 0) s_box[b] = Q.n;
    }
    __syncthreads();

    GatherArgs a;
    a.n = Q.n; a.P = Q.P; a.Pn = Q.Pn; a.n_terms = Q.n_terms; a.nQ = Q.nQ;
    a.w0 = 0; a.gw = Q.Pn; a.G = Q.P;
    a.goff = Q.goff; a.gidx = Q.gidx; a.in_off = Q.in_off; a.in_tr = Q.in_tr;
    a.T = Q.T; a.tnz = Q.tnz;
    a.act_clear = nullptr; a.clear_words = 0; a.ctr = nullptr;
    a.slot_prev = kNoSlot; a.slot_cur = 0;
    a.extra = nullptr; a.extra_act = nullptr;
    a.sel_sum = nullptr; a.sum_pitch = 0;
    a.src_blk = nullptr; a.actn_blk = nullptr; a.Pbs = 0; a.chg = nullptr; a.bytes_ctr = nullptr;
    a.dense_apart = 0;
    a.rep = nullptr;
    a.f_box = nullptr;
    a.chgb = nullptr;
    a.blk_shift = 6;

    WritebackArgs wb;
    wb.n = Q.n; wb.P = Q.P; wb.Pn = Q.Pn; wb.nB = Q.nB; wb.fin_off = Q.fin_off; wb.fin = Q.fin;
    wb.T = Q.T; wb.NT = Q.NT; wb.dNT = Q.dNT; wb.dnt_act = Q.dnt_act; wb.rank = Q.rank;
    wb.ctr = nullptr; wb.slot_base = 0; wb.row_map = nullptr; wb.fresh = 0; wb.row_nz = nullptr;
    wb.state_flags = nullptr; wb.multi = nullptr; wb.skip_if[0] = wb.skip_if[1] = nullptr;
    wb.chg = nullptr; wb.prev_act = nullptr; wb.rows_ctr = nullptr;
    wb.dsum = nullptr; wb.nsum = nullptr; wb.sum_pitch = 0; wb.dhash = nullptr;
    wb.chgb = nullptr; wb.dnb = nullptr; wb.blk_words = kWave;

    uint64_t *D = Q.D, *Dn = Q.Dn, *act = Q.act, *actn = Q.actn;
    const bool narrow = Q.Pn <= kNarrowWords;
    uint32_t it = 0;
    unsigned long long status = 0;
    for (;;) {
        ++it;
        if (Q.max_iters && it > Q.max_iters) {
            status = 1;
            break;
        }
        bool can_seed = (it == 1);
        for (uint32_t b = 0; b < Q.nB; ++b) can_seed |= (s_box[b] != 0 && Q.box_used[b]);
        if (!can_seed) {
            if (it - 1 < Q.stats_cap && threadIdx.x == 0) Q.stats[2 + it - 1] = 0;
            break;
        }
        // Kronecker product with the new edges
        a.sel = Q.dNT; a.sel_act = Q.dnt_act; a.src = Q.T; a.src_pitch = Q.P; a.src_off = 0;
        a.src_act = Q.tnz; a.dn = Dn; a.actn = actn; a.seed_terms = (it == 1);
        if (threadIdx.x == 0) *s_cnt = 0;
        __syncthreads();
        unsigned long long cnt = 0;
        if (narrow) {
            for (uint64_t r = threadIdx.x; r < (uint64_t)Q.nQ * Q.n; r += blockDim.x) {
                const uint32_t f = (uint32_t)(r / Q.n), v = (uint32_t)(r % Q.n);
                if (gather_row_thread<true>(a, f, v, cnt)) {
                    atomicOr((unsigned long long *)&actn[(uint64_t)f * Q.Pn + (v >> 6)], 1ull << (v & 63));
                    atomicOr((unsigned long long *)&Q.tnz[(uint64_t)f * Q.Pn + (v >> 6)], 1ull << (v & 63));
                }
            }
        } else {
            for (uint64_t r = wave; r < (uint64_t)Q.nQ * Q.n; r += nwaves) {
                const uint32_t f = (uint32_t)(r / Q.n), v = (uint32_t)(r % Q.n);
                bool fed;
                unsigned long long by = 0;
                uint64_t blocks = 0;
                if (gather_row<true>(a, f, v, cnt, fed, by, blocks) && lane == 0) {
                    atomicOr((unsigned long long *)&actn[(uint64_t)f * Q.Pn + (v >> 6)], 1ull << (v & 63));
                    atomicOr((unsigned long long *)&Q.tnz[(uint64_t)f * Q.Pn + (v >> 6)], 1ull << (v & 63));
                }
            }
        }
        cnt = wave_sum(cnt);
        if (lane == 0 && cnt) atomicAdd(s_cnt, cnt);
        __syncthreads();
        // incremental closure: frontier levels until no new bit
        while (*s_cnt != 0) {
            uint64_t *t = D; D = Dn; Dn = t;
            t = act; act = actn; actn = t;
            block_fill(actn, (uint64_t)Q.nQ * Q.Pn);
            __syncthreads();
            if (threadIdx.x == 0) *s_cnt = 0;
            __syncthreads();
            a.sel = Q.NT; a.sel_act = nullptr; a.src = D; a.src_pitch = Q.P; a.src_off = 0;
            a.src_act = act; a.dn = Dn; a.actn = actn;
            cnt = 0;
            if (narrow) {
                for (uint64_t r = threadIdx.x; r < (uint64_t)Q.nQ * Q.n; r += blockDim.x) {
                    const uint32_t f = (uint32_t)(r / Q.n), v = (uint32_t)(r % Q.n);
                    if (gather_row_thread<false>(a, f, v, cnt)) {
                        atomicOr((unsigned long long *)&actn[(uint64_t)f * Q.Pn + (v >> 6)], 1ull << (v & 63));
                        atomicOr((unsigned long long *)&Q.tnz[(uint64_t)f * Q.Pn + (v >> 6)], 1ull << (v & 63));
                    }
                }
            } else {
                for (uint64_t r = wave; r < (uint64_t)Q.nQ * Q.n; r += nwaves) {
                    const uint32_t f = (uint32_t)(r / Q.n), v = (uint32_t)(r % Q.n);
                    bool fed;
                    unsigned long long by = 0;
                    uint64_t blocks = 0;
                    if (gather_row<false>(a, f, v, cnt, fed, by, blocks) && lane == 0) {
                        atomicOr((unsigned long long *)&actn[(uint64_t)f * Q.Pn + (v >> 6)], 1ull << (v & 63));
                        atomicOr((unsigned long long *)&Q.tnz[(uint64_t)f * Q.Pn + (v >> 6)], 1ull << (v & 63));
                    }
                }
            }
            cnt = wave_sum(cnt);
            if (lane == 0 && cnt) atomicAdd(s_cnt, cnt);
            __syncthreads();
        }
        // write-back
        block_fill(Q.dnt_act, (uint64_t)Q.nB * Q.Pn);
        if (threadIdx.x < Q.nB) s_box[threadIdx.x] = 0;
        __syncthreads();
        wb.iter = it;
        if (narrow) {
            for (uint64_t r = threadIdx.x; r < (uint64_t)Q.nB * Q.n; r += blockDim.x) {
                const uint32_t N = (uint32_t)(r / Q.n), v = (uint32_t)(r % Q.n);
                if (Q.fin_off[N] == Q.fin_off[N + 1]) continue;
                unsigned long long c = 0;
                if (writeback_row_thread(wb, N, v, c)) {
                    atomicOr((unsigned long long *)&Q.dnt_act[(uint64_t)N * Q.Pn + (v >> 6)], 1ull << (v & 63));
                    atomicAdd(&s_box[N], c);
                }
            }
        } else {
            for (uint64_t r = wave; r < (uint64_t)Q.nB * Q.n; r += nwaves) {
                const uint32_t N = (uint32_t)(r / Q.n), v = (uint32_t)(r % Q.n);
                if (Q.fin_off[N] == Q.fin_off[N + 1]) continue;
                unsigned long long c = 0;
                bool any = false;
                writeback_row(wb, N, v, c, any);
                c = wave_sum(c);
                if (lane == 0 && any) {
                    atomicOr((unsigned long long *)&Q.dnt_act[(uint64_t)N * Q.Pn + (v >> 6)], 1ull << (v & 63));
                    atomicAdd(&s_box[N], c);
                }
            }
        }
        __syncthreads();
        unsigned long long delta = 0;
        for (uint32_t b = 0; b < Q.nB; ++b) delta += s_box[b];
        if (threadIdx.x == 0 && it - 1 < Q.stats_cap) Q.stats[2 + it - 1] = delta;
        if (delta == 0) break;
        // next iteration starts with empty frontier buffers
        block_fill(actn, (uint64_t)Q.nQ * Q.Pn);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Q.stats[0] = it;
        Q.stats[1] = status;
    }
    __syncthreads();
}

// A query whose working set fits the launch's dynamic LDS runs there: its
// copy of the query record points T, the frontiers, M2^N, A2^N and the
// activity bitsets into LDS (rows at an LDS pitch of about Pn words), so
// every row access of the fixpoint is an LDS access instead of an L2 round
// trip; at the end its M2^N rows go out to the result at the global pitch
// (pad words zero).  Other queries run on their global buffers.
__global__ __launch_bounds__(kFusedBlock) void k_fused(const FusedQuery *qs, uint32_t n_queries,
                                                      uint32_t *next_query, uint64_t lds_words) {
    extern __shared__ uint64_t s_ws[];
    __shared__ uint32_t s_q;
    __shared__ unsigned long long s_cnt;
    __shared__ unsigned long long s_box[kFusedMaxBoxes];
    __shared__ FusedQuery s_fq;
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(next_query, 1u);
        __syncthreads();
        const uint32_t qi = s_q;
        __syncthreads();
        if (qi >= n_queries) return;
        const FusedQuery &G = qs[qi];
        const uint32_t n = G.n, Pn = G.Pn, nQ = G.nQ, nB = G.nB;
        const bool in_lds = G.lds_ok && fused_lds_words(n, Pn, Pn, nQ, nB) <= lds_words;
        const uint32_t lp = fused_lds_pitch(n, Pn, nQ, nB, lds_words);
        if (in_lds && threadIdx.x == 0) {
            s_fq = G;
            s_fq.P = lp;
            uint64_t *w = s_ws;   // a generic pointer into LDS
            s_fq.T = w;
            w += (uint64_t)nQ * n * lp;
            s_fq.D = w;
            w += (uint64_t)nQ * n * lp;
            s_fq.Dn = w;
            w += (uint64_t)nQ * n * lp;
            s_fq.NT = w;
            w += (uint64_t)nB * n * lp;
            s_fq.dNT = w;
            w += (uint64_t)nB * n * lp;
            s_fq.act = w;
            w += (uint64_t)nQ * Pn;
            s_fq.actn = w;
            w += (uint64_t)nQ * Pn;
            s_fq.tnz = w;
            w += (uint64_t)nQ * Pn;
            s_fq.dnt_act = w;
        }
        __syncthreads();
        run_fused(in_lds ? s_fq : G, &s_cnt, s_box);   // ends with a workgroup barrier
        if (!in_lds) continue;
        const uint32_t gp = G.P;
        uint64_t *out = G.NT;
        const uint64_t *nt = s_fq.NT;
        for (uint64_t i = threadIdx.x; i < (uint64_t)nB * n * gp; i += blockDim.x) {
            const uint64_t row = i / gp;
            const uint32_t w = (uint32_t)(i - row * gp);
            out[i] = w < Pn ? nt[row * lp + w] : 0ull;
        }
        __syncthreads();
    }
}

uint64_t fused_lds_limit_words() {
    if (!CFPQ_FUSED_LDS) return 0;
    int dev = 0, per_block = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_fused)) != hipSuccess) return 0;
    const int64_t free_bytes = (int64_t)per_block - (int64_t)fa.sharedSizeBytes;
    return free_bytes > 0 ? (uint64_t)free_bytes / 8 : 0;
}

hipError_t launch_fused(const FusedQuery *qs_dev, uint32_t n_queries, uint32_t *next_query, uint64_t lds_words,
                        hipStream_t s) {
    uint32_t grid = n_queries < 1024 ? n_queries : 1024;
    if (!grid) return hipSuccess;
    const size_t lds_bytes = (size_t)lds_words * 8;
    if (lds_bytes) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fused),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_fused, dim3(grid), dim3(kFusedBlock), lds_bytes, s, qs_dev, n_queries, next_query,
                       lds_words);
    return hipGetLastError();
}

}  // namespace cfpq
