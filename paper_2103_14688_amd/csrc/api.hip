// Host side of the C ABI declared in include/cfpq.h: validation, graph and
// RSM staging, the fixpoint driver (Sec. 3.1, Listing 1), result accessors
// and single-witness extraction (Sec. 3.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <array>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>
#include <unordered_set>
#include <unordered_map>
#include <functional>

#include "../../include/cfpq.h"
#include "internal.h"

using namespace cfpq;

namespace {

thread_local std::string g_err;

cfpq_status fail(cfpq_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(CFPQ_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// device memory through the optional allocator hooks
// ---------------------------------------------------------------------------
struct Alloc {
    cfpq_allocator a{};
    bool has = false;
    explicit Alloc(const cfpq_allocator *p = nullptr) {
        if (p && p->alloc && p->free) {
            a = *p;
            has = true;
        }
    }
    void *get(size_t bytes, hipStream_t s) const {
        if (!bytes) bytes = 8;
        if (has) {
            void *p = a.alloc(bytes, (void *)s, a.ctx);
            if (p && ((uintptr_t)p & 255u)) {   // the kernels take whole aligned vectors
                a.free(p, bytes, (void *)s, a.ctx);
                return nullptr;
            }
            return p;
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        return p;
    }
    // bytes the hooks hold unused and can hand out again (0 without hooks)
    size_t cached() const { return has && a.cached ? a.cached(a.ctx) : 0; }
    void put(void *p, size_t bytes, hipStream_t s) const {
        if (!p) return;
        if (!bytes) bytes = 8;
        if (has)
            a.free(p, bytes, (void *)s, a.ctx);
        else
            (void)hipFree(p);
    }
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    const Alloc *al = nullptr;
    hipStream_t s = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        release();
        p = o.p; bytes = o.bytes; al = o.al; s = o.s;
        o.p = nullptr; o.bytes = 0;
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p && al) al->put(p, bytes, s);
        p = nullptr;
        bytes = 0;
    }
    bool alloc(const Alloc *a, size_t nbytes, hipStream_t st) {
        release();
        al = a; s = st; bytes = nbytes ? nbytes : 8;
        p = a->get(bytes, st);
        return p != nullptr;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

uint32_t round_up(uint32_t x, uint32_t m) { return (x + m - 1) / m * m; }
constexpr uint64_t align256(uint64_t b) { return (b + 255) / 256 * 256; }
// row pitch of the device bitsets in 64-bit words: rows start on 128-byte
// cache-line boundaries (with chunk boundaries on them too, the condensed
// level kernel's stores cover whole lines: 1.51 -> 1.47 ms per query on the
// power-law RPQ at n = 10^5, against 64-byte rows)
#ifndef CFPQ_ROW_ALIGN_WORDS
#define CFPQ_ROW_ALIGN_WORDS 16
#endif
constexpr uint32_t kRowAlignWords = CFPQ_ROW_ALIGN_WORDS;
static_assert(kRowAlignWords % 2 == 0, "rows start on 16-byte boundaries");
// rows of at most 8 words keep an 8-word pitch: small graphs (the fused
// path) would otherwise clear and scan twice the memory
uint32_t row_pitch(uint32_t Pn) { return round_up(Pn, Pn <= 8 ? 8u : kRowAlignWords); }

// the graph's successor lists on the host, shared by the graph and the
// results made on it (path extraction reads them after the graph is gone)
struct HostCsr {
    std::vector<uint32_t> off, out;   // label l, vertex u: out[off[l * (n + 1) + u] .. off[l * (n + 1) + u + 1]), sorted
};

}  // namespace

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct cfpq_graph_s {
    int device = 0;
    uint32_t n = 0, n_labels = 0;
    uint64_t n_edges = 0;
    Alloc alloc;
    DevBuf off, idx;                         // CSC per label (predecessors)
    DevBuf soff, sidx;                       // CSR per label (successors)
    std::shared_ptr<HostCsr> hcsr;           // CSR per label (successors), host
    // launch-chain sizes the last condensed query on this graph needed; with
    // all three set, the next condensed query goes out in one piece with
    // these sizes (speculation only: a chain that needs more continues on
    // the host, one that needs less exits its surplus launches at once)
    mutable std::atomic<uint32_t> hint_trim{0}, hint_reach{0}, hint_levels{0};
};

struct cfpq_rsm_s {
    uint32_t n_states = 0, n_terms = 0, n_boxes = 0, start_box = 0;
    std::vector<uint32_t> box_start, state_box, t_src, t_sym, t_dst;
    std::vector<uint8_t> is_final;
};

// Device memory that several results share (the answer matrices of one
// fused batch): freed when the last of them is closed.
struct SharedDev {
    Alloc al;
    DevBuf buf;   // declared after al: freed through it
};

struct cfpq_result_s {
    int device = 0;
    uint32_t n = 0, P = 0, Pn = 0, nB = 0, nQ = 0;
    hipStream_t stream = nullptr;
    Alloc alloc;
    DevBuf NT;        // [nB][n][P] transposed nonterminal matrices (a view into nt_block when set)
    std::shared_ptr<SharedDev> nt_block;
    DevBuf T;         // [nQ][n][P] closure rows (keep_blocks)
    DevBuf rank;      // [nB][n][n] u8 (keep_rank)
    DevBuf scratch;   // small device scratch for accessors
    DevBuf src_mask;  // [Pn] source mask of the start box (optional)
    uint32_t iterations = 0;
    std::vector<uint64_t> deltas;
    double ms = 0.0;
    cfpq_rsm_s rsm;                              // copy
    std::shared_ptr<const HostCsr> hcsr;         // graph successors (the graph's, shared)
    uint32_t n_labels = 0;
    struct WitnessDev;
    std::unique_ptr<WitnessDev> wdev;            // witness search buffers, built on first use
    struct Prof {
        uint64_t launches = 0, bytes = 0;
        double ms = 0.0;
    } prof[9];
    bool profiled = false;
};

// buffers of the device witness search, kept by the result after the first
// extraction: the graph's successor lists, the RSM's transitions by source
// state and its final states, parent pointers and two frontiers
struct cfpq_result_s::WitnessDev {
    DevBuf buf;
    uint32_t *off = nullptr, *idx = nullptr, *s_off = nullptr, *fin = nullptr, *par = nullptr, *psym = nullptr;
    uint32_t *fr[2] = {nullptr, nullptr};
    InTrans *s_tr = nullptr;
    unsigned int *ctr = nullptr;
};

// ---------------------------------------------------------------------------
// graph
// ---------------------------------------------------------------------------
extern "C" cfpq_status cfpq_graph_create(uint32_t n, uint32_t n_labels, const uint32_t *src,
                                         const uint32_t *label, const uint32_t *dst,
                                         uint64_t n_edges, uint32_t flags,
                                         const cfpq_allocator *alloc, void *stream,
                                         cfpq_graph *out) {
    if (!out) return fail(CFPQ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n == 0 || n_labels == 0) return fail(CFPQ_ERR_INVALID, "graph needs n_vertices >= 1 and n_labels >= 1");
    if (n_edges && (!src || !label || !dst)) return fail(CFPQ_ERR_INVALID, "edge array is NULL");
    if (flags & ~(CFPQ_ADD_INVERSES | CFPQ_DEVICE_PTRS)) return fail(CFPQ_ERR_INVALID, "unknown flag");
    if (n == 0xFFFFFFFFu) return fail(CFPQ_ERR_INVALID, "too many vertices");
    std::vector<uint32_t> h_src, h_lbl, h_dst;   // host copies of device edge arrays
    if ((flags & CFPQ_DEVICE_PTRS) && n_edges) {
        try {
            h_src.resize(n_edges);
            h_lbl.resize(n_edges);
            h_dst.resize(n_edges);
        } catch (...) {
            return fail(CFPQ_ERR_OOM, "host allocation failed");
        }
        hipStream_t cs = (hipStream_t)stream;
        HIP_TRY(hipMemcpyAsync(h_src.data(), src, n_edges * 4, hipMemcpyDeviceToHost, cs));
        HIP_TRY(hipMemcpyAsync(h_lbl.data(), label, n_edges * 4, hipMemcpyDeviceToHost, cs));
        HIP_TRY(hipMemcpyAsync(h_dst.data(), dst, n_edges * 4, hipMemcpyDeviceToHost, cs));
        HIP_TRY(hipStreamSynchronize(cs));
        src = h_src.data();
        label = h_lbl.data();
        dst = h_dst.data();
    }
    const bool inv = flags & CFPQ_ADD_INVERSES;
    const uint32_t L = inv ? 2 * n_labels : n_labels;
    if (inv && n_labels > 0x7FFFFFFFu) return fail(CFPQ_ERR_INVALID, "too many labels");
    struct E { uint32_t l, d, s; };
    std::vector<E> e;
    try {
        e.reserve(inv ? 2 * n_edges : n_edges);
    } catch (...) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    for (uint64_t i = 0; i < n_edges; ++i) {
        if (src[i] >= n || dst[i] >= n) return fail(CFPQ_ERR_INVALID, "edge " + std::to_string(i) + ": vertex out of range");
        if (label[i] >= n_labels) return fail(CFPQ_ERR_INVALID, "edge " + std::to_string(i) + ": label out of range");
        e.push_back({label[i], dst[i], src[i]});
        if (inv) e.push_back({label[i] + n_labels, src[i], dst[i]});
    }
    std::sort(e.begin(), e.end(), [](const E &a, const E &b) {
        if (a.l != b.l) return a.l < b.l;
        if (a.d != b.d) return a.d < b.d;
        return a.s < b.s;
    });
    e.erase(std::unique(e.begin(), e.end(), [](const E &a, const E &b) {
                return a.l == b.l && a.d == b.d && a.s == b.s;
            }),
            e.end());
    if (e.size() >= 0xFFFFFFFFull) return fail(CFPQ_ERR_INVALID, "more than 2^32-1 distinct edges");

    std::unique_ptr<cfpq_graph_s> g(new (std::nothrow) cfpq_graph_s);
    if (!g) return fail(CFPQ_ERR_OOM, "host allocation failed");
    HIP_TRY(hipGetDevice(&g->device));
    g->n = n;
    g->n_labels = L;
    g->n_edges = e.size();
    g->alloc = Alloc(alloc);
    hipStream_t s = (hipStream_t)stream;

    const uint64_t noff = (uint64_t)L * (n + 1);
    std::vector<uint32_t> off(noff, 0), idx(e.size());
    try {
        g->hcsr = std::make_shared<HostCsr>();
        g->hcsr->off.assign(noff, 0);
        g->hcsr->out.resize(e.size());
    } catch (...) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    for (const E &x : e) {
        off[(uint64_t)x.l * (n + 1) + x.d + 1]++;
        g->hcsr->off[(uint64_t)x.l * (n + 1) + x.s + 1]++;
    }
    // offsets are global across labels: label l's lists start where l-1's end
    uint64_t run = 0, run2 = 0;
    for (uint32_t l = 0; l < L; ++l) {
        uint32_t *o = &off[(uint64_t)l * (n + 1)];
        uint32_t *o2 = &g->hcsr->off[(uint64_t)l * (n + 1)];
        o[0] = (uint32_t)run;
        o2[0] = (uint32_t)run2;
        for (uint32_t v = 0; v < n; ++v) {
            run += o[v + 1];
            o[v + 1] = (uint32_t)run;
            run2 += o2[v + 1];
            o2[v + 1] = (uint32_t)run2;
        }
    }
    for (uint64_t i = 0; i < e.size(); ++i) idx[i] = e[i].s;  // sorted by (l, d, s)
    {
        std::vector<uint32_t> fill(g->hcsr->off.begin(), g->hcsr->off.end());
        for (const E &x : e) g->hcsr->out[fill[(uint64_t)x.l * (n + 1) + x.s]++] = x.d;
        for (uint32_t l = 0; l < L; ++l)
            for (uint32_t u = 0; u < n; ++u) {
                uint64_t a = g->hcsr->off[(uint64_t)l * (n + 1) + u], b = g->hcsr->off[(uint64_t)l * (n + 1) + u + 1];
                std::sort(g->hcsr->out.begin() + a, g->hcsr->out.begin() + b);
            }
    }
    if (!g->off.alloc(&g->alloc, noff * sizeof(uint32_t), s) ||
        !g->idx.alloc(&g->alloc, idx.size() * sizeof(uint32_t), s) ||
        !g->soff.alloc(&g->alloc, noff * sizeof(uint32_t), s) ||
        !g->sidx.alloc(&g->alloc, idx.size() * sizeof(uint32_t), s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (graph)");
    HIP_TRY(hipMemcpyAsync(g->off.p, off.data(), noff * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(g->soff.p, g->hcsr->off.data(), noff * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    if (!idx.empty()) {
        HIP_TRY(hipMemcpyAsync(g->idx.p, idx.data(), idx.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(g->sidx.p, g->hcsr->out.data(), idx.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    *out = g.release();
    return CFPQ_OK;
}

extern "C" cfpq_status cfpq_graph_info(cfpq_graph g, uint32_t *n, uint32_t *n_labels, uint64_t *n_edges) {
    if (!g) return fail(CFPQ_ERR_INVALID, "graph is NULL");
    if (n) *n = g->n;
    if (n_labels) *n_labels = g->n_labels;
    if (n_edges) *n_edges = g->n_edges;
    return CFPQ_OK;
}

extern "C" void cfpq_graph_destroy(cfpq_graph g) { delete g; }

// ---------------------------------------------------------------------------
// RSM
// ---------------------------------------------------------------------------
extern "C" cfpq_status cfpq_rsm_create(uint32_t n_states, uint32_t n_terminals, uint32_t n_boxes,
                                       const uint32_t *box_start, const uint32_t *state_box,
                                       const uint8_t *is_final, const uint32_t *t_src,
                                       const uint32_t *t_sym, const uint32_t *t_dst,
                                       uint32_t n_trans, uint32_t start_box, cfpq_rsm *out) {
    if (!out) return fail(CFPQ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n_states == 0 || n_boxes == 0) return fail(CFPQ_ERR_INVALID, "RSM needs states and boxes");
    if (!box_start || !state_box || !is_final) return fail(CFPQ_ERR_INVALID, "RSM array is NULL");
    if (n_trans && (!t_src || !t_sym || !t_dst)) return fail(CFPQ_ERR_INVALID, "transition array is NULL");
    if (start_box >= n_boxes) return fail(CFPQ_ERR_INVALID, "start_box out of range");
    if ((uint64_t)n_terminals + n_boxes > 0xFFFFFFFFull) return fail(CFPQ_ERR_INVALID, "too many symbols");
    for (uint32_t q = 0; q < n_states; ++q)
        if (state_box[q] >= n_boxes) return fail(CFPQ_ERR_INVALID, "state_box out of range");
    for (uint32_t b = 0; b < n_boxes; ++b) {
        if (box_start[b] >= n_states) return fail(CFPQ_ERR_INVALID, "box_start out of range");
        if (state_box[box_start[b]] != b) return fail(CFPQ_ERR_INVALID, "box start owned by another box");
    }
    for (uint32_t i = 0; i < n_trans; ++i) {
        if (t_src[i] >= n_states || t_dst[i] >= n_states) return fail(CFPQ_ERR_INVALID, "transition state out of range");
        if (t_sym[i] >= n_terminals + n_boxes) return fail(CFPQ_ERR_INVALID, "transition symbol out of range");
        if (state_box[t_src[i]] != state_box[t_dst[i]]) return fail(CFPQ_ERR_INVALID, "transition crosses boxes");
    }
    std::unique_ptr<cfpq_rsm_s> r(new (std::nothrow) cfpq_rsm_s);
    if (!r) return fail(CFPQ_ERR_OOM, "host allocation failed");
    r->n_states = n_states; r->n_terms = n_terminals; r->n_boxes = n_boxes; r->start_box = start_box;
    r->box_start.assign(box_start, box_start + n_boxes);
    r->state_box.assign(state_box, state_box + n_states);
    r->is_final.resize(n_states);
    for (uint32_t q = 0; q < n_states; ++q) r->is_final[q] = is_final[q] ? 1 : 0;
    // a transition is a set element: drop duplicates
    std::vector<std::array<uint32_t, 3>> tr;
    for (uint32_t i = 0; i < n_trans; ++i) tr.push_back({t_src[i], t_sym[i], t_dst[i]});
    std::sort(tr.begin(), tr.end());
    tr.erase(std::unique(tr.begin(), tr.end()), tr.end());
    for (auto &t : tr) {
        r->t_src.push_back(t[0]); r->t_sym.push_back(t[1]); r->t_dst.push_back(t[2]);
    }
    *out = r.release();
    return CFPQ_OK;
}

extern "C" void cfpq_rsm_destroy(cfpq_rsm r) { delete r; }

// ---------------------------------------------------------------------------
// query planning shared by both strategies
// ---------------------------------------------------------------------------
namespace {

constexpr uint32_t kFusedMaxN = 2048;
constexpr uint32_t kFusedMaxBoxesHost = 64;
constexpr uint32_t kStatsCap = 4096;
constexpr uint64_t kRankMaxBytes = 64ull << 30;   // keep_rank: one byte per pair of every box

struct Plan {
    uint32_t n, Pn, P, nQ, nB, n_terms;
    std::vector<uint32_t> in_off, out_off;
    std::vector<InTrans> in_tr, out_tr;   // out_tr[.].src = target state
    bool has_calls = false;               // some transition is box-labelled
    std::vector<uint32_t> starts;     // box start per box
    std::vector<uint32_t> fin_off, fin;
    std::vector<uint32_t> eps_boxes;  // boxes whose start is final
    std::vector<uint8_t> nullable, box_used;
    std::vector<uint32_t> is_start;      // per state: initial state of its box
    std::vector<uint32_t> nt_src;        // source states of box-labelled transitions
    std::vector<uint32_t> nt_dst;        // target states of box-labelled transitions
    std::vector<uint32_t> f_box;         // per state: the box of its only box-labelled in-transition, else kNoBox
    // the transitions inside one strongly connected component of the RSM's
    // state graph, by target (sin) and by source (sout) state: the only
    // ones a cycle of the product graph can use
    std::vector<uint32_t> sin_off, sout_off;
    std::vector<InTrans> sin_tr, sout_tr;
};

// strongly connected components of the state graph (Kosaraju, iterative):
// comp[q] for every state
std::vector<uint32_t> state_components(const Plan &p) {
    const uint32_t nQ = p.nQ;
    std::vector<uint32_t> order, comp(nQ, 0xFFFFFFFFu);
    std::vector<uint8_t> seen(nQ, 0);
    std::vector<std::pair<uint32_t, uint32_t>> st;   // (state, next out-transition)
    for (uint32_t r = 0; r < nQ; ++r) {
        if (seen[r]) continue;
        seen[r] = 1;
        st.push_back({r, p.out_off[r]});
        while (!st.empty()) {
            auto &[q, t] = st.back();
            if (t < p.out_off[q + 1]) {
                const uint32_t x = p.out_tr[t++].src;   // out_tr: target state in .src
                if (!seen[x]) {
                    seen[x] = 1;
                    st.push_back({x, p.out_off[x]});
                }
            } else {
                order.push_back(q);
                st.pop_back();
            }
        }
    }
    uint32_t nc = 0;
    std::vector<uint32_t> stack;
    for (size_t i = order.size(); i-- > 0;) {
        const uint32_t r = order[i];
        if (comp[r] != 0xFFFFFFFFu) continue;
        comp[r] = nc;
        stack.push_back(r);
        while (!stack.empty()) {
            const uint32_t q = stack.back();
            stack.pop_back();
            for (uint32_t t = p.in_off[q]; t < p.in_off[q + 1]; ++t) {
                const uint32_t x = p.in_tr[t].src;
                if (comp[x] == 0xFFFFFFFFu) {
                    comp[x] = nc;
                    stack.push_back(x);
                }
            }
        }
        ++nc;
    }
    return comp;
}

Plan make_plan(const cfpq_graph_s &g, const cfpq_rsm_s &r) {
    Plan p;
    p.n = g.n;
    p.Pn = (g.n + 63) / 64;
    p.P = row_pitch(p.Pn);
    p.nQ = r.n_states;
    p.nB = r.n_boxes;
    p.n_terms = r.n_terms;
    p.in_off.assign(p.nQ + 1, 0);
    for (size_t i = 0; i < r.t_src.size(); ++i) p.in_off[r.t_dst[i] + 1]++;
    for (uint32_t q = 0; q < p.nQ; ++q) p.in_off[q + 1] += p.in_off[q];
    p.in_tr.resize(r.t_src.size());
    std::vector<uint32_t> fill(p.in_off.begin(), p.in_off.end() - 1);
    for (size_t i = 0; i < r.t_src.size(); ++i) p.in_tr[fill[r.t_dst[i]]++] = InTrans{r.t_src[i], r.t_sym[i]};
    p.out_off.assign(p.nQ + 1, 0);
    for (size_t i = 0; i < r.t_src.size(); ++i) p.out_off[r.t_src[i] + 1]++;
    for (uint32_t q = 0; q < p.nQ; ++q) p.out_off[q + 1] += p.out_off[q];
    p.out_tr.resize(r.t_src.size());
    std::vector<uint32_t> ofill(p.out_off.begin(), p.out_off.end() - 1);
    for (size_t i = 0; i < r.t_src.size(); ++i) p.out_tr[ofill[r.t_src[i]]++] = InTrans{r.t_dst[i], r.t_sym[i]};
    for (size_t i = 0; i < r.t_sym.size(); ++i) p.has_calls |= r.t_sym[i] >= r.n_terms;
    {
        std::vector<uint8_t> seen(p.nQ, 0), seen_dst(p.nQ, 0);
        for (size_t i = 0; i < r.t_sym.size(); ++i) {
            if (r.t_sym[i] < r.n_terms) continue;
            if (!seen[r.t_src[i]]) {
                seen[r.t_src[i]] = 1;
                p.nt_src.push_back(r.t_src[i]);
            }
            if (!seen_dst[r.t_dst[i]]) {
                seen_dst[r.t_dst[i]] = 1;
                p.nt_dst.push_back(r.t_dst[i]);
            }
        }
    }
    p.starts = r.box_start;
    p.is_start.assign(p.nQ, 0);
    for (uint32_t b = 0; b < p.nB; ++b) p.is_start[r.box_start[b]] = 1;
    p.fin_off.assign(p.nB + 1, 0);
    for (uint32_t q = 0; q < p.nQ; ++q)
        if (r.is_final[q]) p.fin_off[r.state_box[q] + 1]++;
    for (uint32_t b = 0; b < p.nB; ++b) p.fin_off[b + 1] += p.fin_off[b];
    p.fin.resize(p.fin_off[p.nB]);
    std::vector<uint32_t> ff(p.fin_off.begin(), p.fin_off.end() - 1);
    for (uint32_t q = 0; q < p.nQ; ++q)
        if (r.is_final[q]) p.fin[ff[r.state_box[q]]++] = q;
    p.nullable.assign(p.nB, 0);
    p.box_used.assign(p.nB, 0);
    for (uint32_t b = 0; b < p.nB; ++b)
        if (r.is_final[r.box_start[b]]) {
            p.nullable[b] = 1;
            p.eps_boxes.push_back(b);
        }
    for (size_t i = 0; i < r.t_sym.size(); ++i)
        if (r.t_sym[i] >= r.n_terms) p.box_used[r.t_sym[i] - r.n_terms] = 1;
    p.f_box.assign(p.nQ, kNoBox);
    {
        std::vector<uint32_t> calls(p.nQ, 0);
        for (size_t i = 0; i < r.t_sym.size(); ++i)
            if (r.t_sym[i] >= r.n_terms) {
                calls[r.t_dst[i]]++;
                p.f_box[r.t_dst[i]] = r.t_sym[i] - r.n_terms;
            }
        for (uint32_t q = 0; q < p.nQ; ++q)
            if (calls[q] != 1) p.f_box[q] = kNoBox;
    }
    {
        const std::vector<uint32_t> comp = state_components(p);
        p.sin_off.assign(p.nQ + 1, 0);
        p.sout_off.assign(p.nQ + 1, 0);
        for (uint32_t q = 0; q < p.nQ; ++q) {
            for (uint32_t t = p.in_off[q]; t < p.in_off[q + 1]; ++t)
                if (comp[p.in_tr[t].src] == comp[q]) p.sin_tr.push_back(p.in_tr[t]);
            for (uint32_t t = p.out_off[q]; t < p.out_off[q + 1]; ++t)
                if (comp[p.out_tr[t].src] == comp[q]) p.sout_tr.push_back(p.out_tr[t]);
            p.sin_off[q + 1] = (uint32_t)p.sin_tr.size();
            p.sout_off[q + 1] = (uint32_t)p.sout_tr.size();
        }
    }
    return p;
}

// device copy of the small per-query tables
struct Tables {
    DevBuf buf;
    uint32_t *in_off = nullptr, *starts = nullptr, *fin_off = nullptr, *fin = nullptr,
             *eps = nullptr, *out_off = nullptr, *is_start = nullptr, *nt_src = nullptr, *nt_dst = nullptr,
             *f_box = nullptr, *sin_off = nullptr, *sout_off = nullptr;
    InTrans *in_tr = nullptr, *out_tr = nullptr, *sin_tr = nullptr, *sout_tr = nullptr;
    uint8_t *nullable = nullptr, *box_used = nullptr;
};

// the tables packed into one host block (16-byte aligned parts) and the
// offset of each part in it
struct TableImage {
    std::vector<uint8_t> host;
    size_t in_off, in_tr, starts, fin_off, fin, eps, nullable, box_used, out_off, out_tr, is_start, nt_src, nt_dst,
        f_box, sin_off, sin_tr, sout_off, sout_tr;
};

void pack_tables(const Plan &p, TableImage &im) {
    std::vector<uint8_t> &host = im.host;
    host.clear();
    auto put = [&](const void *src, size_t bytes) {
        size_t at = (host.size() + 15) / 16 * 16;
        host.resize(at + bytes + 16);
        if (bytes) std::memcpy(host.data() + at, src, bytes);
        return at;
    };
    im.in_off = put(p.in_off.data(), p.in_off.size() * 4);
    im.in_tr = put(p.in_tr.data(), p.in_tr.size() * sizeof(InTrans));
    im.starts = put(p.starts.data(), p.starts.size() * 4);
    im.fin_off = put(p.fin_off.data(), p.fin_off.size() * 4);
    im.fin = put(p.fin.data(), p.fin.size() * 4);
    im.eps = put(p.eps_boxes.data(), p.eps_boxes.size() * 4);
    im.nullable = put(p.nullable.data(), p.nullable.size());
    im.box_used = put(p.box_used.data(), p.box_used.size());
    im.out_off = put(p.out_off.data(), p.out_off.size() * 4);
    im.out_tr = put(p.out_tr.data(), p.out_tr.size() * sizeof(InTrans));
    im.is_start = put(p.is_start.data(), p.is_start.size() * 4);
    im.nt_src = put(p.nt_src.data(), p.nt_src.size() * 4);
    im.nt_dst = put(p.nt_dst.data(), p.nt_dst.size() * 4);
    im.f_box = put(p.f_box.data(), p.f_box.size() * 4);
    im.sin_off = put(p.sin_off.data(), p.sin_off.size() * 4);
    im.sin_tr = put(p.sin_tr.data(), p.sin_tr.size() * sizeof(InTrans));
    im.sout_off = put(p.sout_off.data(), p.sout_off.size() * 4);
    im.sout_tr = put(p.sout_tr.data(), p.sout_tr.size() * sizeof(InTrans));
}

// table pointers into a device copy of the image at b
void bind_tables(const TableImage &im, uint8_t *b, Tables &t) {
    t.in_off = (uint32_t *)(b + im.in_off);
    t.in_tr = (InTrans *)(b + im.in_tr);
    t.starts = (uint32_t *)(b + im.starts);
    t.fin_off = (uint32_t *)(b + im.fin_off);
    t.fin = (uint32_t *)(b + im.fin);
    t.eps = (uint32_t *)(b + im.eps);
    t.nullable = b + im.nullable;
    t.box_used = b + im.box_used;
    t.out_off = (uint32_t *)(b + im.out_off);
    t.out_tr = (InTrans *)(b + im.out_tr);
    t.is_start = (uint32_t *)(b + im.is_start);
    t.nt_src = (uint32_t *)(b + im.nt_src);
    t.nt_dst = (uint32_t *)(b + im.nt_dst);
    t.f_box = (uint32_t *)(b + im.f_box);
    t.sin_off = (uint32_t *)(b + im.sin_off);
    t.sin_tr = (InTrans *)(b + im.sin_tr);
    t.sout_off = (uint32_t *)(b + im.sout_off);
    t.sout_tr = (InTrans *)(b + im.sout_tr);
}

cfpq_status upload_tables(const Plan &p, const Alloc *al, hipStream_t s, Tables &t) {
    TableImage im;
    pack_tables(p, im);
    if (!t.buf.alloc(al, im.host.size(), s)) return fail(CFPQ_ERR_OOM, "device allocation failed (tables)");
    HIP_TRY(hipMemcpyAsync(t.buf.p, im.host.data(), im.host.size(), hipMemcpyHostToDevice, s));
    bind_tables(im, t.buf.as<uint8_t>(), t);
    // the host image dies with this frame: wait for the copy
    HIP_TRY(hipStreamSynchronize(s));
    return CFPQ_OK;
}

cfpq_status check_pair(const cfpq_graph_s *g, const cfpq_rsm_s *r) {
    if (!g || !r) return fail(CFPQ_ERR_INVALID, "graph or RSM is NULL");
    if (r->n_terms > g->n_labels)
        return fail(CFPQ_ERR_INVALID, "RSM uses more terminals than the graph has labels");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != g->device) return fail(CFPQ_ERR_INVALID, "graph lives on another device");
    return CFPQ_OK;
}

// Pinned host buffers for counter read-backs, kept in a process-wide pool:
// allocating and freeing pinned memory per query costs more than a small
// query's kernels.  The pool holds at most one buffer per query that ran at
// the same time and keeps them until the process ends (it is never torn
// down, so no HIP call runs during static destruction).
class PinnedPool {
    std::mutex m_;
    std::vector<std::pair<unsigned long long *, size_t>> free_;

  public:
    static PinnedPool &get() {
        static PinnedPool *pool = new PinnedPool;
        return *pool;
    }
    bool take(size_t n, unsigned long long *&h, size_t &cap) {
        {
            std::lock_guard<std::mutex> lk(m_);
            for (size_t i = 0; i < free_.size(); ++i)
                if (free_[i].second >= n) {
                    h = free_[i].first;
                    cap = free_[i].second;
                    free_[i] = free_.back();
                    free_.pop_back();
                    return true;
                }
        }
        unsigned long long *p = nullptr;
        if (hipHostMalloc((void **)&p, n * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
            return false;
        h = p;
        cap = n;
        return true;
    }
    void put(unsigned long long *h, size_t cap) {
        std::lock_guard<std::mutex> lk(m_);
        free_.emplace_back(h, cap);
    }
};

struct PinnedCounters {
    unsigned long long *h = nullptr;
    size_t cap = 0;
    ~PinnedCounters() {
        if (h) PinnedPool::get().put(h, cap);
    }
    bool ensure(size_t n) {
        if (n <= cap) return true;
        if (h) PinnedPool::get().put(h, cap);
        h = nullptr;
        cap = 0;
        return PinnedPool::get().take(n, h, cap);
    }
};

// HIP events in a process-wide pool per device, like the pinned buffers:
// creating and destroying a query's events costs more than recording them
class EventPool {
    std::mutex m_;
    std::vector<std::pair<int, hipEvent_t>> free_;

  public:
    static EventPool &get() {
        static EventPool *pool = new EventPool;
        return *pool;
    }
    hipError_t take(int dev, hipEvent_t &e) {
        {
            std::lock_guard<std::mutex> lk(m_);
            for (size_t i = 0; i < free_.size(); ++i)
                if (free_[i].first == dev) {
                    e = free_[i].second;
                    free_[i] = free_.back();
                    free_.pop_back();
                    return hipSuccess;
                }
        }
        return hipEventCreate(&e);
    }
    void put(int dev, hipEvent_t e) {
        std::lock_guard<std::mutex> lk(m_);
        free_.emplace_back(dev, e);
    }
};

// a query's events, back to the pool when the query ends
struct PooledEvents {
    int dev = 0;
    std::vector<hipEvent_t> v;
    ~PooledEvents() {
        for (hipEvent_t e : v) EventPool::get().put(dev, e);
    }
    hipError_t ensure(size_t k) {
        if (v.empty()) (void)hipGetDevice(&dev);
        while (v.size() < k) {
            hipEvent_t e = nullptr;
            hipError_t er = EventPool::get().take(dev, e);
            if (er != hipSuccess) return er;
            v.push_back(e);
        }
        return hipSuccess;
    }
};

uint64_t *d_u64(const DevBuf &b) { return b.as<uint64_t>(); }

// Wait for the stream's work: poll it for up to CFPQ_SPIN_US microseconds
// (a query's last read-back is usually done within that), then block.
#ifndef CFPQ_SPIN_US
#define CFPQ_SPIN_US 2000
#endif
hipError_t wait_stream(hipStream_t s) {
    if (CFPQ_SPIN_US > 0) {
        const auto t0 = std::chrono::steady_clock::now();
        for (;;) {
            const hipError_t e = hipStreamQuery(s);
            if (e != hipErrorNotReady) return e;
            if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(CFPQ_SPIN_US)) break;
        }
    }
    return hipStreamSynchronize(s);
}

bool max_iters_hit(const cfpq_query_opts &o, uint32_t it) { return o.max_iters && it > o.max_iters; }

uint32_t gather_grid(uint64_t rows) {
    uint64_t blocks = (rows + (kBlock / kWave) - 1) / (kBlock / kWave);
    const uint64_t cap = 256 * 16;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    return (uint32_t)blocks;
}

// ---------------------------------------------------------------------------
// LEVELS strategy: one launch per closure level, any graph size
// ---------------------------------------------------------------------------
cfpq_status run_levels(const cfpq_graph_s &g, const cfpq_rsm_s &r, const cfpq_query_opts &o,
                       cfpq_result_s &res) {
    hipStream_t s = (hipStream_t)o.stream;
    const Alloc *al = &res.alloc;
    Plan p = make_plan(g, r);
    Tables tb;
    cfpq_status st = upload_tables(p, al, s, tb);
    if (st != CFPQ_OK) return st;

    const uint32_t n = p.n, P = p.P, Pn = p.Pn, nQ = p.nQ, nB = p.nB;
    const uint64_t qw = (uint64_t)nQ * n * P, bw = (uint64_t)nB * n * P;
    // source tile: given, or the widest that fits -- at most kSparseMaxWords
    // words when the sparse nonterminal product applies (it keeps a tile row
    // in LDS), and within the device memory left once the closure (T), the
    // nonterminal matrices and the indexes are placed; the frontier buffers
    // (two, plus the product rows) take 3 nQ n words per word of tile
    uint32_t G = Pn;
    if (o.tile_words) {
        G = std::min<uint32_t>(o.tile_words, Pn);
    } else {
        // with box-labelled transitions, narrower tiles also keep more
        // frontier rows within an ELL list (fewer whole-row ORs), wider ones
        // run fewer passes: measured best near 1600 words, so tiles of at most
        // kTileCapWords, equal
        if (!p.nt_src.empty() && o.nt_mode != CFPQ_NT_ROWS) G = std::min<uint32_t>(G, kTileCapWords);
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
            free_b += al->cached();   // a caching allocator's free blocks are free for this query too
            const double fixed = 8.0 * ((double)qw + 2.0 * (double)bw) + 4.0 * nQ * (double)n * (kEll + 1) +
                                 16.0 * nB * (double)n * ((Pn + 63) / 64) + (o.keep_rank ? (double)nB * n * n : 0.0) +
                                 (256.0 * (1 << 20));
            const double per_word = 8.0 * 3.0 * nQ * (double)n;
            const double room = 0.92 * (double)free_b - fixed;
            if (room < per_word * G) G = room >= per_word ? (uint32_t)(room / per_word) : 1u;
        }
        if (G == 0) G = 1;
        const uint32_t tiles = (Pn + G - 1) / G;
        G = (Pn + tiles - 1) / tiles;   // equal tiles rather than a ragged last one
    }
    if (G == 0) G = 1;
    const uint32_t groups = (Pn + G - 1) / G;
    const uint64_t fw = (uint64_t)nQ * n * G;
    const uint64_t aw = (uint64_t)nQ * Pn;
    const uint64_t ring_words = (uint64_t)kRingSlots * kSlotWords;
    // row summaries (selector rows) and coarse frontier activity: one bit per
    // word of a row, sum_pitch words per row; a frontier's coarse activity
    // array follows its row bitset, Pbs = sum_pitch + 1 words per state (the
    // last one flags "any active row")
    const uint32_t sum_pitch = (Pn + kWave - 1) / kWave;
    const uint32_t Pbs = sum_pitch + 1;
    const uint64_t ab = (uint64_t)nQ * Pbs, aset = aw + ab;

    DevBuf T, dNT, D0, D1, acts, tnz, dnt_act, ctr, ell, chg_buf, nsum, dense_buf;
    // sparse nonterminal product in the seed: ELL lists of the source rows and
    // an LDS row accumulator per wavefront (tiles up to kSparseMaxWords words)
    const bool sparse_nt = !p.nt_src.empty() && G <= kSparseMaxWords && o.nt_mode != CFPQ_NT_ROWS;
    // counts [nQ n] (padded to 4 entries), then the lists, 128-byte aligned
    // (the product loads them 16 bytes at a time)
    const uint64_t ell_pad = ((uint64_t)nQ * n + 31) / 32 * 32;
    if (sparse_nt && !ell.alloc(al, (ell_pad + (uint64_t)nQ * n * kEll) * 4, s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (sparse product index)");
    // source rows with more than kEll bits go through the LDS-blocked dense
    // product: their bitset [nQ][Pn] and its coarse array [nQ][Pbs]
    const uint64_t dense_words = (uint64_t)nQ * Pn + (uint64_t)nQ * ((Pn + kWave - 1) / kWave + 1);
    if (sparse_nt && !dense_buf.alloc(al, dense_words * 8, s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (dense rows)");
    if (!T.alloc(al, qw * 8, s) || !res.NT.alloc(al, bw * 8, s) || !dNT.alloc(al, bw * 8, s) ||
        !D0.alloc(al, fw * 8, s) || !D1.alloc(al, fw * 8, s) || !acts.alloc(al, 3 * aset * 8, s) ||
        !tnz.alloc(al, aw * 8, s) || !dnt_act.alloc(al, 2ull * nB * Pn * 8, s) ||
        !ctr.alloc(al, ring_words * 8, s) || !chg_buf.alloc(al, aw * 8, s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (query state)");
    // summary of the nonterminal matrices' rows (selectors of the closure
    // levels), kept up to date for the rows each write-back changes
    const bool use_nsum = p.has_calls;
    if (use_nsum && !nsum.alloc(al, (uint64_t)nB * n * sum_pitch * 8, s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (selector summary)");
    if (o.keep_rank) {
        if (!res.rank.alloc(al, (uint64_t)nB * n * n, s)) return fail(CFPQ_ERR_OOM, "device allocation failed (rank)");
        HIP_TRY(hipMemsetAsync(res.rank.p, 0xFF, (uint64_t)nB * n * n, s));  // 0xFF = absent
    }
    uint64_t *d_T = T.as<uint64_t>(), *d_NT = res.NT.as<uint64_t>(), *d_dNT = dNT.as<uint64_t>();
    uint64_t *Dbuf[2] = {D0.as<uint64_t>(), D1.as<uint64_t>()};
    uint64_t *act[3] = {acts.as<uint64_t>(), acts.as<uint64_t>() + aset, acts.as<uint64_t>() + 2 * aset};
    uint64_t *blk[3] = {act[0] + aw, act[1] + aw, act[2] + aw};
    // new-edge activity of dNT: dact[cur] belongs to the current dNT (read by
    // the next seed), the other one is written by the next write-back
    uint64_t *dact[2] = {dnt_act.as<uint64_t>(), dnt_act.as<uint64_t>() + (uint64_t)nB * Pn};
    uint32_t cur = 0;
    uint64_t *d_chg = chg_buf.as<uint64_t>();
    unsigned long long *d_ctr = ctr.as<unsigned long long>();

    // events: [0] start, [1] end; profiling pool after that
    std::vector<hipEvent_t> ev;
    struct EvGuard {
        std::vector<hipEvent_t> *v;
        ~EvGuard() {
            for (hipEvent_t e : *v) (void)hipEventDestroy(e);
        }
    } evg{&ev};
    auto event = [&](size_t i) -> hipEvent_t {
        while (ev.size() <= i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev.push_back(e);
        }
        return ev[i];
    };
    if (!event(1)) return fail(CFPQ_ERR_DEVICE, "hipEventCreate failed");
    const bool prof = o.profile != 0;
    res.profiled = prof;
    // launch timing: event before each launch of a chunk plus one after it
    auto prof_mark = [&](uint32_t j) -> cfpq_status {
        if (!prof) return CFPQ_OK;
        hipEvent_t e = event(2 + j);
        if (!e) return fail(CFPQ_ERR_DEVICE, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e, s));
        return CFPQ_OK;
    };
    auto prof_ms = [&](uint32_t j) -> double {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2 + j], ev[3 + j]) != hipSuccess) return 0.0;
        return ms;
    };
    // three marks per closure launch j (the seed, or one level): before its
    // ELL build, before its nonterminal product (sparse or matrix cores) and
    // before its gather; the gather ends at mark (j + 1, 0).  Every kernel is
    // bracketed by marks of its own, so a kind's time is its kernels' time.
    auto prof_mark3 = [&](uint32_t j, int which) -> cfpq_status {
        if (!prof) return CFPQ_OK;
        hipEvent_t e = event(2 + 4 * j + (uint32_t)which);
        if (!e) return fail(CFPQ_ERR_DEVICE, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e, s));
        return CFPQ_OK;
    };
    // marks per group: 0 before the ELL build, 1 before the sparse (or
    // matrix-core) product, 3 before the dense product, 2 before the gather
    auto ev3 = [](uint32_t j, int which) -> size_t { return 2 + 4 * (size_t)j + (size_t)which; };
    auto prof_span = [&](size_t i0, size_t i1) -> double {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[i0], ev[i1]) != hipSuccess) return 0.0;
        return ms;
    };
    // profiling counters: matrix-core instructions issued, bytes of the
    // sparse products, write-back rows visited per box
    DevBuf mops;
    unsigned long long *mfma_ops = nullptr, *sp_bytes = nullptr, *wb_rows = nullptr, *dn_bytes = nullptr;
    if (prof) {
        if (!mops.alloc(al, (3 + (uint64_t)nB) * 8, s))
            return fail(CFPQ_ERR_OOM, "device allocation failed (profile counters)");
        mfma_ops = mops.as<unsigned long long>();
        sp_bytes = mfma_ops + 1;
        dn_bytes = mfma_ops + 2;
        wb_rows = mfma_ops + 3;
        HIP_TRY(launch_fill((uint64_t *)mfma_ops, 3 + (uint64_t)nB, 0, s));
    }
    uint64_t *d_dns = dense_buf.as<uint64_t>(), *d_dblk = d_dns ? d_dns + (uint64_t)nQ * Pn : nullptr;
    DenseArgs dargs{};
    dargs.dns = d_dns; dargs.dblk = d_dblk; dargs.nt_dst = tb.nt_dst; dargs.n_nt_dst = (uint32_t)p.nt_dst.size();
    dargs.ell_idx = sparse_nt ? ell.as<uint32_t>() + ell_pad : nullptr;
    // the dense product: ELL build marks dense rows, the sparse product leaves
    // them, the dense product ORs them in; a.bytes_ctr is the sparse one's
    auto dense_product = [&](GatherArgs &ga, uint64_t *extra, const uint64_t *extra_act) -> cfpq_status {
        dargs.extra = extra; dargs.extra_act = extra_act;
        GatherArgs gd = ga;
        gd.bytes_ctr = dn_bytes;
        HIP_TRY(launch_nt_dense(gd, dargs, s));
        return CFPQ_OK;
    };
    DevBuf Dx, xact;   // matrix-core product rows and their activity, allocated on first use

    HIP_TRY(hipEventRecord(ev[0], s));
    HIP_TRY(launch_fill(d_T, qw, 0, s));
    HIP_TRY(launch_fill(d_NT, bw, 0, s));
    HIP_TRY(launch_fill(d_dNT, bw, 0, s));
    HIP_TRY(launch_fill(tnz.as<uint64_t>(), aw, 0, s));
    HIP_TRY(launch_fill(dnt_act.as<uint64_t>(), 2ull * nB * Pn, 0, s));
    HIP_TRY(launch_fill((uint64_t *)d_ctr, ring_words, 0, s));
    HIP_TRY(launch_seed_diag(d_T, tnz.as<uint64_t>(), n, P, Pn, tb.starts, nB, res.src_mask.as<uint64_t>(), s));
    HIP_TRY(launch_eps(d_NT, d_dNT, dact[cur], o.keep_rank ? res.rank.as<uint8_t>() : nullptr, n, P,
                       Pn, tb.eps, (uint32_t)p.eps_boxes.size(), s));
    if (use_nsum) {
        HIP_TRY(launch_fill(nsum.as<uint64_t>(), (uint64_t)nB * n * sum_pitch, 0, s));
        HIP_TRY(launch_row_summary(d_NT, nB, n, P, Pn, dact[cur], nsum.as<uint64_t>(), sum_pitch, s));
    }
    // the seed's selectors (new nonterminal edges) are scanned once per source
    // tile: with long rows, a summary of their non-zero words, rebuilt after
    // every write-back, lets the scan skip the empty blocks
    DevBuf dsum;
    const bool use_sum = sparse_nt;
    if (use_sum) {
        if (!dsum.alloc(al, (uint64_t)nB * n * sum_pitch * 8, s))
            return fail(CFPQ_ERR_OOM, "device allocation failed (selector summary)");
        // zero first: the write-back rewrites a row's summary only in the
        // blocks it visits
        HIP_TRY(launch_fill(dsum.as<uint64_t>(), (uint64_t)nB * n * sum_pitch, 0, s));
        HIP_TRY(launch_row_summary(d_dNT, nB, n, P, Pn, dact[cur], dsum.as<uint64_t>(), sum_pitch, s));
    }

    std::vector<uint64_t> box_delta(nB, 0);
    for (uint32_t b : p.eps_boxes) box_delta[b] = n;
    // from-scratch closure per iteration (the evaluated variant): the seed
    // takes every edge of M2, all rows selectable
    const bool scratch = o.recompute != 0;
    DevBuf ones;
    if (scratch) {
        if (!ones.alloc(al, (uint64_t)nB * Pn * 8, s)) return fail(CFPQ_ERR_OOM, "device allocation failed");
        HIP_TRY(launch_fill(ones.as<uint64_t>(), (uint64_t)nB * Pn, ~0ull, s));
    }
    // seed deduplication (incremental closure with the sparse product): after
    // each write-back, classes of equal new-edge rows; in the next seed only
    // one row per class computes the product of a target state with a single
    // box-labelled in-transition, the others read its row
#ifndef CFPQ_SEED_DEDUP
#define CFPQ_SEED_DEDUP 1
#endif
    bool dedup = CFPQ_SEED_DEDUP && sparse_nt && use_sum && !scratch && (uint64_t)nB * n < (1ull << 31);
    if (dedup) {
        bool any_box = false;
        for (uint32_t f : p.f_box) any_box |= f != kNoBox;
        dedup = any_box;
    }
    DevBuf dd_buf;
    uint64_t dd_mask = 0;
    uint64_t *dd_hash = nullptr;
    uint32_t *dd_rep = nullptr, *dd_vals = nullptr;
    unsigned long long *dd_keys = nullptr;
    bool rep_valid = false;   // dd_rep holds the classes of the current dNT rows
    if (dedup) {
        const uint64_t rows = (uint64_t)nB * n;
        uint64_t slots = 2;
        while (slots < 2 * rows) slots <<= 1;
        dd_mask = slots - 1;
        // hashes [rows] u64, table keys [slots] u64, values [slots] u32, reps [rows] u32
        const uint64_t words = rows + slots + slots / 2 + (rows + 1) / 2;
        if (!dd_buf.alloc(al, words * 8, s)) return fail(CFPQ_ERR_OOM, "device allocation failed (seed classes)");
        dd_hash = dd_buf.as<uint64_t>();
        dd_keys = (unsigned long long *)(dd_hash + rows);
        dd_vals = (uint32_t *)(dd_hash + rows + slots);
        dd_rep = (uint32_t *)(dd_hash + rows + slots + slots / 2);
    }

    // The seed's ELL lists of the closure rows, kept per source tile across
    // iterations: a row's list is rebuilt only if the row gained bits since
    // the last build (the previous iteration's change bitset).  Closure rows
    // only grow, so a row found dense stays dense.  (Not with the recomputed
    // closure, which clears T every iteration.)
#ifndef CFPQ_SEED_ELL_KEEP
#define CFPQ_SEED_ELL_KEEP 1
#endif
    auto al256b = [](uint64_t x) { return (x + 255) / 256 * 256; };
    const uint64_t seed_ell_bytes = al256b((ell_pad + (uint64_t)nQ * n * kEll) * 4);
    const uint64_t seed_tile_bytes = seed_ell_bytes + al256b(dense_words * 8);
    bool keep_ell = CFPQ_SEED_ELL_KEEP && sparse_nt && !scratch && (uint64_t)groups * seed_tile_bytes <= (8ull << 30);
    // changed blocks: the gathers mark per T row the blocks of blk_words
    // words that gained bits (at most 64 blocks a row), the write-back keeps
    // per dNT row the blocks holding bits, and visits only those blocks
#ifndef CFPQ_WB_BLOCKS
#define CFPQ_WB_BLOCKS 1
#endif
    const bool wb_blocks = CFPQ_WB_BLOCKS != 0;
    uint32_t blk_shift = 6;   // blocks of 2^blk_shift words, at most 64 of them a row
    while (((uint64_t)Pn + (1ull << blk_shift) - 1) >> blk_shift > 64) ++blk_shift;
    const uint32_t blk_words = 1u << blk_shift;
    DevBuf blk_buf;
    if (wb_blocks && !blk_buf.alloc(al, ((uint64_t)nQ * n + (uint64_t)nB * n) * 8, s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (changed blocks)");
    uint64_t *d_chgb = wb_blocks ? blk_buf.as<uint64_t>() : nullptr;
    uint64_t *d_dnb = wb_blocks ? d_chgb + (uint64_t)nQ * n : nullptr;
    if (wb_blocks) HIP_TRY(launch_fill(d_dnb, (uint64_t)nB * n, 0, s));
    DevBuf seed_buf, chg_prev_buf;
    if (keep_ell && (!seed_buf.alloc(al, groups * seed_tile_bytes, s) || !chg_prev_buf.alloc(al, aw * 8, s)))
        return fail(CFPQ_ERR_OOM, "device allocation failed (seed lists)");
    uint64_t *d_chg_prev = chg_prev_buf.as<uint64_t>();
    auto seed_tile = [&](uint32_t gi, uint32_t *&cnt, uint32_t *&idx, uint64_t *&dns, uint64_t *&dblk) {
        uint8_t *b = seed_buf.as<uint8_t>() + (uint64_t)gi * seed_tile_bytes;
        cnt = (uint32_t *)b;
        idx = cnt + ell_pad;
        dns = (uint64_t *)(b + seed_ell_bytes);
        dblk = dns + (uint64_t)nQ * Pn;
    };

    PinnedCounters pc;
    if (!pc.ensure(4096 * kSlotWords)) return fail(CFPQ_ERR_OOM, "pinned host allocation failed");
    uint32_t slot = 0;
    // every slot a launch may use must read zero before the launch; the ring
    // is cleared whole when it would wrap (only at points where the previous
    // launch is known to have run, see below)
    auto need_slots = [&](uint32_t k) -> cfpq_status {
        if (slot + k >= kRingSlots) {
            HIP_TRY(launch_fill((uint64_t *)d_ctr, ring_words, 0, s));
            slot = 0;
        }
        return CFPQ_OK;
    };
    auto fetch = [&](uint32_t first, uint32_t k) -> cfpq_status {
        if (!pc.ensure((size_t)k * kSlotWords)) return fail(CFPQ_ERR_OOM, "pinned host allocation failed");
        HIP_TRY(hipMemcpyAsync(pc.h, d_ctr + (uint64_t)first * kSlotWords, (size_t)k * kSlotWords * 8,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(wait_stream(s));
        return CFPQ_OK;
    };

    const uint32_t grid = gather_grid((uint64_t)nQ * n);
    uint32_t levels_hint = 16;
    uint32_t it = 0;
    res.deltas.clear();
    for (;;) {
        ++it;
        if (o.max_iters && it > o.max_iters)
            return fail(CFPQ_ERR_LIMIT, "fixpoint did not stop within max_iters iterations");
        bool can_seed = (it == 1);
        for (uint32_t b = 0; b < nB; ++b) can_seed |= (box_delta[b] && p.box_used[b]);
        if (!can_seed) {
            res.deltas.push_back(0);
            break;
        }
        if (keep_ell) std::swap(d_chg, d_chg_prev);   // the last iteration's changes pick the lists to rebuild
        HIP_TRY(launch_fill(d_chg, aw, 0, s));   // rows gaining bits in this iteration
        if (wb_blocks) HIP_TRY(launch_fill(d_chgb, (uint64_t)nQ * n, 0, s));   // and their blocks
        if (scratch && it > 1) {   // forget the closure: only the box-start rows' own bits
            HIP_TRY(launch_fill(d_T, qw, 0, s));
            HIP_TRY(launch_fill(tnz.as<uint64_t>(), aw, 0, s));
            HIP_TRY(launch_seed_diag(d_T, tnz.as<uint64_t>(), n, P, Pn, tb.starts, nB, res.src_mask.as<uint64_t>(),
                                     s));
        }
        for (uint32_t gi = 0; gi < groups; ++gi) {
            const uint32_t w0 = gi * G, gw = std::min(G, Pn - w0);
            HIP_TRY(launch_fill(act[0], 3 * aset, 0, s));
            GatherArgs a{};
            a.n = n; a.P = P; a.Pn = Pn; a.n_terms = p.n_terms; a.nQ = nQ;
            a.w0 = w0; a.gw = gw; a.G = G;
            a.goff = g.off.as<uint32_t>(); a.gidx = g.idx.as<uint32_t>();
            a.in_off = tb.in_off; a.in_tr = tb.in_tr;
            a.T = d_T; a.tnz = tnz.as<uint64_t>(); a.ctr = d_ctr; a.clear_words = (uint32_t)aset;
            a.Pbs = Pbs; a.chg = d_chg;
            a.chgb = d_chgb; a.blk_shift = blk_shift;
            // Kronecker product of the RSM with the new edges (seed); the seed
            // and the first chunk of levels always fit before a ring clear
            if ((st = need_slots(levels_hint + 2)) != CFPQ_OK) return st;
            a.sel = scratch ? d_NT : d_dNT; a.sel_act = scratch ? ones.as<uint64_t>() : dact[cur];
            a.sel_sum = scratch ? (use_nsum ? nsum.as<uint64_t>() : nullptr) : (use_sum ? dsum.as<uint64_t>() : nullptr);
            a.sum_pitch = sum_pitch;
            a.src = d_T; a.src_pitch = P; a.src_off = w0; a.src_act = tnz.as<uint64_t>();
            a.src_blk = nullptr;   // closure rows as sources: no coarse activity kept
            a.dn = Dbuf[0]; a.actn = act[0]; a.actn_blk = blk[0]; a.act_clear = nullptr;
            a.slot_prev = kNoSlot; a.slot_cur = slot; a.seed_terms = (it == 1) || scratch;
            a.extra = nullptr; a.extra_act = nullptr; a.bytes_ctr = sp_bytes;
            a.dense_apart = sparse_nt ? 1u : 0u;
            a.rep = rep_valid ? dd_rep : nullptr; a.f_box = tb.f_box;
            if ((st = prof_mark3(0, 0)) != CFPQ_OK) return st;
            if (sparse_nt) {
                // the product rows go to the other frontier buffer and the third
                // activity bitset, both unused until the first level
                uint32_t *ell_cnt = ell.as<uint32_t>(), *ell_idx = ell_cnt + ell_pad;
                uint64_t *sdns = d_dns, *sdblk = d_dblk;
                const uint64_t *rebuild = nullptr;   // null: every row's list
                if (keep_ell) {
                    seed_tile(gi, ell_cnt, ell_idx, sdns, sdblk);
                    if (it > 1) rebuild = d_chg_prev;
                }
                if (!rebuild) HIP_TRY(launch_fill(sdns, dense_words, 0, s));
                HIP_TRY(launch_ell_build_dense(d_T, P, w0, gw, n, tb.nt_src, (uint32_t)p.nt_src.size(), ell_cnt,
                                               ell_idx, rebuild, Pn, nullptr, sdns, sdblk, Pbs, s));
                if ((st = prof_mark3(0, 1)) != CFPQ_OK) return st;
                HIP_TRY(launch_nt_sparse(a, ell_cnt, ell_idx, Dbuf[1], act[2], grid, s));
                if ((st = prof_mark3(0, 3)) != CFPQ_OK) return st;
                dargs.dns = sdns; dargs.dblk = sdblk; dargs.ell_idx = ell_idx;
                st = dense_product(a, Dbuf[1], act[2]);
                dargs.dns = d_dns; dargs.dblk = d_dblk; dargs.ell_idx = ell.as<uint32_t>() + ell_pad;
                if (st != CFPQ_OK) return st;
                a.extra = Dbuf[1]; a.extra_act = act[2];
            } else {
                if ((st = prof_mark3(0, 1)) != CFPQ_OK) return st;
                if ((st = prof_mark3(0, 3)) != CFPQ_OK) return st;
            }
            if ((st = prof_mark3(0, 2)) != CFPQ_OK) return st;
            const uint32_t seed_slot = slot;
            HIP_TRY(launch_gather(a, true, grid, s));
            if ((st = prof_mark3(1, 0)) != CFPQ_OK) return st;
            if (prof) {
                if ((st = fetch(seed_slot, 1)) != CFPQ_OK) return st;
                res.prof[CFPQ_KERNEL_SEED].launches++;
                res.prof[CFPQ_KERNEL_SEED].ms += prof_span(ev3(0, 2), ev3(1, 0));
                if (sparse_nt) {
                    res.prof[CFPQ_KERNEL_ELL].launches++;
                    res.prof[CFPQ_KERNEL_ELL].ms += prof_span(ev3(0, 0), ev3(0, 1));
                    res.prof[CFPQ_KERNEL_NT_SPARSE].launches++;
                    res.prof[CFPQ_KERNEL_NT_SPARSE].ms += prof_span(ev3(0, 1), ev3(0, 3));
                    res.prof[CFPQ_KERNEL_NT_DENSE].launches++;
                    res.prof[CFPQ_KERNEL_NT_DENSE].ms += prof_span(ev3(0, 3), ev3(0, 2));
                }
            }
            uint32_t prev = slot++;
            a.rep = nullptr;   // the levels' products use M2, not the new edges
            uint64_t rows_in = prof ? pc.h[2] : 0;   // frontier rows feeding the next level
            // incremental closure: frontier levels until one adds nothing
            uint32_t li = 1;
            for (;;) {
                const uint32_t li0 = li;
                const uint32_t k = levels_hint;
                if ((st = need_slots(k + 1)) != CFPQ_OK) return st;
                const uint32_t first_slot = slot;
                // after a ring clear the previous count is gone; the previous
                // launch is known to have run (its count was read as nonzero,
                // or it is the seed), so the next one runs unconditionally
                if (first_slot == 0 && prev != 0) prev = kNoSlot;
                a.extra = nullptr; a.extra_act = nullptr;
                // matrix-core products for the nonterminal transitions (only on
                // request: with sparse frontiers the dense product re-reads the
                // selector per source word and the frontier per row tile, and
                // loses to the bit-serial OR of selected rows by 30-70x)
                const bool mfma = p.has_calls && o.nt_mode == CFPQ_NT_MFMA;
                // sparse product in the levels too: frontier rows are mostly a
                // few words, so an ELL list beats ORing the whole tile row
                const bool lsparse = sparse_nt && o.nt_mode == CFPQ_NT_AUTO && gw >= kLevelSparseMinWords;
                if ((mfma || lsparse) && !Dx.p) {
                    if (!Dx.alloc(al, fw * 8, s) || !xact.alloc(al, aw * 8, s))
                        return fail(CFPQ_ERR_OOM, "device allocation failed (matrix-core product)");
                }
                for (uint32_t j = 0; j < k; ++j, ++li) {
                    a.sel = d_NT; a.sel_act = nullptr; a.sel_sum = use_nsum ? nsum.as<uint64_t>() : nullptr;
                    a.src = Dbuf[(li - 1) & 1]; a.src_pitch = G; a.src_off = 0;
                    a.src_act = act[(li - 1) % 3]; a.src_blk = blk[(li - 1) % 3];
                    a.dn = Dbuf[li & 1]; a.actn = act[li % 3]; a.actn_blk = blk[li % 3];
                    a.act_clear = act[(li + 1) % 3];
                    a.slot_prev = prev; a.slot_cur = slot; a.seed_terms = 0;
                    a.dense_apart = lsparse ? 1u : 0u;
                    if ((st = prof_mark3(j, 0)) != CFPQ_OK) return st;
                    if (mfma) {
                        HIP_TRY(launch_fill(xact.as<uint64_t>(), aw, 0, s));
                        if ((st = prof_mark3(j, 1)) != CFPQ_OK) return st;
                        std::vector<uint8_t> first(nQ, 1);
                        for (uint32_t f = 0; f < nQ; ++f)
                            for (uint32_t t = p.in_off[f]; t < p.in_off[f + 1]; ++t) {
                                const InTrans tr = p.in_tr[t];
                                if (tr.sym < p.n_terms) continue;
                                MfmaArgs m{};
                                m.n = n; m.P = P; m.Pn = Pn; m.gw = gw; m.G = G;
                                m.sel = d_NT + (uint64_t)(tr.sym - p.n_terms) * n * P;
                                m.src = a.src + (uint64_t)tr.src * n * G; m.src_pitch = G;
                                m.sact = a.src_act + (uint64_t)tr.src * Pn;
                                m.out = Dx.as<uint64_t>() + (uint64_t)f * n * G;
                                m.out_act = xact.as<uint64_t>() + (uint64_t)f * Pn;
                                m.first = first[f];
                                first[f] = 0;
                                m.ctr_prev = prev == kNoSlot ? nullptr : d_ctr + (uint64_t)prev * kSlotWords;
                                m.mfma_ctr = prof ? mfma_ops : nullptr;
                                HIP_TRY(launch_nt_mfma(m, s));
                            }
                        if ((st = prof_mark3(j, 3)) != CFPQ_OK) return st;
                        a.extra = Dx.as<uint64_t>(); a.extra_act = xact.as<uint64_t>();
                    } else if (lsparse) {
                        HIP_TRY(launch_fill(xact.as<uint64_t>(), aw, 0, s));
                        HIP_TRY(launch_fill(d_dns, dense_words, 0, s));
                        uint32_t *ell_cnt = ell.as<uint32_t>(), *ell_idx = ell_cnt + ell_pad;
                        const unsigned long long *cp =
                            prev == kNoSlot ? nullptr : d_ctr + (uint64_t)prev * kSlotWords;
                        HIP_TRY(launch_ell_build_dense(a.src, G, 0, gw, n, tb.nt_src, (uint32_t)p.nt_src.size(),
                                                       ell_cnt, ell_idx, a.src_act, Pn, cp, d_dns, d_dblk, Pbs, s));
                        if ((st = prof_mark3(j, 1)) != CFPQ_OK) return st;
                        a.extra = nullptr;   // the product reads the selector, not extra
                        HIP_TRY(launch_nt_sparse(a, ell_cnt, ell_idx, Dx.as<uint64_t>(), xact.as<uint64_t>(), grid, s));
                        if ((st = prof_mark3(j, 3)) != CFPQ_OK) return st;
                        if ((st = dense_product(a, Dx.as<uint64_t>(), xact.as<uint64_t>())) != CFPQ_OK) return st;
                        a.extra = Dx.as<uint64_t>(); a.extra_act = xact.as<uint64_t>();
                    } else {
                        if ((st = prof_mark3(j, 1)) != CFPQ_OK) return st;
                        if ((st = prof_mark3(j, 3)) != CFPQ_OK) return st;
                    }
                    a.dense_apart = 0;
                    if ((st = prof_mark3(j, 2)) != CFPQ_OK) return st;
                    HIP_TRY(launch_gather(a, false, grid, s));
                    prev = slot++;
                }
                if ((st = prof_mark3(k, 0)) != CFPQ_OK) return st;
                if ((st = fetch(first_slot, k)) != CFPQ_OK) return st;
                uint32_t used = k;
                for (uint32_t j = 0; j < k; ++j)
                    if (pc.h[(size_t)j * kSlotWords] == 0) {
                        used = j;
                        break;
                    }
                if (prof) {
                    auto &pl = res.prof[CFPQ_KERNEL_LEVEL];
                    for (uint32_t j = 0; j < k; ++j) {
                        pl.launches++;
                        pl.ms += prof_span(ev3(j, 2), ev3(j + 1, 0));
                        if (mfma || lsparse) {
                            auto &pp = res.prof[mfma ? CFPQ_KERNEL_NT_MFMA : CFPQ_KERNEL_NT_SPARSE];
                            pp.launches++;
                            pp.ms += prof_span(ev3(j, 1), ev3(j, 3));
                        }
                        if (lsparse) {
                            res.prof[CFPQ_KERNEL_ELL].launches++;
                            res.prof[CFPQ_KERNEL_ELL].ms += prof_span(ev3(j, 0), ev3(j, 1));
                            res.prof[CFPQ_KERNEL_NT_DENSE].launches++;
                            res.prof[CFPQ_KERNEL_NT_DENSE].ms += prof_span(ev3(j, 3), ev3(j, 2));
                        }
                        const uint64_t fed = pc.h[(size_t)j * kSlotWords + 1];
                        const uint64_t gained = pc.h[(size_t)j * kSlotWords + 2];
                        if (j <= used) pl.bytes += 8ull * gw * (rows_in + 3 * fed);
                        rows_in = gained;
                    }
                }
                if (used < k) {
                    // levels this tile needed; the next tile of the same graph
                    // needs about as many
                    levels_hint = std::max<uint32_t>(4, (li0 - 1) + used + 2);
                    break;
                }
                levels_hint = std::min<uint32_t>(levels_hint * 2, 1024);
            }
        }
        // write-back
        if ((st = need_slots(nB + 1)) != CFPQ_OK) return st;
        HIP_TRY(launch_fill(dact[cur ^ 1], (uint64_t)nB * Pn, 0, s));
        WritebackArgs w{};
        w.n = n; w.P = P; w.Pn = Pn; w.nB = nB; w.fin_off = tb.fin_off; w.fin = tb.fin;
        w.T = d_T; w.NT = d_NT; w.dNT = d_dNT; w.dnt_act = dact[cur ^ 1];
        w.rank = o.keep_rank ? res.rank.as<uint8_t>() : nullptr;
        w.iter = it; w.ctr = d_ctr; w.slot_base = slot;
        w.chg = d_chg; w.prev_act = dact[cur]; w.rows_ctr = wb_rows;
        // the summaries of the rows it changes come out of the write-back
        // itself (every row whose dNT or NT row changes is visited);
        // CFPQ_WB_SUMMARY = 0 rebuilds them in a pass of their own
#ifndef CFPQ_WB_SUMMARY
#define CFPQ_WB_SUMMARY 1
#endif
        w.sum_pitch = sum_pitch;
        if (CFPQ_WB_SUMMARY) {
            w.dsum = use_sum ? dsum.as<uint64_t>() : nullptr;
            w.nsum = use_nsum ? nsum.as<uint64_t>() : nullptr;
        }
        w.dhash = dedup ? dd_hash : nullptr;
        // whole rows in the first iteration (its seed writes T outside the
        // gathers) and when the closure is recomputed
        w.chgb = (wb_blocks && it > 1 && !scratch) ? d_chgb : nullptr;
        w.dnb = d_dnb;
        w.blk_words = blk_words;
        if ((st = prof_mark(0)) != CFPQ_OK) return st;
        HIP_TRY(launch_writeback(w, gather_grid((uint64_t)nB * n), s));
        if ((st = prof_mark(1)) != CFPQ_OK) return st;
        cur ^= 1;
        if (use_sum && !w.dsum)
            HIP_TRY(launch_row_summary(d_dNT, nB, n, P, Pn, dact[cur], dsum.as<uint64_t>(), sum_pitch, s));
        if (use_nsum && !w.nsum)
            HIP_TRY(launch_row_summary(d_NT, nB, n, P, Pn, dact[cur], nsum.as<uint64_t>(), sum_pitch, s));
        if (dedup) {
            HIP_TRY(launch_dedup(nB, n, P, Pn, dact[cur], dd_hash, d_dNT, dsum.as<uint64_t>(), sum_pitch, dd_keys,
                                 dd_vals, dd_mask, dd_rep, s));
            rep_valid = true;
        }
        if ((st = fetch(slot, nB)) != CFPQ_OK) return st;
        if (prof) {
            auto &pw = res.prof[CFPQ_KERNEL_WRITEBACK];
            pw.launches++;
            pw.ms += prof_ms(0);
        }
        slot += nB;
        uint64_t delta = 0;
        for (uint32_t b = 0; b < nB; ++b) {
            box_delta[b] = pc.h[(size_t)b * kSlotWords];
            delta += box_delta[b];
        }
        res.deltas.push_back(delta);
        if (delta == 0) break;
    }
    HIP_TRY(hipEventRecord(ev[1], s));
    HIP_TRY(hipEventSynchronize(ev[1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
    res.ms = ms;
    res.iterations = it;
    if (prof) {
        std::vector<unsigned long long> pc2(3 + nB);
        HIP_TRY(hipMemcpy(pc2.data(), mfma_ops, pc2.size() * 8, hipMemcpyDeviceToHost));
        res.prof[CFPQ_KERNEL_NT_MFMA].bytes = pc2[0] * 65536ull;   // 2 * 32 * 32 * 32 per instruction
        res.prof[CFPQ_KERNEL_NT_SPARSE].bytes = pc2[1];
        res.prof[CFPQ_KERNEL_NT_DENSE].bytes = pc2[2];
        // write-back: per row word processed, the final states' closure
        // words and the M2^N word read, M2^N and A2^N words written
        auto &pw = res.prof[CFPQ_KERNEL_WRITEBACK];
        pw.bytes = 0;
        for (uint32_t b = 0; b < nB; ++b)
            pw.bytes += pc2[3 + b] * 8ull * (uint64_t)(p.fin_off[b + 1] - p.fin_off[b] + 3);
    }
    if (o.keep_blocks) res.T = std::move(T);
    return CFPQ_OK;
}

// ---------------------------------------------------------------------------
// CONDENSED strategy: closure through the strongly connected components of
// the product graph (regular queries: no box-labelled transition)
// ---------------------------------------------------------------------------
cfpq_status run_condensed(const cfpq_graph_s &g, const cfpq_rsm_s &r, const cfpq_query_opts &o,
                          cfpq_result_s &res) {
    hipStream_t s = (hipStream_t)o.stream;
    const Alloc *al = &res.alloc;
    Plan p = make_plan(g, r);
    if (p.has_calls) return fail(CFPQ_ERR_INVALID, "condensed strategy needs an RSM without box-labelled transitions");
    if ((uint64_t)p.nQ * p.n >= 0xFFFFFFFFull) return fail(CFPQ_ERR_LIMIT, "product graph exceeds 2^32-1 nodes");
    // state flags: box start; only final state of its box (then single-member
    // rows of that state are the answer rows themselves); box id
    {
        const bool can_alias = p.eps_boxes.empty() && !o.keep_blocks && !o.keep_rank;
        for (uint32_t q = 0; q < p.nQ; ++q) {
            const uint32_t b = r.state_box[q];
            const bool only_final = r.is_final[q] && p.fin_off[b + 1] - p.fin_off[b] == 1;
            p.is_start[q] = (p.is_start[q] ? kStartState : 0) | ((can_alias && only_final) ? kAliasFinal : 0) |
                            (b << kFlagBoxShift);
        }
    }
    const uint32_t n = p.n, P = p.P, Pn = p.Pn, nQ = p.nQ, nB = p.nB;
    const uint32_t N = nQ * n;
    const uint64_t qw = (uint64_t)nQ * n * P, bw = (uint64_t)nB * n * P;
    const uint64_t N64 = ((uint64_t)N + 63) / 64 * 64;   // byte arrays padded to whole words
    const uint64_t Nu = ((uint64_t)N + 3) / 4 * 4;         // u32 arrays start on 16-byte boundaries
    constexpr uint32_t kCtr = 8192;
    if ((uint64_t)nB * kSlotWords > kCtr) return fail(CFPQ_ERR_LIMIT, "too many boxes for the condensed strategy");
    const uint32_t nch = cond_chunks(Pn);
    const uint64_t nzb = ((uint64_t)N * nch + 63) / 64 * 64;   // non-empty chunk flags

    // one work allocation (every allocation is a call into the caller's
    // allocator): launch counters, node arrays, found and chunk flags (all
    // cleared by one fill), live flags, and the epsilon delta when a box is
    // nullable
    const bool nullable = !p.eps_boxes.empty();
    auto al256 = [](uint64_t x) { return (x + 255) / 256 * 256; };
    const uint64_t o_u32 = al256(((uint64_t)2 * kCtr + 8) * 8);
    // condensation links (kCondLinks per node in each direction, with
    // counts) when the stripe indices fit in 32 bits
#ifndef CFPQ_COND_LINKS
#define CFPQ_COND_LINKS 1
#endif
    const bool links = CFPQ_COND_LINKS && (uint64_t)N * kStripes < (1ull << 32);
    const uint64_t link_u32 = links ? (2 + 2 * (uint64_t)kCondLinks) * Nu : 0;
    // trimming witnesses: two words per node, zero (none) at the start
#ifndef CFPQ_TRIM_WITNESS
#define CFPQ_TRIM_WITNESS 1
#endif
    const uint64_t wit_u32 = CFPQ_TRIM_WITNESS ? 2 * Nu : 0;
    const uint64_t o_fnz = o_u32 + al256(Nu * 4 * (9 + kStripes) + (link_u32 + wit_u32) * 4 + 64);
    const uint64_t o_alive = o_fnz + al256(N64 + nzb + 64);
    const uint64_t o_act = o_alive + al256(N64);
    const uint64_t o_dnt = o_act + al256((uint64_t)nB * Pn * 8);
    // the small tables and the closure rows T share the work allocation
    // (one call into the caller's allocator); T is separate when the query
    // keeps it (keep_blocks)
    TableImage im;
    pack_tables(p, im);
    const uint64_t o_tbl = o_dnt + al256(nullable ? bw * 8 : 8);
    const uint64_t o_T = o_tbl + al256(im.host.size());
    DevBuf T, work;
    if (!res.NT.alloc(al, bw * 8, s) || !work.alloc(al, o_T + (o.keep_blocks ? 0 : qw * 8), s) ||
        (o.keep_blocks && !T.alloc(al, qw * 8, s)))
        return fail(CFPQ_ERR_OOM, "device allocation failed (condensed query)");
    uint8_t *wk = work.as<uint8_t>();
    uint64_t *Tp = o.keep_blocks ? T.as<uint64_t>() : (uint64_t *)(wk + o_T);
    // counter read-backs: [0, kCtr) launch counters, [kCtr, 2 kCtr) level
    // counts, then the search frontier sizes; the table image goes behind
    // them (pinned, so the upload needs no wait: the query's last read-back
    // comes after it on the stream)
    constexpr size_t kPinWords = 2 * (size_t)8192 + 8;
    PinnedCounters pc;
    const size_t img_words = (im.host.size() + 7) / 8;
    if (!pc.ensure(kPinWords + img_words)) return fail(CFPQ_ERR_OOM, "pinned host allocation failed");
    std::memcpy(pc.h + kPinWords, im.host.data(), im.host.size());
    HIP_TRY(hipMemcpyAsync(wk + o_tbl, pc.h + kPinWords, im.host.size(), hipMemcpyHostToDevice, s));
    Tables tb;
    bind_tables(im, wk + o_tbl, tb);
    cfpq_status st = CFPQ_OK;
    uint64_t *dnt_act = (uint64_t *)(wk + o_act), *dNT = (uint64_t *)(wk + o_dnt);
    if (o.keep_rank) {
        if (!res.rank.alloc(al, (uint64_t)nB * n * n, s)) return fail(CFPQ_ERR_OOM, "device allocation failed (rank)");
        HIP_TRY(hipMemsetAsync(res.rank.p, 0xFF, (uint64_t)nB * n * n, s));
    }
    uint32_t *scc = (uint32_t *)(wk + o_u32), *fw = scc + Nu, *bwm = fw + Nu, *color = bwm + Nu, *size = color + Nu,
             *pending = size + Nu, *qa = pending + Nu, *qb = qa + Nu, *lev = qb + Nu, *stripe = lev + Nu;
    uint8_t *found = wk + o_fnz, *nzf = found + N64, *alive = wk + o_alive;
    unsigned long long *cc = (unsigned long long *)wk;
    unsigned long long *lc = cc + kCtr;   // ring of per-level component counts
    ProdGraph pg{};
    pg.n = n; pg.nQ = nQ;
    pg.goff = g.off.as<uint32_t>(); pg.gidx = g.idx.as<uint32_t>();
    pg.soff = g.soff.as<uint32_t>(); pg.sidx = g.sidx.as<uint32_t>();
    pg.in_off = tb.in_off; pg.in_tr = tb.in_tr; pg.out_off = tb.out_off; pg.out_tr = tb.out_tr;
#ifndef CFPQ_SEARCH_INTRA
#define CFPQ_SEARCH_INTRA 1
#endif
    if (CFPQ_SEARCH_INTRA) {
        pg.sin_off = tb.sin_off; pg.sin_tr = tb.sin_tr; pg.sout_off = tb.sout_off; pg.sout_tr = tb.sout_tr;
    } else {
        pg.sin_off = tb.in_off; pg.sin_tr = tb.in_tr; pg.sout_off = tb.out_off; pg.sout_tr = tb.out_tr;
    }
    pg.src_mask = res.src_mask.as<uint64_t>();
    if (links) {
        pg.xin_cnt = stripe + (uint64_t)kStripes * Nu;
        pg.xout_cnt = pg.xin_cnt + Nu;
        pg.xin = pg.xout_cnt + Nu;
        pg.xout = pg.xin + (uint64_t)kCondLinks * Nu;
    }
    if (wit_u32) pg.trim_w = stripe + (uint64_t)kStripes * Nu + link_u32;   // 8-byte aligned (Nu % 4 == 0)

    PooledEvents evp;
    HIP_TRY(evp.ensure(4));
    hipEvent_t *ev = evp.v.data();
    const bool prof = o.profile != 0;
    res.profiled = prof;
    static_assert(2 * kCtr + 8 == kPinWords, "read-back area in front of the table image");
    uint32_t slot = 0;
    // a fresh zeroed counter per launch; the whole array is cleared when used up
    auto next_slot = [&](uint32_t k) -> cfpq_status {
        if (slot + k >= kCtr) {
            HIP_TRY(launch_fill((uint64_t *)cc, kCtr, 0, s));
            slot = 0;
        }
        return CFPQ_OK;
    };
    auto read = [&](uint32_t first, uint32_t k) -> cfpq_status {
        HIP_TRY(hipMemcpyAsync(pc.h, cc + first, (size_t)k * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(wait_stream(s));
        return CFPQ_OK;
    };
    // run launch(i, prev, cur) as a chain until a launch counts zero: chunks of
    // launches go out back to back, each exits at once when its predecessor
    // counted zero, and the host reads the chunk's counters once
    auto chain = [&](auto launch, uint32_t chunk, std::atomic<uint32_t> *used, uint32_t from = 0) -> cfpq_status {
        const unsigned long long *prev = nullptr;
        for (uint32_t i = from;;) {
            if (slot + chunk >= kCtr) {
                // clearing the counters loses prev; the launch it belongs to
                // counted nonzero (else the chain had ended), so run on
                HIP_TRY(launch_fill((uint64_t *)cc, kCtr, 0, s));
                slot = 0;
                prev = nullptr;
            }
            const uint32_t first = slot;
            for (uint32_t j = 0; j < chunk; ++j, ++i) {
                HIP_TRY(launch(i, prev, cc + slot));
                prev = cc + slot++;
            }
            cfpq_status st2 = read(first, chunk);
            if (st2 != CFPQ_OK) return st2;
            for (uint32_t j = 0; j < chunk; ++j)
                if (pc.h[j] == 0) {
                    if (used) used->store(i - chunk + j + 1, std::memory_order_relaxed);
                    return CFPQ_OK;
                }
            chunk = std::min<uint32_t>(chunk * 2, 256);
        }
    };

    HIP_TRY(hipEventRecord(ev[0], s));
    // M2^N is empty unless a box is nullable; then it needs the epsilon loops
    const bool fresh = p.eps_boxes.empty();
    if (!fresh) HIP_TRY(launch_fill(d_u64(res.NT), bw, 0, s));
    HIP_TRY(launch_fill((uint64_t *)wk, o_alive / 8, 0, s));   // counters, node arrays, found and chunk flags
    HIP_TRY(launch_fill((uint64_t *)alive, N64 / 8, 0x0101010101010101ull, s));  // every node live
    if (!fresh) {
        HIP_TRY(launch_fill(dNT, bw, 0, s));
        HIP_TRY(launch_fill(dnt_act, (uint64_t)nB * Pn, 0, s));
        HIP_TRY(launch_eps(d_u64(res.NT), dNT, dnt_act, o.keep_rank ? res.rank.as<uint8_t>() : nullptr,
                           n, P, Pn, tb.eps, (uint32_t)p.eps_boxes.size(), s));
    }

    // ---- strongly connected components of the product graph
    auto chunk0 = [](const std::atomic<uint32_t> &h, uint32_t dflt) {
        const uint32_t v = h.load(std::memory_order_relaxed);
        return v ? std::min<uint32_t>(v, 256) : dflt;
    };
    // the pivot key lives past the launch counters, which a long chain clears
    // and reuses; the pivot goes from k_pivot to the searches on the device
    unsigned long long *best = cc + 2 * kCtr;
    // frontiers of the pivot searches: four node arrays that are free until
    // the colouring (color) and the condensation (pending, qa, qb); their
    // size ring after the pivot key
    ReachQueues rq{};
    rq.q[0][0] = qa;
    rq.q[0][1] = qb;
    rq.q[1][0] = color;
    rq.q[1][1] = pending;
    rq.cnt = cc + 2 * kCtr + 1;
    rq.cap = N;
    auto reach_chain = [&](uint32_t from) -> cfpq_status {
        return chain([&](uint32_t i, const unsigned long long *, unsigned long long *c) {
            return launch_reach(pg, alive, fw, bwm, rq, i, c, s);
        }, chunk0(g.hint_reach, 8), &g.hint_reach, from);
    };
    // colouring rounds until every node has a component
    auto colouring = [&]() -> cfpq_status {
        for (;;) {
            cfpq_status st2;
            if ((st2 = next_slot(1)) != CFPQ_OK) return st2;
            const uint32_t rem_slot = slot++;
            HIP_TRY(launch_color_remove(N, alive, found, cc + rem_slot, s));  // counts live nodes
            if ((st2 = read(rem_slot, 1)) != CFPQ_OK) return st2;
            if (pc.h[0] == 0) return CFPQ_OK;
            HIP_TRY(launch_color_init(N, alive, color, found, s));
            st2 = chain([&](uint32_t, const unsigned long long *pv, unsigned long long *c) {
                return launch_color_prop(pg, alive, color, pv, c, s);
            }, 8, nullptr);
            if (st2 != CFPQ_OK) return st2;
            HIP_TRY(launch_color_roots(N, alive, color, found, scc, s));
            st2 = chain([&](uint32_t, const unsigned long long *pv, unsigned long long *c) {
                return launch_color_back(pg, alive, color, found, scc, pv, c, s);
            }, 8, nullptr);
            if (st2 != CFPQ_OK) return st2;
        }
    };

    // ---- condensation, one topological level per launch
    if ((uint64_t)nB * (kWave + kSlotWords) > kBytesSlot)
        return fail(CFPQ_ERR_LIMIT, "too many boxes for the condensed strategy");
    // answer pairs counted by the closure: kWave stripes per box (the search
    // counters in front of kBytesSlot are not used from here on)
    unsigned long long *box_pairs = cc;
    unsigned long long *wb_ctr = cc + (uint64_t)nB * kWave;
    unsigned long long *bytes_ctr = prof ? box_pairs + kBytesSlot : nullptr;
    // level L's component count lives in lc[L % kCtr]; the launch for level L
    // clears lc[(L + 2) % kCtr] before level L + 1 writes it
    auto condense_setup = [&](const unsigned long long *skip_if) -> cfpq_status {
        HIP_TRY(launch_cond_count(pg, scc, size, stripe, skip_if, s));
        HIP_TRY(launch_cond_seed(n, P, Pn, nQ, tb.starts, nB, scc, size, Tp, nzf, res.src_mask.as<uint64_t>(),
                                 skip_if, s));
        HIP_TRY(launch_cond_roots(N, scc, stripe, pending, lev, lc + 0, skip_if, s));
        HIP_TRY(launch_fill((uint64_t *)box_pairs, (uint64_t)nB * kWave, 0, s));
        HIP_TRY(launch_fill((uint64_t *)box_pairs + kBytesSlot, 2 * kWave, 0, s));
        return CFPQ_OK;
    };
    PooledEvents lev_pool;   // profiling: an event before each level launch, one after the chunk
    std::vector<hipEvent_t> &lev_ev = lev_pool.v;
    // launches for levels L .. L + k - 1 (with profiling events)
    // Profiling times the chain of level launches with one event before its
    // first launch and one after its last: a timing event on the stream
    // costs a drain of the GPU (about 5 us measured between dependent
    // kernels), so per-launch events would add a fifth to the level time
    // they measure.  CFPQ_PROFILE_EACH_LAUNCH = 1 brackets every launch.
#ifndef CFPQ_PROFILE_EACH_LAUNCH
#define CFPQ_PROFILE_EACH_LAUNCH 0
#endif
    const auto lev_end = [](uint32_t k) { return CFPQ_PROFILE_EACH_LAUNCH ? k : 1u; };   // event after the chain
    auto level_chunk = [&](uint32_t L, uint32_t k) -> cfpq_status {
        if (prof) HIP_TRY(lev_pool.ensure(lev_end(k) + 1));
        for (uint32_t j = 0; j < k; ++j) {
            const uint32_t l = L + j;
            if (prof && (CFPQ_PROFILE_EACH_LAUNCH || j == 0)) HIP_TRY(hipEventRecord(lev_ev[j], s));
            HIP_TRY(launch_cond_level(pg, P, Pn, scc, size, stripe, pending, lev, Tp, d_u64(res.NT), nzf,
                                      tb.is_start, l, lc + l % kCtr, lc + (l + 1) % kCtr, lc + (l + 2) % kCtr,
                                      box_pairs, bytes_ctr, s));
        }
        if (prof) HIP_TRY(hipEventRecord(lev_ev[lev_end(k)], s));
        return CFPQ_OK;
    };
    auto level_chunk_times = [&](uint32_t k) -> cfpq_status {
        if (!prof) return CFPQ_OK;
        float t = 0.f;
        if (CFPQ_PROFILE_EACH_LAUNCH) {
            for (uint32_t j = 0; j < k; ++j) {
                HIP_TRY(hipEventElapsedTime(&t, lev_ev[j], lev_ev[j + 1]));
                res.prof[CFPQ_KERNEL_COND_LEVEL].ms += t;
            }
        } else if (k) {
            HIP_TRY(hipEventElapsedTime(&t, lev_ev[0], lev_ev[lev_end(k)]));
            res.prof[CFPQ_KERNEL_COND_LEVEL].ms += t;
        }
        res.prof[CFPQ_KERNEL_COND_LEVEL].launches += k;
        return CFPQ_OK;
    };
    // level chunks from L0 with a host read after each, until a level is empty
    auto levels = [&](uint32_t L0) -> cfpq_status {
        uint32_t L = L0, hint = chunk0(g.hint_levels, 32);
        for (;;) {
            const uint32_t k = hint;
            cfpq_status st2 = level_chunk(L, k);
            if (st2 != CFPQ_OK) return st2;
            HIP_TRY(hipMemcpyAsync(pc.h, lc, (size_t)kCtr * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(wait_stream(s));
            if ((st2 = level_chunk_times(k)) != CFPQ_OK) return st2;
            for (uint32_t j = 0; j <= k; ++j)
                if (pc.h[(L + j) % kCtr] == 0) {
                    g.hint_levels.store(std::max<uint32_t>(L + j, 1), std::memory_order_relaxed);
                    return CFPQ_OK;
                }
            L += k;
            hint = std::min<uint32_t>(hint * 2, 1024);
            if (L > 0xFFFFFFFFu - 2048) return fail(CFPQ_ERR_LIMIT, "condensation too deep");
        }
    };
    // ---- write-back through the component map for the answer rows the
    // closure did not write itself; nothing reads the deltas of a query
    // without box-labelled transitions, so none are kept
    auto writeback = [&](const unsigned long long *skip0, const unsigned long long *skip1) -> cfpq_status {
        HIP_TRY(launch_fill((uint64_t *)wb_ctr, (uint64_t)nB * kSlotWords, 0, s));
        WritebackArgs w{};
        w.n = n; w.P = P; w.Pn = Pn; w.nB = nB; w.fin_off = tb.fin_off; w.fin = tb.fin;
        w.T = Tp; w.NT = d_u64(res.NT); w.dNT = nullptr; w.dnt_act = nullptr; w.fresh = fresh;
        w.rank = o.keep_rank ? res.rank.as<uint8_t>() : nullptr;
        w.iter = 1; w.ctr = wb_ctr; w.slot_base = 0; w.row_map = scc; w.row_nz = nzf;
        w.state_flags = tb.is_start; w.multi = size;
        w.skip_if[0] = skip0; w.skip_if[1] = skip1;
        HIP_TRY(launch_writeback(w, gather_grid((uint64_t)nB * n), s));
        return CFPQ_OK;
    };
    const size_t n_out = (size_t)nB * kWave + (size_t)nB * kSlotWords;   // box pairs and write-back counters

    // Fast path: when the previous query on this graph shows how many
    // trimming sweeps, search frontiers and levels suffice, the whole query
    // goes out with one host read at the end.  Guards on the device turn
    // every step after an unfinished one into a no-op (component assignment
    // waits for both searches to end, the condensation for every node to
    // have a component, the write-back for an empty level), and the host
    // finishes the query from the first unfinished step.
    const uint32_t ht = g.hint_trim.load(std::memory_order_relaxed);
    const uint32_t hr = g.hint_reach.load(std::memory_order_relaxed);
    const uint32_t hl = g.hint_levels.load(std::memory_order_relaxed);
    constexpr uint32_t kSpecBase = kBytesSlot + 2 * kWave;   // past the closure's counters
    const bool spec = ht && hr && hl && hl <= 1024 && (uint64_t)kSpecBase + ht + hr + 2 <= kCtr && !o.keep_blocks;
    bool finished = false;
    float ms_scc = 0.f, ms_wb = 0.f;         // profiling: search with set-up, write-back
    bool scc_timed = false, wb_timed = false;   // taken from the level chain's events
    if (spec) {
        uint32_t sl = kSpecBase;
        const uint32_t trim0 = sl;
        const unsigned long long *prev = nullptr;
        for (uint32_t j = 0; j < ht; ++j, ++sl) {   // trimming need not finish: the searches handle the rest
            HIP_TRY(launch_trim(pg, alive, scc, prev, cc + sl, s));
            prev = cc + sl;
        }
        HIP_TRY(launch_pivot(pg, alive, best, s));
        HIP_TRY(launch_pivot_seed(best, fw, bwm, rq, s));
        const uint32_t reach0 = sl;
        for (uint32_t i = 0; i < hr; ++i, ++sl) HIP_TRY(launch_reach(pg, alive, fw, bwm, rq, i, cc + sl, s));
        // frontier hr empty: both searches are complete
        HIP_TRY(launch_fwbw_assign(N, alive, fw, bwm, best, scc, cc + sl++, rq.cnt + hr % 3, rq.cnt + 3 + hr % 3, s));
        const uint32_t rem = sl++;
        HIP_TRY(launch_color_remove(N, alive, found, cc + rem, s));   // nodes still without a component
        // profiling: the search and the condensation set-up end where the
        // level chain's first event is, the write-back begins at its last
        // (no events of their own: each timing event drains the GPU)
        cfpq_status st2 = condense_setup(cc + rem);
        if (st2 != CFPQ_OK) return st2;
        if ((st2 = level_chunk(0, hl)) != CFPQ_OK) return st2;
        if ((st2 = writeback(cc + rem, lc + hl % kCtr)) != CFPQ_OK) return st2;
        HIP_TRY(hipEventRecord(ev[3], s));
        // one read-back of the whole counter area (pc.h mirrors its layout):
        // answer pairs, write-back and byte counters, the speculative
        // launches' counters, the level counts and the search frontiers
        HIP_TRY(hipMemcpyAsync(pc.h, cc, kPinWords * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(wait_stream(s));
        if ((st2 = level_chunk_times(hl)) != CFPQ_OK) return st2;
        if (prof) {
            HIP_TRY(hipEventElapsedTime(&ms_scc, ev[0], lev_ev[0]));
            HIP_TRY(hipEventElapsedTime(&ms_wb, lev_ev[lev_end(hl)], ev[3]));
            scc_timed = wb_timed = true;   // valid if the query finished here
        }
        // chain lengths for the next query, as the synchronous chains count them
        uint32_t used = 2 * ht;
        for (uint32_t j = 0; j < ht; ++j)
            if (pc.h[trim0 + j] == 0) {
                used = j + 1;
                break;
            }
        g.hint_trim.store(std::min<uint32_t>(used, 256), std::memory_order_relaxed);
        const unsigned long long *fr = pc.h + (rq.cnt - cc);   // frontier sizes
        const bool searched = (fr[hr % 3] | fr[3 + hr % 3]) == 0;
        if (!searched) {
            // the searches go on from frontier hr; nothing after them ran
            if ((st2 = reach_chain(hr)) != CFPQ_OK) return st2;
            if ((st2 = next_slot(1)) != CFPQ_OK) return st2;
            HIP_TRY(launch_fwbw_assign(N, alive, fw, bwm, best, scc, cc + slot++, nullptr, nullptr, s));
        } else {
            for (uint32_t j = 0; j < hr; ++j)
                if (pc.h[reach0 + j] == 0) {
                    g.hint_reach.store(j + 1, std::memory_order_relaxed);
                    break;
                }
        }
        if (!searched || pc.h[rem] != 0) {
            // colouring, then the condensation from the start (its set-up,
            // levels and write-back were no-ops)
            if ((st2 = colouring()) != CFPQ_OK) return st2;
            HIP_TRY(launch_fill((uint64_t *)lc, kCtr, 0, s));
            if ((st2 = condense_setup(nullptr)) != CFPQ_OK) return st2;
            if (prof) HIP_TRY(hipEventRecord(ev[1], s));
            scc_timed = wb_timed = false;
            if ((st2 = levels(0)) != CFPQ_OK) return st2;
        } else {
            uint32_t z = hl + 1;   // first empty level, if one was launched
            for (uint32_t j = 0; j <= hl; ++j)
                if (pc.h[(lc - cc) + j] == 0) {
                    z = j;
                    break;
                }
            if (z <= hl) {
                g.hint_levels.store(std::max<uint32_t>(z, 1), std::memory_order_relaxed);
                finished = true;   // the write-back ran and its counters are read
            } else {
                wb_timed = false;
                if ((st2 = levels(hl)) != CFPQ_OK) return st2;
            }
        }
        if (!finished) {
            if (prof) HIP_TRY(hipEventRecord(ev[2], s));
            if ((st2 = writeback(nullptr, nullptr)) != CFPQ_OK) return st2;
            HIP_TRY(hipEventRecord(ev[3], s));
        }
    } else {
        st = chain([&](uint32_t, const unsigned long long *pv, unsigned long long *c) {
            return launch_trim(pg, alive, scc, pv, c, s);
        }, chunk0(g.hint_trim, 8), &g.hint_trim);
        if (st != CFPQ_OK) return st;
        // the component of a high-degree pivot: forward AND backward reachable
        HIP_TRY(launch_pivot(pg, alive, best, s));
        HIP_TRY(launch_pivot_seed(best, fw, bwm, rq, s));
        if ((st = reach_chain(0)) != CFPQ_OK) return st;
        if ((st = next_slot(1)) != CFPQ_OK) return st;
        HIP_TRY(launch_fwbw_assign(N, alive, fw, bwm, best, scc, cc + slot++, nullptr, nullptr, s));
        if ((st = colouring()) != CFPQ_OK) return st;
        if ((st = condense_setup(nullptr)) != CFPQ_OK) return st;
        if (prof) HIP_TRY(hipEventRecord(ev[1], s));
        if ((st = levels(0)) != CFPQ_OK) return st;
        if (prof) HIP_TRY(hipEventRecord(ev[2], s));
        if ((st = writeback(nullptr, nullptr)) != CFPQ_OK) return st;
        if (o.keep_blocks) HIP_TRY(launch_cond_expand(N, P, Pn, scc, nzf, Tp, s));
        HIP_TRY(hipEventRecord(ev[3], s));
    }
    if (!finished) {
        // answer pairs, write-back counters and (profiling) the level
        // kernel's byte counters in one read
        HIP_TRY(hipMemcpyAsync(pc.h, cc, n_out * 8, hipMemcpyDeviceToHost, s));
        if (prof) HIP_TRY(hipMemcpyAsync(pc.h + kBytesSlot, bytes_ctr, 2 * kWave * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(wait_stream(s));
    }
    uint64_t delta = 0;
    for (uint32_t b = 0; b < nB; ++b) {
        for (uint32_t j = 0; j < kWave; ++j) delta += pc.h[(size_t)b * kWave + j];
        delta += pc.h[(size_t)nB * kWave + (size_t)b * kSlotWords];
    }
    uint64_t level_bytes = 0;
    if (prof)
        for (uint32_t j = 0; j < 2 * kWave; ++j) level_bytes += 8ull * pc.h[kBytesSlot + j];
    // a second iteration would seed from box-labelled transitions only: none
    res.deltas.assign({delta, 0});
    res.iterations = 2;
    if (max_iters_hit(o, 2)) return fail(CFPQ_ERR_LIMIT, "fixpoint did not stop within max_iters iterations");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[3]));
    res.ms = ms;
    if (prof) {
        // search (with the condensation set-up) and write-back times; the
        // events are recorded only when profiling
        if (!scc_timed) HIP_TRY(hipEventElapsedTime(&ms_scc, ev[0], ev[1]));
        if (!wb_timed) HIP_TRY(hipEventElapsedTime(&ms_wb, ev[2], ev[3]));
        res.prof[CFPQ_KERNEL_COND_SCC].launches += 1;
        res.prof[CFPQ_KERNEL_COND_SCC].ms += ms_scc;
        res.prof[CFPQ_KERNEL_COND_LEVEL].bytes += level_bytes;
        res.prof[CFPQ_KERNEL_WRITEBACK].launches += 1;
        res.prof[CFPQ_KERNEL_WRITEBACK].ms += ms_wb;
        for (uint32_t b = 0; b < nB; ++b)
            res.prof[CFPQ_KERNEL_WRITEBACK].bytes +=
                8ull * Pn * n * (uint64_t)(p.fin_off[b + 1] - p.fin_off[b] + (p.fin_off[b + 1] > p.fin_off[b] ? 3 : 0));
    }
    if (o.keep_blocks) res.T = std::move(T);
    return CFPQ_OK;
}

// ---------------------------------------------------------------------------
// PEREDGE strategy: the literal per-edge incremental closure (small graphs)
// ---------------------------------------------------------------------------
constexpr uint64_t kPerEdgeMaxNodes = 65536;          // product nodes nQ * n
constexpr uint64_t kPerEdgeMaxClosureBytes = 512ull << 20;

bool peredge_ok(const cfpq_graph_s &g, const cfpq_rsm_s &r) {
    const uint64_t N = (uint64_t)r.n_states * g.n, W = (N + 63) / 64;
    return N <= kPerEdgeMaxNodes && N * W * 8 <= kPerEdgeMaxClosureBytes;
}

cfpq_status run_peredge(const cfpq_graph_s &g, const cfpq_rsm_s &r, const cfpq_query_opts &o, cfpq_result_s &res) {
    hipStream_t s = (hipStream_t)o.stream;
    const Alloc *al = &res.alloc;
    Plan p = make_plan(g, r);
    Tables tb;
    cfpq_status st = upload_tables(p, al, s, tb);
    if (st != CFPQ_OK) return st;
    const uint32_t n = p.n, nQ = p.nQ, nB = p.nB;
    const uint64_t N = (uint64_t)nQ * n, W = (N + 63) / 64, Wn = p.Pn;
    // transitions as three arrays, in the RSM's order
    std::vector<uint32_t> tr(3 * r.t_src.size());
    for (size_t i = 0; i < r.t_src.size(); ++i) {
        tr[i] = r.t_src[i];
        tr[r.t_src.size() + i] = r.t_sym[i];
        tr[2 * r.t_src.size() + i] = r.t_dst[i];
    }
    DevBuf C, M, dM, trb, stats;
    const uint64_t mw = (uint64_t)nB * n * Wn;
    if (!C.alloc(al, N * W * 8, s) || !M.alloc(al, mw * 8, s) || !dM.alloc(al, mw * 8, s) ||
        !trb.alloc(al, tr.size() * 4 + 16, s) || !stats.alloc(al, (3 + kStatsCap) * 8, s) ||
        !res.NT.alloc(al, (uint64_t)nB * n * p.P * 8, s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (per-edge closure)");
    if (!tr.empty()) HIP_TRY(hipMemcpyAsync(trb.p, tr.data(), tr.size() * 4, hipMemcpyHostToDevice, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct EvGuard {
        hipEvent_t *a, *b;
        ~EvGuard() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } evg{&e0, &e1};
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    HIP_TRY(launch_fill(C.as<uint64_t>(), N * W, 0, s));
    HIP_TRY(launch_fill(M.as<uint64_t>(), mw, 0, s));
    HIP_TRY(launch_fill(dM.as<uint64_t>(), mw, 0, s));
    PerEdgeQuery q{};
    q.n = n; q.nQ = nQ; q.nB = nB; q.n_terms = p.n_terms; q.n_trans = (uint32_t)r.t_src.size();
    q.N = (uint32_t)N; q.W = (uint32_t)W; q.Wn = (uint32_t)Wn;
    q.soff = g.soff.as<uint32_t>(); q.sidx = g.sidx.as<uint32_t>();
    q.t_src = trb.as<uint32_t>(); q.t_sym = q.t_src + r.t_src.size(); q.t_dst = q.t_sym + r.t_src.size();
    q.starts = tb.starts; q.fin_off = tb.fin_off; q.fin = tb.fin; q.nullable = tb.nullable;
    q.C = C.as<uint64_t>(); q.M = M.as<uint64_t>(); q.dM = dM.as<uint64_t>();
    q.stats = stats.as<unsigned long long>();
    q.max_iters = o.max_iters; q.stats_cap = kStatsCap;
    HIP_TRY(launch_peredge(q, s));
    HIP_TRY(hipEventRecord(e1, s));
    // result layout: row v of box N holds the sources u (transposed rows)
    HIP_TRY(launch_fill(res.NT.as<uint64_t>(), (uint64_t)nB * n * p.P, 0, s));
    for (uint32_t b = 0; b < nB; ++b)
        HIP_TRY(launch_transpose(M.as<uint64_t>() + (uint64_t)b * n * Wn, (uint32_t)Wn,
                                 res.NT.as<uint64_t>() + (uint64_t)b * n * p.P, p.P, n, s));
    std::vector<unsigned long long> h(3 + kStatsCap);
    HIP_TRY(hipMemcpyAsync(h.data(), stats.p, h.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(wait_stream(s));
    if (h[1] != 0) return fail(CFPQ_ERR_LIMIT, "fixpoint did not stop within max_iters iterations");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    res.ms = ms;
    res.iterations = (uint32_t)h[0];
    res.deltas.assign(h.begin() + 3, h.begin() + 3 + std::min<uint64_t>(h[0], kStatsCap));
    return CFPQ_OK;
}

// ---------------------------------------------------------------------------
// FUSED strategy: a workgroup per query, many queries per launch
// ---------------------------------------------------------------------------
struct FusedJob {
    Plan plan;
    Tables tb;
    DevBuf work, T;
    FusedQuery q{};
    cfpq_result_s *res = nullptr;
    bool keep_blocks = false;
};

bool fused_ok(const cfpq_graph_s &g, const cfpq_rsm_s &r) {
    return g.n <= kFusedMaxN && r.n_boxes <= kFusedMaxBoxesHost;
}

// words of the fused kernel's work area beyond T and NT: the frontiers D, Dn,
// dNT, three activity bitsets, dnt_act and the statistics
uint64_t fused_work_words(const Plan &p) {
    const uint64_t qw = (uint64_t)p.nQ * p.n * p.P, bw = (uint64_t)p.nB * p.n * p.P;
    const uint64_t aw = (uint64_t)p.nQ * p.Pn, bb = (uint64_t)p.nB * p.Pn;
    return 2 * qw + bw + 3 * aw + bb + 2 + kStatsCap;
}

// the fused query's arguments with its buffers carved from work
// (fused_work_words(p) words); rank off, no iteration limit
void fill_fused(const Plan &p, const cfpq_graph_s &g, const Tables &tb, uint64_t *T, uint64_t *NT, uint64_t *w,
                FusedQuery &q) {
    const uint64_t qw = (uint64_t)p.nQ * p.n * p.P, bw = (uint64_t)p.nB * p.n * p.P;
    const uint64_t aw = (uint64_t)p.nQ * p.Pn, bb = (uint64_t)p.nB * p.Pn;
    q = FusedQuery{};
    q.n = p.n; q.P = p.P; q.Pn = p.Pn; q.n_terms = p.n_terms; q.nQ = p.nQ; q.nB = p.nB;
    q.goff = g.off.as<uint32_t>(); q.gidx = g.idx.as<uint32_t>();
    q.in_off = tb.in_off; q.in_tr = tb.in_tr; q.starts = tb.starts;
    q.fin_off = tb.fin_off; q.fin = tb.fin; q.nullable = tb.nullable; q.box_used = tb.box_used;
    q.T = T; q.NT = NT;
    q.D = w; w += qw;
    q.Dn = w; w += qw;
    q.dNT = w; w += bw;
    q.act = w; w += aw;
    q.actn = w; w += aw;
    q.tnz = w; w += aw;
    q.dnt_act = w; w += bb;
    q.stats = (unsigned long long *)w;
    q.rank = nullptr;
    q.max_iters = 0;
    q.stats_cap = kStatsCap;
    q.lds_ok = 1;
}

// Dynamic LDS words of a fused launch over queries qs[0..k): the largest
// working set that fits the device (with the odd LDS pitch where that fits
// too); 0 when none fits.  The device's limit is read once per device.
uint64_t fused_launch_lds(const FusedQuery *qs, size_t k) {
    constexpr int kMaxDevices = 64;
    static std::atomic<uint64_t> limit_plus1[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
    uint64_t lim = limit_plus1[dev].load(std::memory_order_relaxed);
    if (!lim) {
        lim = fused_lds_limit_words() + 1;
        limit_plus1[dev].store(lim, std::memory_order_relaxed);
    }
    const uint64_t limit = lim - 1;
    uint64_t words = 0;
    for (size_t i = 0; i < k; ++i) {
        const FusedQuery &q = qs[i];
        if (!q.lds_ok) continue;
        uint64_t need = fused_lds_words(q.n, q.Pn, q.Pn | 1u, q.nQ, q.nB);
        if (!CFPQ_FUSED_LDS_ODD || need > limit) need = fused_lds_words(q.n, q.Pn, q.Pn, q.nQ, q.nB);
        if (need <= limit && need > words) words = need;
    }
    return words;
}

cfpq_status prepare_fused(const cfpq_graph_s &g, const cfpq_rsm_s &r, const cfpq_query_opts &o,
                          cfpq_result_s &res, FusedJob &job) {
    hipStream_t s = (hipStream_t)o.stream;
    const Alloc *al = &res.alloc;
    job.plan = make_plan(g, r);
    cfpq_status st = upload_tables(job.plan, al, s, job.tb);
    if (st != CFPQ_OK) return st;
    const Plan &p = job.plan;
    const uint64_t qw = (uint64_t)p.nQ * p.n * p.P, bw = (uint64_t)p.nB * p.n * p.P;
    const uint64_t words = fused_work_words(p);
    if (!job.T.alloc(al, qw * 8, s) || !res.NT.alloc(al, bw * 8, s) || !job.work.alloc(al, words * 8, s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (fused query)");
    if (o.keep_rank) {
        if (!res.rank.alloc(al, (uint64_t)p.nB * p.n * p.n, s)) return fail(CFPQ_ERR_OOM, "device allocation failed (rank)");
        HIP_TRY(hipMemsetAsync(res.rank.p, 0xFF, (uint64_t)p.nB * p.n * p.n, s));
    }
    fill_fused(p, g, job.tb, job.T.as<uint64_t>(), res.NT.as<uint64_t>(), job.work.as<uint64_t>(), job.q);
    job.q.rank = o.keep_rank ? res.rank.as<uint8_t>() : nullptr;
    job.q.lds_ok = !o.keep_blocks;   // kept closure rows live in T's global buffer
    job.q.max_iters = o.max_iters;
    job.res = &res;
    job.keep_blocks = o.keep_blocks;
    return CFPQ_OK;
}

cfpq_status run_fused_jobs(std::vector<FusedJob> &jobs, const cfpq_query_opts &o, const Alloc *al) {
    if (jobs.empty()) return CFPQ_OK;
    hipStream_t s = (hipStream_t)o.stream;
    std::vector<FusedQuery> qs;
    for (auto &j : jobs) qs.push_back(j.q);
    DevBuf dq;
    if (!dq.alloc(al, qs.size() * sizeof(FusedQuery) + 64, s)) return fail(CFPQ_ERR_OOM, "device allocation failed");
    uint8_t *base = dq.as<uint8_t>();
    uint32_t *next = (uint32_t *)(base + qs.size() * sizeof(FusedQuery));
    HIP_TRY(hipMemcpyAsync(base, qs.data(), qs.size() * sizeof(FusedQuery), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(next, 0, 4, s));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    struct EvGuard {
        hipEvent_t *a, *b;
        ~EvGuard() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } evg{&ev0, &ev1};
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    HIP_TRY(hipEventRecord(ev0, s));
    HIP_TRY(launch_fused((const FusedQuery *)base, (uint32_t)qs.size(), next, fused_launch_lds(qs.data(), qs.size()), s));
    HIP_TRY(hipEventRecord(ev1, s));
    HIP_TRY(hipEventSynchronize(ev1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    std::vector<unsigned long long> stats(2 + kStatsCap);
    for (auto &j : jobs) {
        HIP_TRY(hipMemcpy(stats.data(), j.q.stats, stats.size() * 8, hipMemcpyDeviceToHost));
        if (stats[1] != 0) return fail(CFPQ_ERR_LIMIT, "fixpoint did not stop within max_iters iterations");
        j.res->iterations = (uint32_t)stats[0];
        j.res->deltas.assign(stats.begin() + 2, stats.begin() + 2 + std::min<uint64_t>(stats[0], kStatsCap));
        j.res->ms = ms;  // the launch's time, shared by the batch
        if (j.keep_blocks) j.res->T = std::move(j.T);
    }
    return CFPQ_OK;
}

// Fused queries prepared as one batch (queries that keep neither ranks nor
// closure blocks): one pinned staging buffer and one host-to-device copy for
// every table image, query record and the queue head; one work allocation
// (those, every query's statistics at a common pitch, then T and the work
// area of each query); one allocation for all answer matrices, which the
// results share; one read-back of every query's first statistics words.
constexpr uint32_t kBatchStatWords = 2 + 64;   // iterations, status, first 64 deltas
cfpq_status run_fused_batch(const std::vector<const cfpq_graph_s *> &gs, const std::vector<const cfpq_rsm_s *> &rs,
                            const std::vector<cfpq_result_s *> &out, const cfpq_query_opts &o) {
    const size_t k = out.size();
    if (!k) return CFPQ_OK;
    hipStream_t s = (hipStream_t)o.stream;
    std::vector<Plan> plans(k);
    std::vector<TableImage> ims(k);
    std::vector<uint64_t> o_tab(k), o_T(k), o_work(k), o_nt(k);
    uint64_t at = 0;
    for (size_t j = 0; j < k; ++j) {
        plans[j] = make_plan(*gs[j], *rs[j]);
        pack_tables(plans[j], ims[j]);
        o_tab[j] = at;
        at += align256(ims[j].host.size());
    }
    const uint64_t o_rec = at, o_head = o_rec + align256(k * sizeof(FusedQuery));
    const uint64_t staged = o_head + 256;   // these go up in one copy
    const uint64_t stat_pitch = 2 + kStatsCap;
    const uint64_t o_stats = staged;
    uint64_t total = o_stats + align256(k * stat_pitch * 8), nt_total = 0;
    for (size_t j = 0; j < k; ++j) {
        const Plan &p = plans[j];
        const uint64_t qw = (uint64_t)p.nQ * p.n * p.P, bw = (uint64_t)p.nB * p.n * p.P;
        o_T[j] = total;
        total += align256(qw * 8);
        o_work[j] = total;
        total += align256(fused_work_words(p) * 8);
        o_nt[j] = nt_total;
        nt_total += align256(bw * 8);
    }
    DevBuf work;
    auto ntb = std::make_shared<SharedDev>();
    ntb->al = out[0]->alloc;
    if (!work.alloc(&out[0]->alloc, total, s) || !ntb->buf.alloc(&ntb->al, nt_total, s))
        return fail(CFPQ_ERR_OOM, "device allocation failed (fused batch)");
    PinnedCounters pin;   // the staging area, later the statistics read-back
    if (!pin.ensure(std::max<uint64_t>(staged / 8, k * kBatchStatWords)))
        return fail(CFPQ_ERR_OOM, "pinned host allocation failed");
    uint8_t *h = reinterpret_cast<uint8_t *>(pin.h);
    uint8_t *wk = work.as<uint8_t>(), *ntp = ntb->buf.as<uint8_t>();
    std::vector<FusedQuery> rec(k);
    for (size_t j = 0; j < k; ++j) {
        std::memcpy(h + o_tab[j], ims[j].host.data(), ims[j].host.size());
        Tables tb;
        bind_tables(ims[j], wk + o_tab[j], tb);
        fill_fused(plans[j], *gs[j], tb, (uint64_t *)(wk + o_T[j]), (uint64_t *)(ntp + o_nt[j]),
                   (uint64_t *)(wk + o_work[j]), rec[j]);
        rec[j].stats = (unsigned long long *)(wk + o_stats) + j * stat_pitch;
        rec[j].max_iters = o.max_iters;
    }
    std::memcpy(h + o_rec, rec.data(), k * sizeof(FusedQuery));
    std::memset(h + o_head, 0, 256);
    HIP_TRY(hipMemcpyAsync(wk, h, staged, hipMemcpyHostToDevice, s));
    PooledEvents evp;
    HIP_TRY(evp.ensure(2));
    HIP_TRY(hipEventRecord(evp.v[0], s));
    HIP_TRY(launch_fused((const FusedQuery *)(wk + o_rec), (uint32_t)k, (uint32_t *)(wk + o_head),
                         fused_launch_lds(rec.data(), k), s));
    HIP_TRY(hipEventRecord(evp.v[1], s));
    // after the staging copy on the same stream: the pinned area is free
    HIP_TRY(hipMemcpy2DAsync(h, kBatchStatWords * 8, wk + o_stats, stat_pitch * 8, kBatchStatWords * 8, k,
                             hipMemcpyDeviceToHost, s));
    HIP_TRY(wait_stream(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, evp.v[0], evp.v[1]));
    const unsigned long long *st = pin.h;
    for (size_t j = 0; j < k; ++j) {
        const unsigned long long *sj = st + j * kBatchStatWords;
        if (sj[1] != 0) return fail(CFPQ_ERR_LIMIT, "fixpoint did not stop within max_iters iterations");
        const uint64_t it = sj[0], nd = std::min<uint64_t>(it, kStatsCap);
        cfpq_result_s &res = *out[j];
        res.iterations = (uint32_t)it;
        res.deltas.assign(sj + 2, sj + 2 + std::min<uint64_t>(nd, kBatchStatWords - 2));
        if (nd > kBatchStatWords - 2) {   // a long fixpoint: the rest of its deltas
            res.deltas.resize(nd);
            HIP_TRY(hipMemcpy(res.deltas.data() + (kBatchStatWords - 2), rec[j].stats + kBatchStatWords,
                              (nd - (kBatchStatWords - 2)) * 8, hipMemcpyDeviceToHost));
        }
        res.ms = ms;   // the launch's time, shared by the batch
        res.NT.release();
        res.NT.p = ntp + o_nt[j];
        res.NT.bytes = (size_t)plans[j].nB * plans[j].n * plans[j].P * 8;
        res.NT.al = nullptr;   // a view: the block is freed with its last result
        res.NT.s = s;
        res.nt_block = ntb;
    }
    return CFPQ_OK;
}

cfpq_result_s *new_result(const cfpq_graph_s &g, const cfpq_rsm_s &r, const cfpq_query_opts &o) {
    cfpq_result_s *res = new (std::nothrow) cfpq_result_s;
    if (!res) return nullptr;
    res->device = g.device;
    res->n = g.n;
    res->Pn = (g.n + 63) / 64;
    res->P = row_pitch(res->Pn);
    res->nB = r.n_boxes;
    res->nQ = r.n_states;
    res->stream = (hipStream_t)o.stream;
    res->alloc = Alloc(o.alloc);
    res->rsm = r;
    res->n_labels = g.n_labels;
    res->hcsr = g.hcsr;
    return res;
}

bool has_calls(const cfpq_rsm_s &r) {
    for (uint32_t sym : r.t_sym)
        if (sym >= r.n_terms) return true;
    return false;
}

cfpq_status check_opts(const cfpq_graph_s &g, const cfpq_rsm_s &r, const cfpq_query_opts &o) {
    if (o.strategy > CFPQ_STRATEGY_PEREDGE) return fail(CFPQ_ERR_INVALID, "unknown strategy");
    if (o.strategy == CFPQ_STRATEGY_PEREDGE) {
        if (o.keep_rank || o.keep_blocks)
            return fail(CFPQ_ERR_INVALID, "per-edge strategy keeps neither ranks nor closure blocks");
        if (!peredge_ok(g, r))
            return fail(CFPQ_ERR_LIMIT, "per-edge strategy needs states * n <= 65536 (the whole product closure)");
    }
    if (o.nt_mode > CFPQ_NT_MFMA) return fail(CFPQ_ERR_INVALID, "unknown nt_mode");
    if (o.strategy == CFPQ_STRATEGY_CONDENSED && has_calls(r))
        return fail(CFPQ_ERR_INVALID, "condensed strategy needs an RSM without box-labelled transitions");
    if (o.keep_rank && (uint64_t)r.n_boxes * g.n * g.n > kRankMaxBytes)
        return fail(CFPQ_ERR_LIMIT, "keep_rank: boxes * n^2 bytes of ranks exceed the 64 GiB limit");
    if (o.strategy == CFPQ_STRATEGY_FUSED && !fused_ok(g, r))
        return fail(CFPQ_ERR_LIMIT, "fused strategy needs n <= 2048 and at most 64 boxes");
    return CFPQ_OK;
}

// AUTO runs a single query fused up to 512 vertices: rows of at most 8 words
// get a thread each there; past that a wavefront per row makes the one
// workgroup 10x slower (n = 512 -> 640: brackets 1.8 -> 18 ms, same
// generation 0.9 -> 10 ms, alias 3.7 -> 65 ms), while the multi-launch
// strategies take 0.5-5 ms at these sizes
constexpr uint32_t kFusedAutoMaxN = 512;

bool use_fused(const cfpq_graph_s &g, const cfpq_rsm_s &r, const cfpq_query_opts &o) {
    if (o.strategy == CFPQ_STRATEGY_FUSED) return true;
    if (o.strategy != CFPQ_STRATEGY_AUTO) return false;
    return fused_ok(g, r) && g.n <= kFusedAutoMaxN;
}

cfpq_status run_big(const cfpq_graph_s &g, const cfpq_rsm_s &r, const cfpq_query_opts &o, cfpq_result_s &res) {
    if (o.strategy == CFPQ_STRATEGY_PEREDGE) return run_peredge(g, r, o, res);
    const bool cond = o.strategy == CFPQ_STRATEGY_CONDENSED ||
                      (o.strategy == CFPQ_STRATEGY_AUTO && !has_calls(r) && (uint64_t)r.n_states * g.n < 0xFFFFFFFFull);
    return cond ? run_condensed(g, r, o, res) : run_levels(g, r, o, res);
}

}  // namespace

extern "C" cfpq_status cfpq_query(cfpq_graph g, cfpq_rsm r, const cfpq_query_opts *opts, cfpq_result *out) {
    if (!out) return fail(CFPQ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    cfpq_status st = check_pair(g, r);
    if (st != CFPQ_OK) return st;
    cfpq_query_opts o{};
    if (opts) o = *opts;
    if ((st = check_opts(*g, *r, o)) != CFPQ_OK) return st;
    std::unique_ptr<cfpq_result_s> res(new_result(*g, *r, o));
    if (!res) return fail(CFPQ_ERR_OOM, "host allocation failed");
    try {
        // masks: device copies with the bits past n cleared
        DevBuf dmask;
        const uint32_t Pn = (g->n + 63) / 64;
        hipStream_t s = (hipStream_t)o.stream;
        uint64_t *d_src = nullptr, *d_dst = nullptr;
        if (o.src_mask || o.dst_mask) {
            if (!dmask.alloc(&res->alloc, 2ull * Pn * 8, s)) return fail(CFPQ_ERR_OOM, "device allocation failed (masks)");
            std::vector<uint64_t> h(2ull * Pn, ~0ull);
            if (o.src_mask) std::memcpy(h.data(), o.src_mask, (size_t)Pn * 8);
            if (o.dst_mask) std::memcpy(h.data() + Pn, o.dst_mask, (size_t)Pn * 8);
            if (g->n % 64) {
                const uint64_t keep = (1ull << (g->n % 64)) - 1;
                h[Pn - 1] &= keep;
                h[2 * Pn - 1] &= keep;
            }
            HIP_TRY(hipMemcpyAsync(dmask.p, h.data(), h.size() * 8, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            d_src = o.src_mask ? dmask.as<uint64_t>() : nullptr;
            d_dst = o.dst_mask ? dmask.as<uint64_t>() + Pn : nullptr;
            // a query without box-labelled transitions searches only the
            // masked sources; with them every source is needed
            if (d_src && !has_calls(*r)) {
                if (!res->src_mask.alloc(&res->alloc, (size_t)Pn * 8, s))
                    return fail(CFPQ_ERR_OOM, "device allocation failed (masks)");
                HIP_TRY(hipMemcpyAsync(res->src_mask.p, d_src, (size_t)Pn * 8, hipMemcpyDeviceToDevice, s));
            }
        }
        if (use_fused(*g, *r, o) && !o.keep_rank && !o.keep_blocks) {
            if ((st = run_fused_batch({g}, {r}, {res.get()}, o)) != CFPQ_OK) return st;
        } else if (use_fused(*g, *r, o)) {
            std::vector<FusedJob> jobs(1);
            if ((st = prepare_fused(*g, *r, o, *res, jobs[0])) != CFPQ_OK) return st;
            if ((st = run_fused_jobs(jobs, o, &res->alloc)) != CFPQ_OK) return st;
        } else {
            if ((st = run_big(*g, *r, o, *res)) != CFPQ_OK) return st;
        }
        if (d_src || d_dst) {
            const uint64_t P = res->P;
            HIP_TRY(launch_mask_rows(res->NT.as<uint64_t>() + (uint64_t)r->start_box * g->n * P, g->n, (uint32_t)P,
                                     Pn, d_src, d_dst, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    } catch (const std::bad_alloc &) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    *out = res.release();
    return CFPQ_OK;
}

extern "C" cfpq_status cfpq_query_batch(const cfpq_graph *graphs, const cfpq_rsm *rsms, uint32_t k,
                                        const cfpq_query_opts *opts, cfpq_result *results) {
    if (!results || (k && (!graphs || !rsms))) return fail(CFPQ_ERR_INVALID, "NULL array");
    for (uint32_t i = 0; i < k; ++i) results[i] = nullptr;
    cfpq_query_opts o{};
    if (opts) o = *opts;
    if (o.src_mask || o.dst_mask) return fail(CFPQ_ERR_INVALID, "vertex masks are not accepted by the batched call");
    std::vector<std::unique_ptr<cfpq_result_s>> res(k);
    cfpq_status st = CFPQ_OK;
    try {
        std::vector<FusedJob> jobs;
        std::vector<uint32_t> big;
        // fused queries that keep neither ranks nor blocks: one batch
        const bool batched = !o.keep_rank && !o.keep_blocks;
        std::vector<const cfpq_graph_s *> bg;
        std::vector<const cfpq_rsm_s *> br;
        std::vector<cfpq_result_s *> bres;
        for (uint32_t i = 0; i < k; ++i) {
            if ((st = check_pair(graphs[i], rsms[i])) != CFPQ_OK) return st;
            if ((st = check_opts(*graphs[i], *rsms[i], o)) != CFPQ_OK) return st;
            res[i].reset(new_result(*graphs[i], *rsms[i], o));
            if (!res[i]) return fail(CFPQ_ERR_OOM, "host allocation failed");
            if (use_fused(*graphs[i], *rsms[i], o) && batched) {
                bg.push_back(graphs[i]);
                br.push_back(rsms[i]);
                bres.push_back(res[i].get());
            } else if (use_fused(*graphs[i], *rsms[i], o)) {
                jobs.emplace_back();
                if ((st = prepare_fused(*graphs[i], *rsms[i], o, *res[i], jobs.back())) != CFPQ_OK) return st;
            } else {
                big.push_back(i);
            }
        }
        if ((st = run_fused_batch(bg, br, bres, o)) != CFPQ_OK) return st;
        if ((st = run_fused_jobs(jobs, o, k ? &res[0]->alloc : nullptr)) != CFPQ_OK) return st;
        jobs.clear();
        for (uint32_t i : big)
            if ((st = run_big(*graphs[i], *rsms[i], o, *res[i])) != CFPQ_OK) return st;
    } catch (const std::bad_alloc &) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    for (uint32_t i = 0; i < k; ++i) results[i] = res[i].release();
    return CFPQ_OK;
}

// ---------------------------------------------------------------------------
// query without device allocation: the fused fixpoint with its whole working
// set in a static device array
// ---------------------------------------------------------------------------
namespace noalloc {
// One copy per device, resident from the library's first use of that device
// until the process ends.  Host code never takes this name's address: a
// kernel given it would fault.  It uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint64_t scratch[CFPQ_NOALLOC_SCRATCH_BYTES / 8];
}  // namespace noalloc

namespace {

constexpr int kNoAllocDevices = 64;
// per device: a lock held for a whole call (calls in one process never
// overlap on a device) and the device address of that device's array
std::mutex g_noalloc_mu[kNoAllocDevices];
uint64_t *g_noalloc_ptr[kNoAllocDevices];

// the array's device address on device dev (current); the caller holds
// g_noalloc_mu[dev]
cfpq_status noalloc_scratch(int dev, uint64_t **out) {
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc::scratch));
        if (e != hipSuccess || !p)
            return fail(CFPQ_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_noalloc_ptr[dev] = static_cast<uint64_t *>(p);
    }
    *out = g_noalloc_ptr[dev];
    return CFPQ_OK;
}

}  // namespace

extern "C" cfpq_status cfpq_query_noalloc(cfpq_graph g, cfpq_rsm r, uint32_t box, uint64_t *dst, uint64_t dst_words,
                                          uint64_t *pairs, uint32_t *iterations, void *stream) {
    cfpq_status st = check_pair(g, r);
    if (st != CFPQ_OK) return st;
    if (box >= r->n_boxes) return fail(CFPQ_ERR_INVALID, "box out of range");
    if (!dst) return fail(CFPQ_ERR_INVALID, "dst is NULL");
    const uint32_t n = g->n, Pn = (n + 63) / 64;
    const uint64_t need = (uint64_t)n * Pn;
    if (dst_words < need) return fail(CFPQ_ERR_BUFFER, "bitmap buffer too small: need " + std::to_string(need) + " words");
    if (!fused_ok(*g, *r)) return fail(CFPQ_ERR_LIMIT, "cfpq_query_noalloc needs n <= 2048 and at most 64 boxes");
    const int dev = g->device;
    if (dev < 0 || dev >= kNoAllocDevices) return fail(CFPQ_ERR_LIMIT, "device index beyond the static table");
    hipStream_t s = (hipStream_t)stream;
    try {
        const Plan p = make_plan(*g, *r);
        TableImage im;
        pack_tables(p, im);
        // layout: control words (queue head, pair count), the query's
        // arguments, the tables, T, NT, the rest of the work area
        const uint64_t qw = (uint64_t)p.nQ * p.n * p.P, bw = (uint64_t)p.nB * p.n * p.P;
        const uint64_t o_args = 256, o_tab = o_args + align256(sizeof(FusedQuery));
        const uint64_t o_T = o_tab + align256(im.host.size());
        const uint64_t o_NT = o_T + align256(qw * 8), o_work = o_NT + align256(bw * 8);
        const uint64_t total = o_work + fused_work_words(p) * 8;
        if (total > CFPQ_NOALLOC_SCRATCH_BYTES)
            return fail(CFPQ_ERR_LIMIT, "query needs " + std::to_string(total) + " bytes of working set, the static " +
                                            "array holds " + std::to_string((uint64_t)CFPQ_NOALLOC_SCRATCH_BYTES));
        std::lock_guard<std::mutex> lk(g_noalloc_mu[dev]);
        uint64_t *base = nullptr;
        if ((st = noalloc_scratch(dev, &base)) != CFPQ_OK) return st;
        uint8_t *b8 = reinterpret_cast<uint8_t *>(base);
        Tables tb;
        bind_tables(im, b8 + o_tab, tb);
        FusedQuery q{};
        fill_fused(p, *g, tb, (uint64_t *)(b8 + o_T), (uint64_t *)(b8 + o_NT), (uint64_t *)(b8 + o_work), q);
        uint32_t *next = (uint32_t *)b8;
        unsigned long long *count = (unsigned long long *)(b8 + 8);
        // the previous call's contents are still there: the queue head and
        // the count start at zero; the kernel clears its own buffers
        HIP_TRY(launch_fill(base, 2, 0, s));
        HIP_TRY(hipMemcpyAsync(b8 + o_tab, im.host.data(), im.host.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b8 + o_args, &q, sizeof(q), hipMemcpyHostToDevice, s));
        HIP_TRY(launch_fused((const FusedQuery *)(b8 + o_args), 1, next, fused_launch_lds(&q, 1), s));
        const uint64_t *rows = q.NT + (uint64_t)box * n * p.P;
        HIP_TRY(launch_transpose(rows, p.P, dst, Pn, n, s));
        HIP_TRY(launch_popcount(rows, n, p.P, Pn, count, s));
        unsigned long long stats[2] = {0, 0}, cnt = 0;
        HIP_TRY(hipMemcpyAsync(stats, q.stats, sizeof(stats), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&cnt, count, sizeof(cnt), hipMemcpyDeviceToHost, s));
        HIP_TRY(wait_stream(s));
        if (stats[1] != 0) return fail(CFPQ_ERR_LIMIT, "fixpoint did not stop");
        if (pairs) *pairs = cnt;
        if (iterations) *iterations = (uint32_t)stats[0];
    } catch (const std::bad_alloc &) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    return CFPQ_OK;
}

// ---------------------------------------------------------------------------
// result accessors
// ---------------------------------------------------------------------------
namespace {

cfpq_status check_box(cfpq_result r, uint32_t box) {
    if (!r) return fail(CFPQ_ERR_INVALID, "result is NULL");
    if (box >= r->nB) return fail(CFPQ_ERR_INVALID, "box out of range");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != r->device) return fail(CFPQ_ERR_INVALID, "result lives on another device");
    return CFPQ_OK;
}

cfpq_status scratch_u64(cfpq_result r, unsigned long long **p) {
    if (!r->scratch.p && !r->scratch.alloc(&r->alloc, 64, r->stream))
        return fail(CFPQ_ERR_OOM, "device allocation failed");
    *p = r->scratch.as<unsigned long long>();
    return CFPQ_OK;
}

// transposed rows [n][P] -> row-major bitmap [n][Pn] at dst (device)
cfpq_status to_rowmajor(cfpq_result r, const uint64_t *src, uint64_t *dst_dev) {
    HIP_TRY(launch_transpose(src, r->P, dst_dev, r->Pn, r->n, r->stream));
    return CFPQ_OK;
}

cfpq_status fetch_bitmap(cfpq_result r, const uint64_t *src, uint64_t *dst, uint64_t dst_words,
                         int on_device) {
    const uint64_t need = (uint64_t)r->n * r->Pn;
    if (!dst) return fail(CFPQ_ERR_INVALID, "dst is NULL");
    if (dst_words < need) return fail(CFPQ_ERR_BUFFER, "bitmap buffer too small: need " + std::to_string(need) + " words");
    if (on_device) {
        cfpq_status st = to_rowmajor(r, src, dst);
        if (st != CFPQ_OK) return st;
        HIP_TRY(hipStreamSynchronize(r->stream));
        return CFPQ_OK;
    }
    DevBuf tmp;
    if (!tmp.alloc(&r->alloc, need * 8, r->stream)) return fail(CFPQ_ERR_OOM, "device allocation failed");
    cfpq_status st = to_rowmajor(r, src, tmp.as<uint64_t>());
    if (st != CFPQ_OK) return st;
    HIP_TRY(hipMemcpyAsync(dst, tmp.p, need * 8, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return CFPQ_OK;
}

const uint64_t *box_rows(cfpq_result r, uint32_t box) {
    return r->NT.as<uint64_t>() + (uint64_t)box * r->n * r->P;
}

}  // namespace

extern "C" cfpq_status cfpq_result_count(cfpq_result r, uint32_t box, uint64_t *pairs) {
    cfpq_status st = check_box(r, box);
    if (st != CFPQ_OK) return st;
    if (!pairs) return fail(CFPQ_ERR_INVALID, "pairs is NULL");
    unsigned long long *d = nullptr;
    if ((st = scratch_u64(r, &d)) != CFPQ_OK) return st;
    HIP_TRY(hipMemsetAsync(d, 0, 8, r->stream));
    HIP_TRY(launch_popcount(box_rows(r, box), r->n, r->P, r->Pn, d, r->stream));
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, d, 8, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    *pairs = h;
    return CFPQ_OK;
}

extern "C" cfpq_status cfpq_result_hash(cfpq_result r, uint32_t box, uint64_t *hash) {
    cfpq_status st = check_box(r, box);
    if (st != CFPQ_OK) return st;
    if (!hash) return fail(CFPQ_ERR_INVALID, "hash is NULL");
    unsigned long long *d = nullptr;
    if ((st = scratch_u64(r, &d)) != CFPQ_OK) return st;
    HIP_TRY(hipMemsetAsync(d, 0, 8, r->stream));
    HIP_TRY(launch_hash(box_rows(r, box), r->n, r->P, d, r->stream));
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, d, 8, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    *hash = h;
    return CFPQ_OK;
}

extern "C" cfpq_status cfpq_result_bitmap(cfpq_result r, uint32_t box, uint64_t *dst, uint64_t dst_words,
                                          int dst_on_device) {
    cfpq_status st = check_box(r, box);
    if (st != CFPQ_OK) return st;
    return fetch_bitmap(r, box_rows(r, box), dst, dst_words, dst_on_device);
}

extern "C" cfpq_status cfpq_result_pairs(cfpq_result r, uint32_t box, uint32_t *uv, uint64_t cap_pairs,
                                         uint64_t *n_pairs) {
    cfpq_status st = check_box(r, box);
    if (st != CFPQ_OK) return st;
    if (!n_pairs) return fail(CFPQ_ERR_INVALID, "n_pairs is NULL");
    uint64_t cnt = 0;
    if ((st = cfpq_result_count(r, box, &cnt)) != CFPQ_OK) return st;
    *n_pairs = cnt;
    if (cap_pairs < cnt) return fail(CFPQ_ERR_BUFFER, "pairs buffer too small: need " + std::to_string(cnt));
    if (cnt && !uv) return fail(CFPQ_ERR_INVALID, "uv is NULL");
    std::vector<uint64_t> bm;
    try {
        bm.resize((uint64_t)r->n * r->Pn);
    } catch (...) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    if ((st = fetch_bitmap(r, box_rows(r, box), bm.data(), bm.size(), 0)) != CFPQ_OK) return st;
    uint64_t k = 0;
    for (uint32_t u = 0; u < r->n; ++u)
        for (uint32_t w = 0; w < r->Pn; ++w) {
            uint64_t bits = bm[(uint64_t)u * r->Pn + w];
            while (bits) {
                const int b = __builtin_ctzll(bits);
                bits &= bits - 1;
                uv[2 * k] = u;
                uv[2 * k + 1] = w * 64 + b;
                ++k;
            }
        }
    return CFPQ_OK;
}

extern "C" cfpq_status cfpq_result_block(cfpq_result r, uint32_t q_start, uint32_t q_final, uint64_t *dst,
                                         uint64_t dst_words) {
    if (!r) return fail(CFPQ_ERR_INVALID, "result is NULL");
    if (!r->T.p) return fail(CFPQ_ERR_INVALID, "closure blocks were not kept (keep_blocks)");
    if (q_start >= r->nQ || q_final >= r->nQ) return fail(CFPQ_ERR_INVALID, "state out of range");
    const uint32_t b = r->rsm.state_box[q_final];
    if (r->rsm.box_start[b] != q_start)
        return fail(CFPQ_ERR_INVALID, "q_start is not the initial state of q_final's box");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != r->device) return fail(CFPQ_ERR_INVALID, "result lives on another device");
    return fetch_bitmap(r, r->T.as<uint64_t>() + (uint64_t)q_final * r->n * r->P, dst, dst_words, 0);
}

extern "C" cfpq_status cfpq_result_stats(cfpq_result r, uint32_t *iterations, uint64_t *delta, uint32_t cap,
                                         double *fixpoint_ms) {
    if (!r) return fail(CFPQ_ERR_INVALID, "result is NULL");
    if (iterations) *iterations = r->iterations;
    if (delta)
        for (uint32_t i = 0; i < cap && i < r->deltas.size(); ++i) delta[i] = r->deltas[i];
    if (fixpoint_ms) *fixpoint_ms = r->ms;
    return CFPQ_OK;
}

extern "C" cfpq_status cfpq_result_profile(cfpq_result r, uint32_t kind, uint64_t *launches, double *ms,
                                           uint64_t *bytes) {
    if (!r) return fail(CFPQ_ERR_INVALID, "result is NULL");
    if (!r->profiled) return fail(CFPQ_ERR_INVALID, "query was not profiled (opts.profile)");
    if (kind > CFPQ_KERNEL_NT_DENSE) return fail(CFPQ_ERR_INVALID, "unknown kernel kind");
    if (launches) *launches = r->prof[kind].launches;
    if (ms) *ms = r->prof[kind].ms;
    if (bytes) *bytes = r->prof[kind].bytes;
    return CFPQ_OK;
}

// ---------------------------------------------------------------------------
// single witness (Sec. 3.2)
// ---------------------------------------------------------------------------
namespace {

struct Witness {
    cfpq_result r;
    std::vector<uint32_t> *out;
    uint64_t limit;
    bool overflow = false;
    cfpq_status err = CFPQ_OK;

    uint8_t rank(uint32_t N, uint32_t u, uint32_t v) {
        uint8_t b = 0xFF;
        if (hipMemcpy(&b, r->rank.as<uint8_t>() + ((uint64_t)N * r->n + u) * r->n + v, 1, hipMemcpyDeviceToHost) !=
            hipSuccess)
            err = fail(CFPQ_ERR_DEVICE, "rank read failed");
        return b;
    }

    // breadth-first search on the device inside box N from (start, u) to
    // (final, v), over terminal edges and nonterminal edges of rank < rk;
    // the path found is expanded (nonterminal edges recursively)
    bool expand(uint32_t N, uint32_t u, uint32_t v, uint8_t rk) {
        if (overflow || err != CFPQ_OK) return false;
        if (rk == 0) return u == v;  // the epsilon loop: empty path
        cfpq_result_s::WitnessDev &W = *r->wdev;
        const cfpq_rsm_s &R = r->rsm;
        const uint32_t n = r->n;
        const uint64_t nodes = (uint64_t)R.n_states * n;
        hipStream_t s = r->stream;
        const uint32_t s0 = R.box_start[N] * n + u;
        if ((err = fill_start(W, nodes, s0, s)) != CFPQ_OK) return false;
        WitnessBfs b{};
        b.n = n; b.n_terms = R.n_terms; b.s_off = W.s_off; b.s_tr = W.s_tr; b.final = W.fin;
        b.soff = W.off; b.sidx = W.idx; b.rank = r->rank.p ? r->rank.as<uint8_t>() : nullptr; b.rk = rk;
        b.v_target = v; b.par = W.par; b.psym = W.psym; b.ctr = W.ctr;
        uint32_t *cur = W.fr[0], *nxt = W.fr[1];
        uint32_t ncur = 1, hit = kNoSlot;
        while (ncur && hit == kNoSlot) {
            b.cur = cur; b.ncur = ncur; b.next = nxt;
            if (hipMemsetAsync(W.ctr, 0, 4, s) != hipSuccess || launch_witness_bfs(b, s) != hipSuccess) {
                err = fail(CFPQ_ERR_DEVICE, "witness search launch failed");
                return false;
            }
            unsigned int c[2] = {0, 0};
            if (hipMemcpyAsync(c, W.ctr, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
                err = fail(CFPQ_ERR_DEVICE, "witness search read failed");
                return false;
            }
            ncur = c[0];
            hit = c[1];
            std::swap(cur, nxt);
        }
        if (hit == kNoSlot) return false;
        // walk back along the parent pointers
        std::vector<std::array<uint32_t, 3>> steps;  // (x, sym, y)
        for (uint32_t id = hit; id != s0;) {
            uint32_t ps[2];
            if (hipMemcpy(&ps[0], W.par + id, 4, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(&ps[1], W.psym + id, 4, hipMemcpyDeviceToHost) != hipSuccess) {
                err = fail(CFPQ_ERR_DEVICE, "witness path read failed");
                return false;
            }
            steps.push_back({ps[0] % n, ps[1], id % n});
            id = ps[0];
            if (steps.size() > nodes) {
                err = fail(CFPQ_ERR_DEVICE, "internal error: parent pointers form a cycle");
                return false;
            }
        }
        std::reverse(steps.begin(), steps.end());
        for (auto &st : steps) {
            if (st[1] < R.n_terms) {
                if (out->size() / 3 >= limit) {
                    overflow = true;
                    return false;
                }
                out->push_back(st[0]);
                out->push_back(st[1]);
                out->push_back(st[2]);
            } else {
                const uint32_t M = st[1] - R.n_terms;
                const uint8_t rm = rank(M, st[0], st[2]);
                if (err != CFPQ_OK || !expand(M, st[0], st[2], rm)) return false;
            }
        }
        return true;
    }

    // no node reached yet except s0, which is its own parent and frontier 0
    static cfpq_status fill_start(cfpq_result_s::WitnessDev &W, uint64_t nodes, uint32_t s0, hipStream_t s) {
        HIP_TRY(launch_fill_u32(W.par, nodes, kNoSlot, s));
        HIP_TRY(launch_fill_u32(W.par + s0, 1, s0, s));
        HIP_TRY(launch_fill_u32(W.fr[0], 1, s0, s));
        HIP_TRY(launch_fill_u32(W.ctr + 1, 1, kNoSlot, s));
        return CFPQ_OK;
    }
};

cfpq_status witness_setup(cfpq_result r) {
    if (r->wdev) return CFPQ_OK;
    const cfpq_rsm_s &R = r->rsm;
    const uint32_t n = r->n, nQ = R.n_states;
    const uint64_t nodes = (uint64_t)nQ * n;
    const HostCsr &H = *r->hcsr;
    std::vector<uint32_t> s_off(nQ + 1, 0);
    std::vector<InTrans> s_tr(R.t_src.size());
    for (size_t i = 0; i < R.t_src.size(); ++i) s_off[R.t_src[i] + 1]++;
    for (uint32_t q = 0; q < nQ; ++q) s_off[q + 1] += s_off[q];
    std::vector<uint32_t> fill(s_off.begin(), s_off.end() - 1);
    for (size_t i = 0; i < R.t_src.size(); ++i) s_tr[fill[R.t_src[i]]++] = InTrans{R.t_dst[i], R.t_sym[i]};
    std::vector<uint32_t> fin(nQ);
    for (uint32_t q = 0; q < nQ; ++q) fin[q] = R.is_final[q] ? 1u : 0u;
    // layout (4-byte words): off, idx, s_off, s_tr (2 words each), fin, par, psym, fr0, fr1, ctr
    const uint64_t w_off = H.off.size(), w_idx = H.out.size() + 1, w_soff = s_off.size(), w_str = 2 * s_tr.size() + 2,
                   w_fin = fin.size(), w_node = nodes;
    const uint64_t total = w_off + w_idx + w_soff + w_str + w_fin + 4 * w_node + 4;
    auto W = std::make_unique<cfpq_result_s::WitnessDev>();
    if (!W->buf.alloc(&r->alloc, total * 4, r->stream)) return fail(CFPQ_ERR_OOM, "device allocation failed (witness)");
    uint32_t *b = W->buf.as<uint32_t>();
    W->off = b; b += w_off;
    W->idx = b; b += w_idx;
    W->s_off = b; b += w_soff;
    W->s_tr = reinterpret_cast<InTrans *>(b); b += w_str;
    W->fin = b; b += w_fin;
    W->par = b; b += w_node;
    W->psym = b; b += w_node;
    W->fr[0] = b; b += w_node;
    W->fr[1] = b; b += w_node;
    W->ctr = reinterpret_cast<unsigned int *>(b);
    hipStream_t s = r->stream;
    HIP_TRY(hipMemcpyAsync(W->off, H.off.data(), H.off.size() * 4, hipMemcpyHostToDevice, s));
    if (!H.out.empty()) HIP_TRY(hipMemcpyAsync(W->idx, H.out.data(), H.out.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W->s_off, s_off.data(), s_off.size() * 4, hipMemcpyHostToDevice, s));
    if (!s_tr.empty()) HIP_TRY(hipMemcpyAsync(W->s_tr, s_tr.data(), s_tr.size() * sizeof(InTrans), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W->fin, fin.data(), fin.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));   // the host vectors die with this frame
    r->wdev = std::move(W);
    return CFPQ_OK;
}

bool has_box_calls(const cfpq_rsm_s &R) {
    for (uint32_t sym : R.t_sym)
        if (sym >= R.n_terms) return true;
    return false;
}

}  // namespace

extern "C" cfpq_status cfpq_extract_path(cfpq_result r, uint32_t box, uint32_t u, uint32_t v, uint32_t *edges,
                                         uint64_t cap_edges, uint64_t *n_edges) {
    cfpq_status st = check_box(r, box);
    if (st != CFPQ_OK) return st;
    if (!n_edges) return fail(CFPQ_ERR_INVALID, "n_edges is NULL");
    const bool calls = has_box_calls(r->rsm);
    if (calls && !r->rank.p) return fail(CFPQ_ERR_INVALID, "ranks were not kept (keep_rank)");
    if (u >= r->n || v >= r->n) return fail(CFPQ_ERR_INVALID, "vertex out of range");
    if (calls && r->iterations > 254) return fail(CFPQ_ERR_LIMIT, "more than 254 iterations: ranks saturated");
    try {
        {   // the relation as returned (a vertex mask may have removed the pair)
            uint64_t word = 0;
            HIP_TRY(hipMemcpy(&word, r->NT.as<uint64_t>() + ((uint64_t)box * r->n + v) * r->P + (u >> 6), 8,
                              hipMemcpyDeviceToHost));
            if (!((word >> (u & 63)) & 1ull)) return fail(CFPQ_ERR_NOT_FOUND, "pair not in the relation");
        }
        if ((st = witness_setup(r)) != CFPQ_OK) return st;
        std::vector<uint32_t> out;
        Witness w{r, &out, (uint64_t)1 << 26};
        // rank of the pair: the iteration that added it (0: the epsilon loop);
        // a regular query has no ranks: a path of length >= 1, or the empty
        // path where the box derives the empty word
        uint8_t rk;
        if (calls) {
            rk = w.rank(box, u, v);
            if (w.err != CFPQ_OK) return w.err;
            if (rk == 0xFF) return fail(CFPQ_ERR_NOT_FOUND, "pair not in the relation");
        } else {
            rk = (u == v && r->rsm.is_final[r->rsm.box_start[box]]) ? 0 : 1;
        }
        if (!w.expand(box, u, v, rk)) {
            if (w.err != CFPQ_OK) return w.err;
            if (w.overflow) return fail(CFPQ_ERR_LIMIT, "witness longer than 2^26 edges");
            return fail(CFPQ_ERR_DEVICE, "internal error: no witness through lower-rank edges");
        }
        *n_edges = out.size() / 3;
        if (cap_edges < out.size() / 3) return fail(CFPQ_ERR_BUFFER, "edge buffer too small");
        if (!out.empty()) {
            if (!edges) return fail(CFPQ_ERR_INVALID, "edges is NULL");
            std::memcpy(edges, out.data(), out.size() * 4);
        }
    } catch (const std::bad_alloc &) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    return CFPQ_OK;
}

extern "C" void cfpq_result_destroy(cfpq_result r) { delete r; }

// ---------------------------------------------------------------------------
// all paths of bounded length (Sec. 3.2, paths extraction)
//
// Grammar view of the RSM: X_q derives the words that lead from state q to a
// final state of q's box (rules X_q -> eps if q is final, X_q -> T_t X_q' for
// a terminal transition, X_q -> X_start(N) X_q' for a box-labelled one; T_t
// -> t), so box N's language is L(X_start(N)).  Removing epsilon rules gives
// A+ (the non-empty words of A) with rules A+ -> B+ C+, A+ -> C+ (B nullable)
// and A+ -> B+ (C nullable); unit rules are closed once (U(A)).  Every
// binary split then gives both parts at least one edge, so the expansion of
// a length-l path recurses on shorter lengths only and always terminates.
// F(A, x, l) = vertices y with a length-l path x -> y derived from A+,
// memoised as bitsets, prunes every split.
// ---------------------------------------------------------------------------
struct cfpq_paths_s {
    uint32_t n = 0, W = 0, nQ = 0, nT = 0;
    std::shared_ptr<const HostCsr> csr;                             // successors per label (sorted)
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> bin;    // A+ -> B+ C+
    std::vector<std::vector<uint32_t>> unit;                        // U(A), A included
    std::vector<uint8_t> nullable;
    uint32_t S = 0, u = 0, v = 0, max_edges = 0, next_len = 0;
    std::unordered_map<uint64_t, std::vector<uint64_t>> memo;
    std::vector<std::vector<uint32_t>> batch;                       // paths of the current length
    size_t pos = 0;
    bool empty = false;

    uint64_t key(uint32_t A, uint32_t x, uint32_t l) const {
        return ((uint64_t)A * n + x) * (uint64_t)(max_edges + 1) + l;
    }
    bool has_edge(uint32_t x, uint32_t t, uint32_t y) const {
        const uint32_t *b = csr->out.data() + csr->off[(uint64_t)t * (n + 1) + x];
        const uint32_t *e = csr->out.data() + csr->off[(uint64_t)t * (n + 1) + x + 1];
        return std::binary_search(b, e, y);
    }
    static bool test(const std::vector<uint64_t> &s, uint32_t y) { return (s[y >> 6] >> (y & 63)) & 1ull; }

    const std::vector<uint64_t> &F(uint32_t A, uint32_t x, uint32_t l) {
        const uint64_t k = key(A, x, l);
        auto it = memo.find(k);
        if (it != memo.end()) return it->second;
        std::vector<uint64_t> s(W, 0);
        for (uint32_t B : unit[A]) {
            if (B >= nQ) {   // T_t
                if (l == 1) {
                    const uint32_t t = B - nQ;
                    const std::vector<uint32_t> &off = csr->off, &out = csr->out;
                    for (uint32_t e = off[(uint64_t)t * (n + 1) + x]; e < off[(uint64_t)t * (n + 1) + x + 1]; ++e)
                        s[out[e] >> 6] |= 1ull << (out[e] & 63);
                }
                continue;
            }
            for (const auto &cd : bin[B])
                for (uint32_t l1 = 1; l1 < l; ++l1) {
                    const std::vector<uint64_t> fc = F(cd.first, x, l1);   // copy: the memo grows below
                    for (uint32_t w = 0; w < W; ++w)
                        for (uint64_t m = fc[w]; m; m &= m - 1) {
                            const uint32_t z = w * 64 + (uint32_t)__builtin_ctzll(m);
                            const std::vector<uint64_t> &fd = F(cd.second, z, l - l1);
                            for (uint32_t i = 0; i < W; ++i) s[i] |= fd[i];
                        }
                }
        }
        return memo.emplace(k, std::move(s)).first->second;
    }

    // every derivation of a length-l path x -> y from A+; k runs with path
    // holding the path so far
    void gen(uint32_t A, uint32_t x, uint32_t y, uint32_t l, std::vector<uint32_t> &path,
             const std::function<void()> &k) {
        for (uint32_t B : unit[A]) {
            if (B >= nQ) {
                const uint32_t t = B - nQ;
                if (l == 1 && has_edge(x, t, y)) {
                    path.insert(path.end(), {x, t, y});
                    k();
                    path.resize(path.size() - 3);
                }
                continue;
            }
            for (const auto &cd : bin[B])
                for (uint32_t l1 = 1; l1 < l; ++l1) {
                    const std::vector<uint64_t> fc = F(cd.first, x, l1);
                    for (uint32_t w = 0; w < W; ++w)
                        for (uint64_t m = fc[w]; m; m &= m - 1) {
                            const uint32_t z = w * 64 + (uint32_t)__builtin_ctzll(m);
                            if (!test(F(cd.second, z, l - l1), y)) continue;
                            gen(cd.first, x, z, l1, path, [&] { gen(cd.second, z, y, l - l1, path, k); });
                        }
                }
        }
    }

    struct VecHash {
        size_t operator()(const std::vector<uint32_t> &p) const {
            uint64_t h = 1469598103934665603ull;
            for (uint32_t x : p) h = (h ^ x) * 1099511628211ull;
            return (size_t)h;
        }
    };

    cfpq_status fill(uint32_t l) {
        batch.clear();
        pos = 0;
        if (l == 0) {
            if (u == v && nullable[S]) batch.emplace_back();
            return CFPQ_OK;
        }
        if (!test(F(S, u, l), v)) return CFPQ_OK;
        std::unordered_set<std::vector<uint32_t>, VecHash> seen;
        std::vector<uint32_t> path;
        uint64_t words = 0;
        bool over = false;
        gen(S, u, v, l, path, [&] {
            if (over) return;
            if (seen.insert(path).second) {
                words += path.size();
                if (words > (1ull << 24) * 3) over = true;
                else batch.push_back(path);
            }
        });
        if (over) return fail(CFPQ_ERR_LIMIT, "paths of one length exceed 2^24 edges");
        return CFPQ_OK;
    }
};

extern "C" cfpq_status cfpq_paths_open(cfpq_result r, uint32_t box, uint32_t u, uint32_t v, uint32_t max_edges,
                                       cfpq_paths *out) {
    if (!out) return fail(CFPQ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    cfpq_status st = check_box(r, box);
    if (st != CFPQ_OK) return st;
    if (u >= r->n || v >= r->n) return fail(CFPQ_ERR_INVALID, "vertex out of range");
    if (max_edges > 4096) return fail(CFPQ_ERR_INVALID, "max_edges above 4096");
    try {
        std::unique_ptr<cfpq_paths_s> it(new cfpq_paths_s);
        const cfpq_rsm_s &R = r->rsm;
        it->n = r->n;
        it->W = (r->n + 63) / 64;
        it->nQ = R.n_states;
        it->nT = R.n_terms;
        it->u = u;
        it->v = v;
        it->max_edges = max_edges;
        it->csr = r->hcsr;   // lists sorted at graph creation
        const uint32_t nA = it->nQ + it->nT;
        // nullable X_q: least fixpoint
        it->nullable.assign(nA, 0);
        for (uint32_t q = 0; q < it->nQ; ++q) it->nullable[q] = R.is_final[q] != 0;
        auto sym_nt = [&](uint32_t sym) { return sym < R.n_terms ? it->nQ + sym : R.box_start[sym - R.n_terms]; };
        for (bool grew = true; grew;) {
            grew = false;
            for (size_t t = 0; t < R.t_src.size(); ++t) {
                const uint32_t q = R.t_src[t];
                if (!it->nullable[q] && it->nullable[sym_nt(R.t_sym[t])] && it->nullable[R.t_dst[t]]) {
                    it->nullable[q] = 1;
                    grew = true;
                }
            }
        }
        // epsilon-free rules
        it->bin.assign(nA, {});
        std::vector<std::vector<uint32_t>> unit_edges(nA);
        for (size_t t = 0; t < R.t_src.size(); ++t) {
            const uint32_t A = R.t_src[t], B = sym_nt(R.t_sym[t]), C = R.t_dst[t];
            it->bin[A].push_back({B, C});
            if (it->nullable[B]) unit_edges[A].push_back(C);
            if (it->nullable[C]) unit_edges[A].push_back(B);
        }
        it->unit.assign(nA, {});
        for (uint32_t A = 0; A < nA; ++A) {
            std::vector<uint8_t> in(nA, 0);
            std::vector<uint32_t> q{A};
            in[A] = 1;
            for (size_t h = 0; h < q.size(); ++h)
                for (uint32_t B : unit_edges[q[h]])
                    if (!in[B]) {
                        in[B] = 1;
                        q.push_back(B);
                    }
            it->unit[A] = q;
        }
        it->S = R.box_start[box];
        // the pair must be in the relation as returned (masks included)
        uint64_t word = 0;
        HIP_TRY(hipMemcpy(&word, r->NT.as<uint64_t>() + ((uint64_t)box * r->n + v) * r->P + (u >> 6), 8,
                          hipMemcpyDeviceToHost));
        it->empty = !((word >> (u & 63)) & 1ull);
        *out = it.release();
    } catch (const std::bad_alloc &) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    return CFPQ_OK;
}

extern "C" cfpq_status cfpq_paths_next(cfpq_paths it, uint32_t *edges, uint64_t cap_edges, uint64_t *n_edges) {
    if (!it || !n_edges) return fail(CFPQ_ERR_INVALID, "NULL argument");
    try {
        while (!it->empty && it->pos >= it->batch.size()) {
            if (it->next_len > it->max_edges) {
                it->empty = true;
                break;
            }
            cfpq_status st = it->fill(it->next_len++);
            if (st != CFPQ_OK) return st;
        }
        if (it->empty) return fail(CFPQ_ERR_NOT_FOUND, "no path left");
        const std::vector<uint32_t> &p = it->batch[it->pos];
        *n_edges = p.size() / 3;
        if (cap_edges < p.size() / 3) return fail(CFPQ_ERR_BUFFER, "edge buffer too small");
        if (!p.empty()) {
            if (!edges) return fail(CFPQ_ERR_INVALID, "edges is NULL");
            std::memcpy(edges, p.data(), p.size() * 4);
        }
        ++it->pos;
    } catch (const std::bad_alloc &) {
        return fail(CFPQ_ERR_OOM, "host allocation failed");
    }
    return CFPQ_OK;
}

extern "C" void cfpq_paths_close(cfpq_paths it) { delete it; }

extern "C" const char *cfpq_last_error(void) { return g_err.c_str(); }

extern "C" const char *cfpq_version(void) { return "cfpq-gfx950 0.8"; }
