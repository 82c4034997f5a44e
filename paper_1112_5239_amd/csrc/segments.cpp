// segments.cpp -- batched uneven streams and request batches (plain variant).
//
// A stream's run of L outputs is cut into chunks ("segments") so that long
// runs use many lanes.  Segment k of a run starts at position P_k (P_0 = 0,
// P_k = h + k*chunk, h = outputs needed to reach a 16-byte-aligned address),
// from the state A'^{P_k} v obtained with a jump polynomial X^{P_k} mod q (see
// gf2.cpp).  The lane that owns the run's final segment writes the end state
// to state_next; a small commit kernel copies those states back after the
// segment kernel, so no lane reads a state another lane of the same launch is
// rewriting.
//
// Batched uneven streams run as one hipGraph (queue reset, persistent segment
// kernel, commit) that is built once per (lengths, offsets, out, tuning) and
// replayed.  Request batches are built per call and launched directly.
#include <algorithm>
#include <cstring>
#include <memory>
#include <unordered_map>
#include <vector>

#include "host.h"
#include "tune.h"

namespace cprng_impl {

struct RaggedPlan {
    std::vector<uint64_t> lengths, offsets;
    uint32_t *out = nullptr;
    uint32_t chunk = 0, unroll = 0, waves = 0, block = 0;
    SegDesc *d_segs = nullptr;
    uint32_t nseg = 0;
    uint32_t *d_polys = nullptr;
    uint32_t npolys = 0;
    uint32_t *d_ids = nullptr;
    uint32_t nids = 0;
    uint32_t grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

namespace {

uint64_t g_use_clock = 0;

void free_plan(RaggedPlan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_segs) (void)hipFree(p->d_segs);
    if (p->d_polys) (void)hipFree(p->d_polys);
    if (p->d_ids) (void)hipFree(p->d_ids);
    delete p;
}

// Table of X^(h + k*chunk) mod q for h in 0..3, k in 0..kcap-1 (index
// h*kcap + k); entry 0 is X^0 = 1, the "no jump" polynomial.
void build_table(uint32_t chunk, uint32_t kcap, std::vector<uint32_t> &tab)
{
    tab.assign((size_t)4 * kcap * 5, 0u);
    const JPoly step = jump_xpow(chunk);
    for (uint32_t h = 0; h < 4; ++h) {
        JPoly p = jump_xpow(h);
        for (uint32_t k = 0; k < kcap; ++k) {
            jump_pack(p, &tab[((size_t)h * kcap + k) * 5]);
            p = jump_mul(p, step);
        }
    }
}

uint32_t head_of(uint64_t addr)
{
    return (uint32_t)((4u - (uint32_t)((addr / 4u) % 4u)) % 4u);
}

// Cut one run into segments.  `skip` > 0 (not the first run of the stream in
// this call) takes its jump polynomials from `extra`.
struct Cutter {
    uint32_t chunk = 0, kcap = 0;
    std::vector<SegDesc> segs;
    std::vector<uint32_t> extra;       // packed polynomials, index n_table + i
    uint32_t n_table = 0;
    bool need_bigger_table = false;

    void run(uint32_t stream, uint64_t addr, uint64_t len, uint64_t skip)
    {
        const uint32_t h = head_of(addr);
        uint64_t pos = 0;
        uint32_t k = 0;
        while (pos < len) {
            const uint64_t cap = (k == 0) ? (uint64_t)h + chunk : chunk;
            const uint64_t sl = std::min<uint64_t>(cap, len - pos);
            SegDesc d;
            std::memset(&d, 0, sizeof d);
            d.out = addr + 4u * pos;
            d.stream = stream;
            d.len = (uint32_t)sl;
            d.head = (k == 0) ? h : 0u;
            const uint64_t dist = skip + pos;
            if (skip == 0) {
                if (k >= kcap) need_bigger_table = true;
                d.poly = (k == 0) ? 0u : h * kcap + k;
            } else {
                uint32_t w[5];
                jump_pack(jump_xpow(dist), w);
                d.poly = n_table + (uint32_t)(extra.size() / 5);
                extra.insert(extra.end(), w, w + 5);
            }
            segs.push_back(d);
            pos += sl;
            ++k;
        }
    }
};

int ensure_common(cprng_t *h)
{
    std::string why;
    if (!jump_init(&why)) return set_error(CPRNG_E_UNSUPPORTED, "jump polynomials: " + why);
    if (!h->d_state_next) {
        if (hipMalloc(&h->d_state_next, (size_t)5 * h->ns * sizeof(uint32_t)) != hipSuccess)
            return set_error(CPRNG_E_NOMEM, "hipMalloc state_next");
    }
    if (!h->d_counter) {
        if (hipMalloc(&h->d_counter, 64) != hipSuccess) return set_error(CPRNG_E_NOMEM, "hipMalloc counter");
        if (hipMemset(h->d_counter, 0, 64) != hipSuccess) return set_error(CPRNG_E_HIP, "hipMemset counter");
    }
    return CPRNG_OK;
}

uint32_t kcap_for(uint64_t max_len, uint32_t chunk)
{
    const uint64_t k = max_len / chunk + 2;
    uint32_t cap = 64;
    while (cap < k) cap *= 2;
    return cap;
}

struct SegCfg {
    uint32_t chunk, unroll, waves, block;
};

SegCfg resolve_seg_cfg(const cprng_t *h, uint64_t total, uint64_t max_len)
{
    SegCfg c{8192, 32, 8, 256};
    TuneEntry e;
    if (tune_cache_lookup_key(tune_key_ragged(h, total, max_len), &e)) {
        if (e.chunk) c.chunk = e.chunk;
        if (e.unroll) c.unroll = e.unroll;
        if (e.waves) c.waves = e.waves;
        if (e.block) c.block = e.block;
    }
    if (h->tuning.chunk) c.chunk = h->tuning.chunk;
    if (h->tuning.waves_per_cu) c.waves = h->tuning.waves_per_cu;
    if (h->tuning.unroll) c.unroll = h->tuning.unroll;
    if (h->tuning.block) c.block = h->tuning.block;
    return c;
}

uint32_t persistent_grid(const cprng_t *h, const SegCfg &c, uint32_t nseg)
{
    const uint32_t waves_per_block = c.block / 64;
    uint64_t grid = (uint64_t)h->n_cu * c.waves / waves_per_block;
    const uint64_t needed = ((uint64_t)nseg + 63) / 64;          // one grab per wave
    const uint64_t needed_blocks = (needed + waves_per_block - 1) / waves_per_block;
    if (grid > needed_blocks) grid = needed_blocks;
    return (uint32_t)(grid ? grid : 1);
}

template <typename T>
int upload(T **dptr, const std::vector<T> &v)
{
    if (v.empty()) return CPRNG_OK;
    if (hipMalloc(dptr, v.size() * sizeof(T)) != hipSuccess) return set_error(CPRNG_E_NOMEM, "hipMalloc plan buffer");
    if (hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return set_error(CPRNG_E_HIP, "hipMemcpy plan buffer");
    return CPRNG_OK;
}

int build_plan(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets,
               const SegCfg &c, RaggedPlan **res)
{
    std::unique_ptr<RaggedPlan, void (*)(RaggedPlan *)> p(new RaggedPlan(), free_plan);
    p->lengths.assign(lengths, lengths + h->ns);
    p->offsets.resize(h->ns);
    uint64_t acc = 0, max_len = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        p->offsets[s] = offsets ? offsets[s] : acc;
        acc += lengths[s];
        max_len = std::max(max_len, lengths[s]);
    }
    p->out = out;
    p->chunk = c.chunk;
    p->unroll = c.unroll;
    p->waves = c.waves;
    p->block = c.block;

    Cutter cut;
    cut.chunk = c.chunk;
    cut.kcap = kcap_for(max_len, c.chunk);
    cut.n_table = 4 * cut.kcap;
    std::vector<uint32_t> ids;
    for (uint32_t s = 0; s < h->ns; ++s) {
        const uint64_t L = p->lengths[s];
        if (L == 0) continue;
        const size_t first = cut.segs.size();
        cut.run(s, (uint64_t)(uintptr_t)out + 4u * p->offsets[s], L, 0);
        cut.segs.back().last = 1;
        (void)first;
        ids.push_back(s);
    }
    if (cut.need_bigger_table) return set_error(CPRNG_E_INVAL, "internal: jump table too small");
    // Longest segments first so that short tails fill the end of the queue.
    std::stable_sort(cut.segs.begin(), cut.segs.end(),
                     [](const SegDesc &a, const SegDesc &b) { return a.len > b.len; });
    std::vector<uint32_t> tab;
    build_table(c.chunk, cut.kcap, tab);
    p->nseg = (uint32_t)cut.segs.size();
    p->nids = (uint32_t)ids.size();
    p->npolys = cut.n_table;
    int rc = upload(&p->d_segs, cut.segs);
    if (!rc) rc = upload(&p->d_polys, tab);
    if (!rc) rc = upload(&p->d_ids, ids);
    if (rc) return rc;
    p->grid = persistent_grid(h, c, p->nseg);

    SegArgs a;
    std::memset(&a, 0, sizeof a);
    a.segs = p->d_segs;
    a.nseg = p->nseg;
    a.ns = h->ns;
    a.polys = p->d_polys;
    a.polys_extra = nullptr;
    a.n_table = p->npolys;
    a.state = h->d_state;
    a.state_next = h->d_state_next;
    a.counter = h->d_counter;
    a.unroll = c.unroll;

    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return set_error(CPRNG_E_HIP, "hipStreamCreate (capture)");
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_zero_u32(h->d_counter, 1, cs);
    if (e == hipSuccess && p->nseg) e = launch_segments(a, p->grid, c.block, 0, cs);
    if (e == hipSuccess) e = launch_commit(h->d_state, h->d_state_next, p->d_ids, p->nids, h->ns, cs);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_error(e, "capture of the batched kernel");
    }
    if (e2 != hipSuccess) return hip_error(e2, "hipStreamEndCapture");
    p->graph = graph;
    e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_error(e, "hipGraphInstantiate");
    *res = p.release();
    return CPRNG_OK;
}

RaggedPlan *find_plan(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets,
                      const SegCfg &c)
{
    for (RaggedPlan *p : h->plans) {
        if (p->out != out || p->chunk != c.chunk || p->unroll != c.unroll || p->waves != c.waves ||
            p->block != c.block)
            continue;
        if (std::memcmp(p->lengths.data(), lengths, sizeof(uint64_t) * h->ns) != 0) continue;
        bool same = true;
        uint64_t acc = 0;
        for (uint32_t s = 0; s < h->ns && same; ++s) {
            same = p->offsets[s] == (offsets ? offsets[s] : acc);
            acc += lengths[s];
        }
        if (same) return p;
    }
    return nullptr;
}

int check_ragged_args(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets,
                      uint64_t *total, uint64_t *max_len)
{
    if (!h || !out || !lengths) return set_error(CPRNG_E_INVAL, "NULL argument");
    if (h->variant != CPRNG_V0_PLAIN)
        return set_error(CPRNG_E_UNSUPPORTED, "batched uneven streams need the V0 variant (GF(2)-linear jump-ahead)");
    if (h->flags & CPRNG_F_INTERLEAVED) return set_error(CPRNG_E_UNSUPPORTED, "interleaved layout has no ragged form");
    if ((uintptr_t)out % 4u) return set_error(CPRNG_E_INVAL, "out must be 4-byte aligned");
    uint64_t acc = 0, mx = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        if (lengths[s] > (1ull << 40)) return set_error(CPRNG_E_INVAL, "length too large");
        acc += lengths[s];
        mx = std::max(mx, lengths[s]);
    }
    if (offsets) {
        // Runs must not overlap: sort by offset and check.
        std::vector<std::pair<uint64_t, uint64_t>> r;
        for (uint32_t s = 0; s < h->ns; ++s)
            if (lengths[s]) r.emplace_back(offsets[s], lengths[s]);
        std::sort(r.begin(), r.end());
        for (size_t i = 1; i < r.size(); ++i)
            if (r[i - 1].first + r[i - 1].second > r[i].first)
                return set_error(CPRNG_E_INVAL, "output runs overlap");
    }
    *total = acc;
    *max_len = mx;
    return CPRNG_OK;
}

}  // namespace

void destroy_plans(cprng_t *h)
{
    for (RaggedPlan *p : h->plans) free_plan(p);
    h->plans.clear();
}

int ragged_with(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets,
                hipStream_t st, const SegCfg &c)
{
    RaggedPlan *p = find_plan(h, out, lengths, offsets, c);
    if (!p) {
        int rc = build_plan(h, out, lengths, offsets, c, &p);
        if (rc) return rc;
        if (h->plans.size() >= 8) {
            auto it = std::min_element(h->plans.begin(), h->plans.end(),
                                       [](RaggedPlan *a, RaggedPlan *b) { return a->last_use < b->last_use; });
            free_plan(*it);
            h->plans.erase(it);
        }
        h->plans.push_back(p);
    }
    p->last_use = ++g_use_clock;
    if (h->timing && hipEventRecord(h->ev0, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
    hipError_t e = hipGraphLaunch(p->exec, st);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    if (h->timing) {
        if (hipEventRecord(h->ev1, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
        h->ev_pending = true;
    }
    return CPRNG_OK;
}

}  // namespace cprng_impl

using namespace cprng_impl;

namespace {
struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace

extern "C" int cprng_generate_ragged(cprng_t *h, uint32_t *out, const uint64_t *lengths,
                                     const uint64_t *offsets, cprng_stream_t stream)
{
    uint64_t total = 0, max_len = 0;
    int rc = check_ragged_args(h, out, lengths, offsets, &total, &max_len);
    if (rc) return rc;
    DevGuard g(h->device);
    rc = ensure_common(h);
    if (rc) return rc;
    const SegCfg c = resolve_seg_cfg(h, total, max_len);
    return ragged_with(h, out, lengths, offsets, (hipStream_t)stream, c);
}

extern "C" int cprng_autotune_ragged(cprng_t *h, uint32_t *out, const uint64_t *lengths,
                                     const uint64_t *offsets, cprng_stream_t stream)
{
    uint64_t total = 0, max_len = 0;
    int rc = check_ragged_args(h, out, lengths, offsets, &total, &max_len);
    if (rc) return rc;
    DevGuard g(h->device);
    rc = ensure_common(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(CPRNG_E_HIP, "hipEventCreate");
    const uint32_t chunks[] = {2048, 4096, 8192, 16384, 32768};
    const uint32_t waves[] = {4, 8, 16};
    const uint32_t unrolls[] = {16, 32};
    float best = 1e30f;
    SegCfg best_c{8192, 32, 8, 256};
    const bool saved_timing = h->timing;
    h->timing = false;
    for (uint32_t ch : chunks)
        for (uint32_t w : waves)
            for (uint32_t u : unrolls) {
                SegCfg c{ch, u, w, 256};
                std::vector<float> t;
                for (int r = 0; r < 4 && rc == CPRNG_OK; ++r) {
                    if (hipEventRecord(e0, st) != hipSuccess) rc = set_error(CPRNG_E_HIP, "hipEventRecord");
                    if (!rc) rc = ragged_with(h, out, lengths, offsets, st, c);
                    if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = set_error(CPRNG_E_HIP, "hipEventRecord");
                    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = set_error(CPRNG_E_HIP, "hipEventSynchronize");
                    float ms = 0.f;
                    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = set_error(CPRNG_E_HIP, "elapsed");
                    if (r > 0) t.push_back(ms);
                }
                // Drop this candidate's graph again; only the winner is kept.
                if (RaggedPlan *p = find_plan(h, out, lengths, offsets, c)) {
                    h->plans.erase(std::find(h->plans.begin(), h->plans.end(), p));
                    free_plan(p);
                }
                if (rc) break;
                std::sort(t.begin(), t.end());
                if (t[t.size() / 2] < best) {
                    best = t[t.size() / 2];
                    best_c = c;
                }
            }
    h->timing = saved_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    TuneEntry e;
    e.block = best_c.block;
    e.unroll = best_c.unroll;
    e.chunk = best_c.chunk;
    e.waves = best_c.waves;
    tune_cache_store(tune_key_ragged(h, total, max_len), e);
    return CPRNG_OK;
}

// ---------------------------------------------------------------------------
// Request batches.
// ---------------------------------------------------------------------------
namespace {

template <typename T>
int ensure_dev(T **p, size_t *cap, size_t need)
{
    if (need <= *cap) return CPRNG_OK;
    size_t n = std::max<size_t>(need, *cap * 2);
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, n * sizeof(T)) != hipSuccess) return set_error(CPRNG_E_NOMEM, "hipMalloc request buffer");
    *cap = n;
    return CPRNG_OK;
}

// Per-handle X^(h + k*chunk) table for requests, grown on demand.
int request_table(cprng_t *h, uint32_t chunk, uint32_t kcap_needed, const uint32_t **dptr, uint32_t *kcap)
{
    auto it = h->req_poly_tables.find(chunk);
    uint32_t have = (it == h->req_poly_tables.end()) ? 0u : (uint32_t)(it->second.size() / 20);
    if (have >= kcap_needed) {
        *dptr = h->d_req_poly_tables[chunk];
        *kcap = have;
        return CPRNG_OK;
    }
    uint32_t cap = 64;
    while (cap < kcap_needed) cap *= 2;
    std::vector<uint32_t> tab;
    build_table(chunk, cap, tab);
    uint32_t *d = nullptr;
    // The old table may still be read by queued work; wait before freeing it.
    if (hipDeviceSynchronize() != hipSuccess) return set_error(CPRNG_E_HIP, "hipDeviceSynchronize");
    if (hipMalloc(&d, tab.size() * sizeof(uint32_t)) != hipSuccess) return set_error(CPRNG_E_NOMEM, "hipMalloc table");
    if (hipMemcpy(d, tab.data(), tab.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return set_error(CPRNG_E_HIP, "hipMemcpy table");
    }
    auto dit = h->d_req_poly_tables.find(chunk);
    if (dit != h->d_req_poly_tables.end()) (void)hipFree(dit->second);
    h->d_req_poly_tables[chunk] = d;
    h->req_poly_tables[chunk] = std::move(tab);
    *dptr = d;
    *kcap = cap;
    return CPRNG_OK;
}

}  // namespace

extern "C" int cprng_generate_requests(cprng_t *h, const cprng_request_t *reqs, uint32_t count,
                                       cprng_stream_t stream)
{
    if (!h || (!reqs && count)) return set_error(CPRNG_E_INVAL, "NULL argument");
    if (h->variant != CPRNG_V0_PLAIN)
        return set_error(CPRNG_E_UNSUPPORTED, "requests need the V0 variant (GF(2)-linear jump-ahead)");
    if (count == 0) return CPRNG_OK;
    uint64_t total = 0, max_len = 0;
    for (uint32_t r = 0; r < count; ++r) {
        if (reqs[r].stream >= h->ns) return set_error(CPRNG_E_INVAL, "request stream id out of range");
        if (reqs[r].length && (!reqs[r].out || (uintptr_t)reqs[r].out % 4u))
            return set_error(CPRNG_E_INVAL, "request out must be non-NULL and 4-byte aligned");
        if (reqs[r].length > (1ull << 40)) return set_error(CPRNG_E_INVAL, "request too large");
        total += reqs[r].length;
        max_len = std::max(max_len, reqs[r].length);
    }
    DevGuard g(h->device);
    int rc = ensure_common(h);
    if (rc) return rc;
    SegCfg c = resolve_seg_cfg(h, total, max_len);
    // Keep enough segments to fill the GPU when the batch is small.
    if (!h->tuning.chunk) {
        const uint64_t lanes_wanted = (uint64_t)h->n_cu * 4 * 64 * 2;
        while (c.chunk > 1024 && total / c.chunk < lanes_wanted) c.chunk /= 2;
    }
    const uint32_t *d_tab = nullptr;
    uint32_t kcap = 0;
    rc = request_table(h, c.chunk, kcap_for(max_len, c.chunk), &d_tab, &kcap);
    if (rc) return rc;

    Cutter cut;
    cut.chunk = c.chunk;
    cut.kcap = kcap;
    cut.n_table = 4 * kcap;
    std::unordered_map<uint32_t, uint64_t> done;   // outputs already assigned per stream
    std::unordered_map<uint32_t, size_t> last_seg; // index of the stream's last segment
    for (uint32_t r = 0; r < count; ++r) {
        const cprng_request_t &q = reqs[r];
        if (q.length == 0) continue;
        uint64_t &skip = done[q.stream];
        cut.run(q.stream, (uint64_t)(uintptr_t)q.out, q.length, skip);
        skip += q.length;
        last_seg[q.stream] = cut.segs.size() - 1;
    }
    if (cut.need_bigger_table) return set_error(CPRNG_E_INVAL, "internal: jump table too small");
    std::vector<uint32_t> ids;
    ids.reserve(last_seg.size());
    for (auto &kv : last_seg) {
        cut.segs[kv.second].last = 1;
        ids.push_back(kv.first);
    }
    if (cut.segs.empty()) return CPRNG_OK;
    std::vector<size_t> order(cut.segs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return cut.segs[a].len > cut.segs[b].len; });
    std::vector<SegDesc> sorted(cut.segs.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = cut.segs[order[i]];

    hipStream_t st = (hipStream_t)stream;
    rc = ensure_dev(&h->d_req_segs, &h->req_segs_cap, sorted.size());
    if (!rc) rc = ensure_dev(&h->d_req_polys, &h->req_polys_cap, std::max<size_t>(cut.extra.size(), 5));
    if (!rc) rc = ensure_dev(&h->d_req_ids, &h->req_ids_cap, ids.size());
    if (rc) return rc;
    // Stage through pinned memory; wait until the previous call's upload has
    // left the staging buffer before overwriting it.
    const size_t bytes = sorted.size() * sizeof(SegDesc) + cut.extra.size() * 4 + ids.size() * 4 + 64;
    if (!h->ev_stage && hipEventCreateWithFlags(&h->ev_stage, hipEventDisableTiming) != hipSuccess)
        return set_error(CPRNG_E_HIP, "hipEventCreate");
    if (hipEventSynchronize(h->ev_stage) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventSynchronize");
    if (bytes > h->h_stage_cap) {
        if (h->h_stage) (void)hipHostFree(h->h_stage);
        h->h_stage = nullptr;
        h->h_stage_cap = 0;
        if (hipHostMalloc(&h->h_stage, bytes * 2, hipHostMallocDefault) != hipSuccess)
            return set_error(CPRNG_E_NOMEM, "hipHostMalloc staging");
        h->h_stage_cap = bytes * 2;
    }
    char *hs = (char *)h->h_stage;
    const size_t o_segs = 0, o_polys = sorted.size() * sizeof(SegDesc),
                 o_ids = o_polys + cut.extra.size() * 4;
    std::memcpy(hs + o_segs, sorted.data(), sorted.size() * sizeof(SegDesc));
    if (!cut.extra.empty()) std::memcpy(hs + o_polys, cut.extra.data(), cut.extra.size() * 4);
    std::memcpy(hs + o_ids, ids.data(), ids.size() * 4);
    hipError_t e = hipMemcpyAsync(h->d_req_segs, hs + o_segs, sorted.size() * sizeof(SegDesc), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !cut.extra.empty())
        e = hipMemcpyAsync(h->d_req_polys, hs + o_polys, cut.extra.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->d_req_ids, hs + o_ids, ids.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(h->ev_stage, st);
    if (e != hipSuccess) return hip_error(e, "request upload");

    SegArgs a;
    std::memset(&a, 0, sizeof a);
    a.segs = h->d_req_segs;
    a.nseg = (uint32_t)sorted.size();
    a.ns = h->ns;
    a.polys = d_tab;
    a.polys_extra = h->d_req_polys;
    a.n_table = cut.n_table;
    a.state = h->d_state;
    a.state_next = h->d_state_next;
    a.counter = h->d_counter;
    a.unroll = c.unroll;
    if (h->timing && hipEventRecord(h->ev0, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
    e = launch_zero_u32(h->d_counter, 1, st);
    if (e == hipSuccess) e = launch_segments(a, persistent_grid(h, c, a.nseg), c.block, 0, st);
    if (e == hipSuccess) e = launch_commit(h->d_state, h->d_state_next, h->d_req_ids, (uint32_t)ids.size(), h->ns, st);
    if (e != hipSuccess) return hip_error(e, "request kernels");
    if (h->timing) {
        if (hipEventRecord(h->ev1, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
        h->ev_pending = true;
    }
    return CPRNG_OK;
}
