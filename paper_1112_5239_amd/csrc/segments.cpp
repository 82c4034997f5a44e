// segments.cpp -- batched uneven streams and request batches (plain variant).
//
// A run of L outputs of one stream is cut into chunks ("segments") so that
// long runs use many lanes (see RunDesc in internal.h).  Segment k >= 1 of a
// run starts at position h + k*chunk from the state A'^(h + k*chunk) v, whose
// jump polynomial X^(h + k*chunk) mod q (gf2.cpp) comes from a table indexed
// by (h, k); the kernel decodes its segment from the run descriptors, so the
// host work per launch is proportional to the number of runs.  The lane that
// owns a run's final segment writes the stream's end state to state_next; a
// commit kernel copies those states back after the segment kernel, so no lane
// reads a state that another lane of the same launch rewrites.
//
// Batched uneven streams run as one hipGraph (queue-reset kernel, persistent
// segment kernel, commit kernel) built once per (lengths, offsets, out,
// tuning) and replayed.  Request batches are built per call; requests of one
// stream are served in order by consecutive launches on the call's stream,
// each launch holding at most one run per stream.
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
    uint32_t chunk = 0, unroll = 0, waves = 0, block = 0, store = 0;
    RunDesc *d_runs = nullptr;
    uint32_t nrun = 0, nseg = 0, kcap = 0;
    uint32_t *d_polys = nullptr;
    uint32_t *d_ids = nullptr;
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
    // A replay of this plan may still be queued or running: let the device
    // finish before the graph and its tables go.
    if (p->exec) (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_runs) (void)hipFree(p->d_runs);
    if (p->d_polys) (void)hipFree(p->d_polys);
    if (p->d_ids) (void)hipFree(p->d_ids);
    delete p;
}

// Outputs before the first 256-byte boundary of a run: the run's segment 0
// stores them one by one, so every later segment (a multiple of 64 outputs)
// starts on a 256-byte boundary and the tiles write whole lines.
uint32_t head_of(uint64_t addr) { return (uint32_t)((64u - (uint32_t)((addr / 4u) % 64u)) % 64u); }

uint64_t segments_of(uint64_t len, uint32_t head, uint32_t chunk)
{
    const uint64_t seg0 = (uint64_t)head + chunk;
    return len <= seg0 ? 1 : 1 + (len - seg0 + chunk - 1) / chunk;
}

uint32_t kcap_for(uint64_t max_segments)
{
    uint32_t cap = 64;
    while (cap < max_segments + 1) cap *= 2;
    return cap;
}

// Runs of one launch, with their segment numbering.
struct RunList {
    std::vector<RunDesc> runs;
    uint64_t nseg = 0, max_seg = 0;
    // Returns false if the launch would exceed 2^31 segments.
    bool add(uint32_t stream, uint64_t addr, uint64_t len, uint32_t chunk, uint32_t last)
    {
        RunDesc r;
        std::memset(&r, 0, sizeof r);
        r.out = addr;
        r.len = len;
        r.stream = stream;
        r.head = head_of(addr);
        r.first_seg = (uint32_t)nseg;
        r.last = last;
        const uint64_t k = segments_of(len, r.head, chunk);
        nseg += k;
        max_seg = std::max(max_seg, k);
        runs.push_back(r);
        return nseg < (1ull << 31);
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

struct SegCfg {
    uint32_t chunk, unroll, waves, block, store;
};

// Store codes of the chunk kernels: ST_LDS / ST_LDS_NT persistent waves
// taking grabs from the per-XCD queues (waves = persistent waves per CU);
// ST_PIPE / ST_PIPE_NT one workgroup per grab, banded over the XCDs and
// scheduled by the hardware (waves = residency cap through LDS, 0 = none);
// ST_DIRECT per-lane stores, persistent.
bool seg_persistent(const SegCfg &c) { return c.store != ST_PIPE && c.store != ST_PIPE_NT; }

uint32_t seg_kernel_store(const SegCfg &c)
{
    if (c.store == ST_PIPE) return ST_LDS;
    if (c.store == ST_PIPE_NT) return ST_LDS_NT;
    return c.store;
}

// Tiled stores (one wave per workgroup) take K in {32, 64, 128, 256};
// per-lane stores take K in {8, 16, 32} and any block size.
void normalize(SegCfg &c)
{
    if (c.store == ST_LDS || c.store == ST_LDS_NT || c.store == ST_PIPE || c.store == ST_PIPE_NT) {
        c.block = 64;
        if (c.unroll < 32) c.unroll = 32;
        if (c.unroll > 256) c.unroll = 256;
    } else {
        c.store = ST_DIRECT;
        if (c.unroll > 32) c.unroll = 32;
        if (c.unroll < 8) c.unroll = 8;
    }
    if (c.waves == 0 && seg_persistent(c)) c.waves = 4;
}

// Default measured on MI355X for 4,096 streams of 1e3..1e7 outputs:
// LDS-tiled non-temporal stores of K = 128 outputs per row and round,
// 2048-output chunks (a wave's 64 chunks span 512 KiB of the output),
// three persistent waves per CU.  With runs aligned to 256 bytes every
// round writes whole lines; then 3 waves per CU keep enough SIMDs busy
// without widening the set of rows written at once too far.
constexpr SegCfg kDefaultSeg{2048, 128, 3, 64, ST_LDS_NT};

SegCfg resolve_seg_cfg(const cprng_t *h, uint64_t total, uint64_t max_len)
{
    SegCfg c = kDefaultSeg;
    TuneEntry e;
    if (tune_cache_lookup_key(tune_key_ragged(h, total, max_len), &e)) {
        if (e.chunk) c.chunk = e.chunk;
        if (e.unroll) c.unroll = e.unroll;
        if (e.waves) c.waves = e.waves;
        if (e.block) c.block = e.block;
        if (e.store) c.store = e.store;
    }
    if (h->tuning.chunk) c.chunk = h->tuning.chunk;
    if (h->tuning.waves_per_cu) c.waves = h->tuning.waves_per_cu;
    if (h->tuning.unroll) c.unroll = h->tuning.unroll;
    if (h->tuning.block) c.block = h->tuning.block;
    if (h->tuning.store) c.store = h->tuning.store == ST_DIRECT_NT ? (uint32_t)ST_DIRECT : h->tuning.store;
    normalize(c);
    return c;
}

uint32_t persistent_grid(const cprng_t *h, const SegCfg &c, uint64_t nseg)
{
    const uint32_t waves_per_block = c.block / 64;
    if (!seg_persistent(c)) {                          // one grab of 64 segments per wave
        const uint64_t grabs = (nseg + 63) / 64;
        const uint64_t blocks = (grabs + waves_per_block - 1) / waves_per_block;
        return (uint32_t)(blocks ? blocks : 1);
    }
    uint64_t grid = (uint64_t)h->n_cu * c.waves / waves_per_block;
    const uint64_t needed = (nseg + 63) / 64;          // one grab per wave
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

SegArgs seg_args(const cprng_t *h, const SegCfg &c, const RunDesc *runs, uint32_t nrun, uint64_t nseg,
                 uint32_t kcap, const uint32_t *polys, uint32_t *counter)
{
    SegArgs a;
    std::memset(&a, 0, sizeof a);
    a.runs = runs;
    a.nrun = nrun;
    a.nseg = (uint32_t)nseg;
    a.chunk = c.chunk;
    a.kcap = kcap;
    a.polys = polys;
    a.ns = h->ns;
    a.state = h->d_state;
    a.state_next = h->d_state_next;
    a.counter = counter;
    a.unroll = c.unroll;
    a.persistent = seg_persistent(c) ? 1u : 0u;
    return a;
}

uint32_t seg_lds_min(const SegCfg &c) { return seg_persistent(c) ? 0u : lds_for_waves(c.block, c.waves); }

int build_plan(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets,
               const SegCfg &c, RaggedPlan **res)
{
    std::unique_ptr<RaggedPlan, void (*)(RaggedPlan *)> p(new RaggedPlan(), free_plan);
    p->lengths.assign(lengths, lengths + h->ns);
    p->offsets.resize(h->ns);
    uint64_t acc = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        p->offsets[s] = offsets ? offsets[s] : acc;
        acc += lengths[s];
    }
    p->out = out;
    p->chunk = c.chunk;
    p->unroll = c.unroll;
    p->waves = c.waves;
    p->block = c.block;
    p->store = c.store;

    // Longest runs first, so that the queue ends with short segments.
    std::vector<uint32_t> order;
    for (uint32_t s = 0; s < h->ns; ++s)
        if (lengths[s]) order.push_back(s);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return lengths[a] > lengths[b]; });
    RunList rl;
    std::vector<uint32_t> ids;
    for (uint32_t s : order) {
        if (!rl.add(s, (uint64_t)(uintptr_t)out + 4u * p->offsets[s], lengths[s], c.chunk, 1))
            return set_error(CPRNG_E_INVAL, "too many segments (raise the chunk length)");
        ids.push_back(s);
    }
    p->nrun = (uint32_t)rl.runs.size();
    p->nseg = (uint32_t)rl.nseg;
    p->kcap = kcap_for(rl.max_seg);
    std::vector<uint32_t> tab;
    jump_table(c.chunk, p->kcap, tab);
    int rc = upload(&p->d_runs, rl.runs);
    if (!rc) rc = upload(&p->d_polys, tab);
    if (!rc) rc = upload(&p->d_ids, ids);
    if (rc) return rc;
    p->grid = persistent_grid(h, c, p->nseg);

    const SegArgs a = seg_args(h, c, p->d_runs, p->nrun, p->nseg, p->kcap, p->d_polys, h->d_counter);
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return set_error(CPRNG_E_HIP, "hipStreamCreate (capture)");
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_zero_u32(h->d_counter, 8, cs);
    if (e == hipSuccess && p->nseg) e = launch_segments(a, p->grid, c.block, seg_kernel_store(c), seg_lds_min(c), cs);
    if (e == hipSuccess) e = launch_commit(h->d_state, h->d_state_next, p->d_ids, (uint32_t)ids.size(), h->ns, cs);
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
            p->block != c.block || p->store != c.store)
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
    if (h->variant == CPRNG_V3_BBS)
        return set_error(CPRNG_E_UNSUPPORTED, "batched uneven streams: the BBS variant has no jump-ahead");
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

void destroy_req_slots(cprng_t *h)
{
    for (ReqSlot *r : h->req_slots) {
        if (r->d_counter) (void)hipFree(r->d_counter);
        if (r->d_buf) (void)hipFree(r->d_buf);
        if (r->h_stage) (void)hipHostFree(r->h_stage);
        if (r->ev_stage) (void)hipEventDestroy(r->ev_stage);
        if (r->d_sub_ctl) (void)hipFree(r->d_sub_ctl);
        if (r->d_sub_buf) (void)hipFree(r->d_sub_buf);
        delete r;
    }
    h->req_slots.clear();
    for (auto &kv : h->d_req_poly_tables) (void)hipFree(kv.second);
    h->d_req_poly_tables.clear();
    h->req_poly_kcap.clear();
    for (auto &kv : h->d_sub_tables) (void)hipFree(kv.second);
    h->d_sub_tables.clear();
    if (h->d_sub_mark) (void)hipFree(h->d_sub_mark);
    h->d_sub_mark = nullptr;
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

int plan_ragged_v0(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, V0Launch &p)
{
    uint64_t total = 0, max_len = 0;
    int rc = check_ragged_args(h, out, lengths, offsets, &total, &max_len);
    if (rc) return rc;
    if (h->variant != CPRNG_V0_PLAIN) return set_error(CPRNG_E_UNSUPPORTED, "this path covers the V0 variant");
    std::string why;
    if (!jump_init(&why)) return set_error(CPRNG_E_UNSUPPORTED, "jump polynomials: " + why);
    const SegCfg c = resolve_seg_cfg(h, total, max_len);
    p = V0Launch{};
    p.chunk = c.chunk;
    p.unroll = c.unroll;
    p.waves = c.waves;
    p.block = c.block;
    p.store = c.store;
    // Longest runs first, so that the queues end with short segments.
    std::vector<uint32_t> order;
    for (uint32_t s = 0; s < h->ns; ++s)
        if (lengths[s]) order.push_back(s);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return lengths[a] > lengths[b]; });
    std::vector<uint64_t> offs(h->ns);
    uint64_t acc = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        offs[s] = offsets ? offsets[s] : acc;
        acc += lengths[s];
    }
    RunList rl;
    for (uint32_t s : order) {
        if (!rl.add(s, (uint64_t)(uintptr_t)out + 4u * offs[s], lengths[s], c.chunk, 1))
            return set_error(CPRNG_E_INVAL, "too many segments (raise the chunk length)");
        p.ids.push_back(s);
    }
    p.runs = std::move(rl.runs);
    p.nseg = rl.nseg;
    p.max_seg = rl.max_seg;
    p.kcap = kcap_for(rl.max_seg);
    return CPRNG_OK;
}

hipError_t launch_ragged_v0(const cprng_t *h, const V0Launch &p, const RunDesc *d_runs, const uint32_t *d_ids,
                            const uint32_t *d_polys, uint32_t *d_counter, uint32_t *d_state_next, hipStream_t st)
{
    const SegCfg c{p.chunk, p.unroll, p.waves, p.block, p.store};
    SegArgs a = seg_args(h, c, d_runs, (uint32_t)p.runs.size(), p.nseg, p.kcap, d_polys, d_counter);
    a.state_next = d_state_next;
    hipError_t e = launch_zero_u32(d_counter, 8, st);
    if (e == hipSuccess && p.nseg)
        e = launch_segments(a, persistent_grid(h, c, p.nseg), c.block, seg_kernel_store(c), seg_lds_min(c), st);
    if (e == hipSuccess) e = launch_commit(h->d_state, d_state_next, d_ids, (uint32_t)p.ids.size(), h->ns, st);
    return e;
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
    if (h->variant == CPRNG_V1_NAIVE3) return ragged_v1(h, out, lengths, offsets, (hipStream_t)stream, true);
    if (h->variant != CPRNG_V0_PLAIN) return ragged_groups(h, out, lengths, offsets, (hipStream_t)stream);
    rc = ensure_common(h);
    if (rc) return rc;
    const SegCfg c = resolve_seg_cfg(h, total, max_len);
    return ragged_with(h, out, lengths, offsets, (hipStream_t)stream, c);
}

extern "C" int cprng_resolved_tuning_ragged(cprng_t *h, const uint64_t *lengths, cprng_tuning_t *out, int *source)
{
    if (!h || !lengths || !out) return set_error(CPRNG_E_INVAL, "NULL argument");
    if (h->variant == CPRNG_V3_BBS || (h->flags & CPRNG_F_INTERLEAVED))
        return set_error(CPRNG_E_UNSUPPORTED, "no batched uneven form for this handle");
    uint64_t total = 0, max_len = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        total += lengths[s];
        max_len = std::max(max_len, lengths[s]);
    }
    DevGuard g(h->device);
    TuneEntry e;
    const bool cached = tune_cache_lookup_key(tune_key_ragged(h, total, max_len), &e);
    std::memset(out, 0, sizeof *out);
    if (h->variant == CPRNG_V0_PLAIN) {
        const SegCfg c = resolve_seg_cfg(h, total, max_len);
        out->chunk = c.chunk;
        out->unroll = c.unroll;
        out->waves_per_cu = c.waves;
        out->block = c.block;
        out->store = c.store;
    } else {
        const ChunkCfg c = resolve_chunk_cfg(h, total, max_len);
        uint64_t chunk = 0;
        const int rc = chunk_for(h, lengths, c, &chunk);
        if (rc) return rc;
        out->chunk = (uint32_t)std::min<uint64_t>(chunk, 0xFFFFFFFFull);
        out->unroll = c.round;
        out->block = 64u * c.wg_waves;
        out->streams_per_lane = h->variant == CPRNG_V1_NAIVE3 ? c.parts : 0u;
    }
    if (source) {
        const cprng_tuning_t &t = h->tuning;
        *source = (t.block || t.unroll || t.store || t.chunk || t.waves_per_cu || t.streams_per_lane || t.exchange)
                      ? 2 : cached ? 1 : 0;
    }
    return CPRNG_OK;
}

extern "C" int cprng_autotune_ragged(cprng_t *h, uint32_t *out, const uint64_t *lengths,
                                     const uint64_t *offsets, cprng_stream_t stream)
{
    uint64_t total = 0, max_len = 0;
    int rc = check_ragged_args(h, out, lengths, offsets, &total, &max_len);
    if (rc) return rc;
    DevGuard g(h->device);
    hipStream_t st = (hipStream_t)stream;
    StateBackup backup;
    if ((rc = backup.save(h, st))) return rc;
    if (h->variant != CPRNG_V0_PLAIN) {
        rc = autotune_chunked(h, out, lengths, offsets, st, total, max_len);
        const int rrc = backup.restore(h, st);
        return rc ? rc : rrc;
    }
    rc = ensure_common(h);
    if (rc) return rc;
    const uint32_t chunks[] = {1024, 2048, 4096, 8192, 16384};
    const uint32_t waves[] = {1, 2, 3, 4, 8};
    // (store, unroll, block): per-lane stores and LDS tiles of several widths
    const uint32_t modes[][3] = {{ST_DIRECT, 16, 256}, {ST_DIRECT, 32, 256}, {ST_LDS, 32, 64},
                                 {ST_LDS, 64, 64}, {ST_LDS, 128, 64}, {ST_LDS_NT, 32, 64},
                                 {ST_LDS_NT, 128, 64}, {ST_PIPE, 64, 64}, {ST_PIPE, 128, 64},
                                 {ST_PIPE_NT, 128, 64}};
    std::vector<SegCfg> cands;
    SegCfg d = kDefaultSeg;
    normalize(d);
    cands.push_back(d);                                      // candidate 0: the default
    for (uint32_t ch : chunks)
        for (uint32_t w : waves)
            for (const auto &m : modes) {
                SegCfg c{ch, m[1], w, m[2], m[0]};
                normalize(c);
                cands.push_back(c);
            }
    const bool saved_timing = h->timing;
    h->timing = false;
    auto drop = [&](const SegCfg &c) {
        if (RaggedPlan *p = find_plan(h, out, lengths, offsets, c)) {
            h->plans.erase(std::find(h->plans.begin(), h->plans.end(), p));
            free_plan(p);
        }
    };
    size_t best = 0;
    rc = tune_select(
        cands.size(), 0, st,
        [&](size_t i) {
            const int r = ragged_with(h, out, lengths, offsets, st, cands[i]);
            return r;
        },
        [&](size_t i, bool kept) {
            if (!kept) drop(cands[i]);
        },
        &best);
    // Only the winner's graph is kept.
    for (size_t i = 0; i < cands.size(); ++i)
        if (i != best) drop(cands[i]);
    h->timing = saved_timing;
    const int rrc = backup.restore(h, st);
    if (rc) return rc;
    if (rrc) return rrc;
    const SegCfg best_c = cands[best];
    TuneEntry e;
    e.block = best_c.block;
    e.unroll = best_c.unroll;
    e.chunk = best_c.chunk;
    e.waves = best_c.waves;
    e.store = best_c.store;
    tune_cache_store(tune_key_ragged(h, total, max_len), e);
    return CPRNG_OK;
}

// ---------------------------------------------------------------------------
// Request batches.
// ---------------------------------------------------------------------------
namespace {

// Per-handle jump table for requests with chunk `chunk`, grown on demand.
int request_table(cprng_t *h, uint32_t chunk, uint64_t max_seg, const uint32_t **dptr, uint32_t *kcap)
{
    const uint32_t need = kcap_for(max_seg);
    auto it = h->req_poly_kcap.find(chunk);
    if (it != h->req_poly_kcap.end() && it->second >= need) {
        *dptr = h->d_req_poly_tables[chunk];
        *kcap = it->second;
        return CPRNG_OK;
    }
    std::vector<uint32_t> tab;
    jump_table(chunk, need, tab);
    // The old table may still be read by queued work; wait before freeing it.
    if (hipDeviceSynchronize() != hipSuccess) return set_error(CPRNG_E_HIP, "hipDeviceSynchronize");
    uint32_t *d = nullptr;
    if (hipMalloc(&d, tab.size() * sizeof(uint32_t)) != hipSuccess) return set_error(CPRNG_E_NOMEM, "hipMalloc table");
    if (hipMemcpy(d, tab.data(), tab.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return set_error(CPRNG_E_HIP, "hipMemcpy table");
    }
    auto dit = h->d_req_poly_tables.find(chunk);
    if (dit != h->d_req_poly_tables.end()) (void)hipFree(dit->second);
    h->d_req_poly_tables[chunk] = d;
    h->req_poly_kcap[chunk] = need;
    *dptr = d;
    *kcap = need;
    return CPRNG_OK;
}

// Chunk length of a request batch: the tuned chunk, halved (down to 1,024)
// while the batch would not give every SIMD two lanes of work, then (down
// to 256) while it gives fewer than 4,096 lanes.  Such a batch is
// latency-bound: each lane walks its jump and then its chunk serially, so
// shorter chunks finish sooner (one request of 2^17 numbers: 56 -> 42 us
// round trip), while larger batches would only add jumps (2^22 numbers:
// 59 us at 1,024-output chunks, 62 us at 256).
constexpr uint32_t kMinRequestChunk = 256;

uint32_t request_chunk(const cprng_t *h, uint32_t chunk, uint64_t total)
{
    if (h->tuning.chunk) return chunk;
    const uint64_t lanes_wanted = (uint64_t)h->n_cu * 4 * 64 * 2;
    while (chunk > 1024 && total / chunk < lanes_wanted) chunk /= 2;
    while (chunk > kMinRequestChunk && total / chunk < 4096) chunk /= 2;
    return chunk;
}

ReqSlot *find_slot(cprng_t *h, hipStream_t st, int *rc)
{
    for (ReqSlot *r : h->req_slots)
        if (r->stream == st) return r;
    if (h->req_slots.size() >= 16) {
        *rc = set_error(CPRNG_E_UNSUPPORTED, "request batches on more than 16 distinct HIP streams");
        return nullptr;
    }
    ReqSlot *r = new ReqSlot();
    r->stream = st;
    r->index = (uint32_t)h->req_slots.size();
    // The queue counters start at zero; each request launch's commit kernel
    // clears them again for the next launch on this stream.
    if (hipMalloc(&r->d_counter, 64) != hipSuccess || hipMemset(r->d_counter, 0, 64) != hipSuccess ||
        hipEventCreateWithFlags(&r->ev_stage, hipEventDisableTiming) != hipSuccess) {
        if (r->d_counter) (void)hipFree(r->d_counter);
        delete r;
        *rc = set_error(CPRNG_E_NOMEM, "request slot allocation");
        return nullptr;
    }
    h->req_slots.push_back(r);
    return r;
}

}  // namespace

extern "C" int cprng_generate_requests(cprng_t *h, const cprng_request_t *reqs, uint32_t count,
                                       cprng_stream_t stream)
{
    if (!h || (!reqs && count)) return set_error(CPRNG_E_INVAL, "NULL argument");
    if (h->variant != CPRNG_V0_PLAIN && h->variant != CPRNG_V1_NAIVE3)
        return set_error(CPRNG_E_UNSUPPORTED, "requests need the V0 or V1 variant (per-stream jump-ahead)");
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
    if (total == 0) return CPRNG_OK;
    DevGuard g(h->device);
    if (h->variant == CPRNG_V1_NAIVE3) {
        // Round j serves the j-th non-empty request of every stream as one
        // batched uneven call; outputs are addressed from the lowest request
        // address.
        std::unordered_map<uint32_t, uint32_t> seen;
        std::vector<std::vector<const cprng_request_t *>> rounds;
        uintptr_t lo = ~(uintptr_t)0;
        for (uint32_t r = 0; r < count; ++r) {
            if (reqs[r].length == 0) continue;
            const uint32_t j = seen[reqs[r].stream]++;
            if (j >= rounds.size()) rounds.emplace_back();
            rounds[j].push_back(&reqs[r]);
            lo = std::min(lo, (uintptr_t)reqs[r].out);
        }
        std::vector<uint64_t> lengths(h->ns), offs(h->ns);
        for (const auto &rd : rounds) {
            std::fill(lengths.begin(), lengths.end(), 0);
            std::fill(offs.begin(), offs.end(), 0);
            for (const cprng_request_t *q : rd) {
                lengths[q->stream] = q->length;
                offs[q->stream] = ((uintptr_t)q->out - lo) / 4u;
            }
            const int rc = ragged_v1(h, (uint32_t *)lo, lengths.data(), offs.data(), (hipStream_t)stream, false);
            if (rc) return rc;
        }
        return CPRNG_OK;
    }
    int rc = ensure_common(h);
    if (rc) return rc;
    SegCfg c = resolve_seg_cfg(h, total, max_len);
    c.chunk = request_chunk(h, c.chunk, total);

    // Launch j serves the j-th non-empty request of every stream.
    std::unordered_map<uint32_t, uint32_t> seen;
    std::vector<RunList> launches;
    std::vector<std::vector<uint32_t>> ids;
    uint64_t max_seg = 0;
    for (uint32_t r = 0; r < count; ++r) {
        const cprng_request_t &q = reqs[r];
        if (q.length == 0) continue;
        const uint32_t j = seen[q.stream]++;
        if (j >= launches.size()) {
            launches.emplace_back();
            ids.emplace_back();
        }
        if (!launches[j].add(q.stream, (uint64_t)(uintptr_t)q.out, q.length, c.chunk, 1))
            return set_error(CPRNG_E_INVAL, "too many segments in one launch");
        ids[j].push_back(q.stream);
        max_seg = std::max(max_seg, launches[j].max_seg);
    }
    const uint32_t *d_tab = nullptr;
    uint32_t kcap = 0;
    rc = request_table(h, c.chunk, max_seg, &d_tab, &kcap);
    if (rc) return rc;

    hipStream_t st = (hipStream_t)stream;
    ReqSlot *slot = find_slot(h, st, &rc);
    if (!slot) return rc;

    // Small batches (every launch at most kInlineRuns runs, tiled persistent
    // stores) carry their runs and commit ids in the kernel arguments: no
    // upload, no wait for the staging buffer.
    bool inline_ok = seg_persistent(c) && (seg_kernel_store(c) == ST_LDS || seg_kernel_store(c) == ST_LDS_NT);
    for (size_t j = 0; j < launches.size() && inline_ok; ++j)
        inline_ok = launches[j].runs.size() <= kInlineRuns && ids[j].size() <= kInlineRuns;
    if (inline_ok) {
        if (h->timing && hipEventRecord(h->ev0, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
        hipError_t e = hipSuccess;
        for (size_t j = 0; j < launches.size() && e == hipSuccess; ++j) {
            SegInline si;
            std::memset(&si, 0, sizeof si);
            si.a = seg_args(h, c, nullptr, (uint32_t)launches[j].runs.size(), launches[j].nseg, kcap, d_tab,
                            slot->d_counter);
            std::memcpy(si.runs, launches[j].runs.data(), launches[j].runs.size() * sizeof(RunDesc));
            std::memcpy(si.ids, ids[j].data(), ids[j].size() * sizeof(uint32_t));
            si.n_ids = (uint32_t)ids[j].size();
            if (!slot->counters_clean) e = launch_zero_u32(slot->d_counter, 8, st);
            slot->counters_clean = false;
            if (e == hipSuccess) e = launch_segments_inline(si, persistent_grid(h, c, si.a.nseg), seg_kernel_store(c), st);
            if (e == hipSuccess) e = launch_commit_inline(si, h->d_state, st);
            if (e == hipSuccess) slot->counters_clean = true;
        }
        if (e != hipSuccess) return hip_error(e, "request kernels");
        if (h->timing) {
            if (hipEventRecord(h->ev1, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
            h->ev_pending = true;
        }
        return CPRNG_OK;
    }

    // Stage every launch's runs and ids in one pinned buffer and copy it with
    // one transfer.  The previous call on this stream may still be running:
    // wait until its transfer has left the staging buffer; on the device the
    // buffer is reused in stream order.
    size_t bytes = 0;
    std::vector<size_t> run_off(launches.size()), id_off(launches.size());
    for (size_t j = 0; j < launches.size(); ++j) {
        run_off[j] = bytes;
        bytes += launches[j].runs.size() * sizeof(RunDesc);
    }
    for (size_t j = 0; j < launches.size(); ++j) {
        id_off[j] = bytes;
        bytes += ids[j].size() * sizeof(uint32_t);
    }
    if (hipEventSynchronize(slot->ev_stage) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventSynchronize");
    if (bytes > slot->buf_cap) {
        if (slot->d_buf) (void)hipFree(slot->d_buf);       // hipFree waits for the device
        if (slot->h_stage) (void)hipHostFree(slot->h_stage);
        slot->d_buf = nullptr;
        slot->h_stage = nullptr;
        slot->buf_cap = 0;
        const size_t cap = std::max<size_t>(bytes * 2, 1 << 16);
        if (hipMalloc(&slot->d_buf, cap) != hipSuccess) return set_error(CPRNG_E_NOMEM, "hipMalloc request buffer");
        if (hipHostMalloc(&slot->h_stage, cap, hipHostMallocDefault) != hipSuccess)
            return set_error(CPRNG_E_NOMEM, "hipHostMalloc staging");
        slot->buf_cap = cap;
    }
    char *hs = (char *)slot->h_stage;
    for (size_t j = 0; j < launches.size(); ++j) {
        std::memcpy(hs + run_off[j], launches[j].runs.data(), launches[j].runs.size() * sizeof(RunDesc));
        std::memcpy(hs + id_off[j], ids[j].data(), ids[j].size() * sizeof(uint32_t));
    }
    hipError_t e = hipMemcpyAsync(slot->d_buf, hs, bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(slot->ev_stage, st);
    if (e != hipSuccess) return hip_error(e, "request upload");

    char *db = (char *)slot->d_buf;
    if (h->timing && hipEventRecord(h->ev0, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
    for (size_t j = 0; j < launches.size() && e == hipSuccess; ++j) {
        const SegArgs a = seg_args(h, c, (const RunDesc *)(db + run_off[j]), (uint32_t)launches[j].runs.size(),
                                   launches[j].nseg, kcap, d_tab, slot->d_counter);
        // The counters are zero unless an earlier launch failed before its
        // commit could clear them.
        if (!slot->counters_clean) e = launch_zero_u32(slot->d_counter, 8, st);
        slot->counters_clean = false;
        if (e == hipSuccess) e = launch_segments(a, persistent_grid(h, c, a.nseg), c.block, seg_kernel_store(c), seg_lds_min(c), st);
        if (e == hipSuccess)
            e = launch_commit(h->d_state, h->d_state_next, (const uint32_t *)(db + id_off[j]),
                              (uint32_t)ids[j].size(), h->ns, st, slot->d_counter);
        if (e == hipSuccess) slot->counters_clean = true;
    }
    if (e != hipSuccess) return hip_error(e, "request kernels");
    if (h->timing) {
        if (hipEventRecord(h->ev1, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
        h->ev_pending = true;
    }
    return CPRNG_OK;
}

namespace {

// Chunking of subset calls: the handle's tuning over the batched default, in
// a persistent store mode (the launch grid cannot follow a segment count
// that only the device knows).
SegCfg subset_cfg(const cprng_t *h)
{
    SegCfg c = kDefaultSeg;
    if (h->tuning.chunk) c.chunk = h->tuning.chunk;
    if (h->tuning.waves_per_cu) c.waves = h->tuning.waves_per_cu;
    if (h->tuning.unroll) c.unroll = h->tuning.unroll;
    if (h->tuning.block) c.block = h->tuning.block;
    if (h->tuning.store) c.store = h->tuning.store == ST_DIRECT_NT ? (uint32_t)ST_DIRECT : h->tuning.store;
    normalize(c);
    if (!seg_persistent(c)) c.store = seg_kernel_store(c);
    return c;
}

// Jump tables of subset calls for one chunk length, one allocation: rows
// X^(k * chunk) mod q, then rows X^(k * 2^13 * chunk) mod q, k < 2^13, five
// words each.
int subset_tables(cprng_t *h, uint32_t chunk, const uint32_t **lo, const uint32_t **hi)
{
    const uint32_t rows = 1u << kSubsetLoBits;
    auto it = h->d_sub_tables.find(chunk);
    if (it == h->d_sub_tables.end()) {
        std::vector<uint32_t> tab;
        jump_table(chunk, rows, tab);
        tab.resize((size_t)rows * 10u);
        const JPoly step = jump_xpow((uint64_t)chunk << kSubsetLoBits);
        JPoly r = jump_one();
        for (uint32_t k = 0; k < rows; ++k) {
            jump_pack(r, &tab[(size_t)(rows + k) * 5u]);
            r = jump_mul(r, step);
        }
        uint32_t *d = nullptr;
        if (hipMalloc(&d, tab.size() * sizeof(uint32_t)) != hipSuccess)
            return set_error(CPRNG_E_NOMEM, "hipMalloc subset jump table");
        if (hipMemcpy(d, tab.data(), tab.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            return set_error(CPRNG_E_HIP, "hipMemcpy subset jump table");
        }
        it = h->d_sub_tables.emplace(chunk, d).first;
    }
    *lo = it->second;
    *hi = it->second + (size_t)rows * 5u;
    return CPRNG_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte offsets in a slot's subset buffer for cap descriptors: segment counts,
// block sums, run descriptors.
void subset_layout(uint32_t cap, size_t *off_bsum, size_t *off_runs, size_t *total)
{
    *off_bsum = align_up((size_t)cap * 4u, 256);
    *off_runs = align_up(*off_bsum + (size_t)((cap + 255u) / 256u) * 8u, 256);
    *total = *off_runs + (size_t)cap * sizeof(RunDesc);
}

// The handle's stream marks and the slot's control block and buffers for
// count descriptors.  Allocates only on a slot's first call and when count
// exceeds every earlier call's.
int subset_buffers(cprng_t *h, ReqSlot *slot, uint32_t count)
{
    if (!h->d_sub_mark) {
        if (hipMalloc(&h->d_sub_mark, (size_t)h->ns * 8u) != hipSuccess)
            return set_error(CPRNG_E_NOMEM, "hipMalloc subset marks");
        if (hipMemset(h->d_sub_mark, 0, (size_t)h->ns * 8u) != hipSuccess)
            return set_error(CPRNG_E_HIP, "hipMemset subset marks");
    }
    if (!slot->d_sub_ctl) {
        SubsetCtl c;
        std::memset(&c, 0, sizeof c);
        c.epoch = ((unsigned long long)(slot->index + 1u) << 56) | 1ull;   // never 0, the marks' initial value
        if (hipMalloc(&slot->d_sub_ctl, sizeof c) != hipSuccess)
            return set_error(CPRNG_E_NOMEM, "hipMalloc subset control block");
        if (hipMemcpy(slot->d_sub_ctl, &c, sizeof c, hipMemcpyHostToDevice) != hipSuccess)
            return set_error(CPRNG_E_HIP, "hipMemcpy subset control block");
    }
    if (count > slot->sub_cap) {
        if (slot->d_sub_buf) (void)hipFree(slot->d_sub_buf);   // hipFree waits for the device
        slot->d_sub_buf = nullptr;
        slot->sub_cap = 0;
        const uint32_t cap = (uint32_t)std::min<uint64_t>(h->ns, std::max<uint64_t>(1024u, 2ull * count));
        size_t ob, orr, total;
        subset_layout(cap, &ob, &orr, &total);
        if (hipMalloc(&slot->d_sub_buf, total) != hipSuccess) return set_error(CPRNG_E_NOMEM, "hipMalloc subset buffers");
        slot->sub_cap = cap;
    }
    return CPRNG_OK;
}

}  // namespace

extern "C" int cprng_generate_subset(cprng_t *h, const uint32_t *ids, const uint64_t *lens,
                                     const uint64_t *out_offsets, uint32_t count, uint32_t *out_base,
                                     int32_t *status, cprng_stream_t stream)
{
    if (!h) return set_error(CPRNG_E_INVAL, "NULL handle");
    if (h->variant != CPRNG_V0_PLAIN)
        return set_error(CPRNG_E_UNSUPPORTED, "subsets need the V0 variant (per-stream jump-ahead planned on the device)");
    if (count == 0) return CPRNG_OK;
    if (!ids || !lens || !out_offsets || !out_base) return set_error(CPRNG_E_INVAL, "NULL argument");
    if ((uintptr_t)ids % 4u || (uintptr_t)lens % 8u || (uintptr_t)out_offsets % 8u || (uintptr_t)out_base % 4u ||
        (uintptr_t)status % 4u)
        return set_error(CPRNG_E_INVAL, "misaligned argument (ids, out_base, status: 4 bytes; lens, offsets: 8)");
    if (count > h->ns) return set_error(CPRNG_E_INVAL, "more descriptors than streams (a stream id would repeat)");
    DevGuard g(h->device);
    int rc = ensure_common(h);
    if (rc) return rc;
    const SegCfg c = subset_cfg(h);
    if (c.chunk % 64u || c.chunk < kSubsetMinChunk)
        return set_error(CPRNG_E_INVAL, "subset calls need a chunk length of at least 2048, a multiple of 64");
    const uint32_t *lo = nullptr, *hi = nullptr;
    if ((rc = subset_tables(h, c.chunk, &lo, &hi))) return rc;
    hipStream_t st = (hipStream_t)stream;
    ReqSlot *slot = find_slot(h, st, &rc);
    if (!slot) return rc;
    if ((rc = subset_buffers(h, slot, count))) return rc;

    size_t ob, orr, total;
    subset_layout(slot->sub_cap, &ob, &orr, &total);
    char *buf = (char *)slot->d_sub_buf;
    SubsetArgs sa;
    std::memset(&sa, 0, sizeof sa);
    sa.ids = ids;
    sa.lens = lens;
    sa.offs = out_offsets;
    sa.count = count;
    sa.ns = h->ns;
    sa.chunk = c.chunk;
    sa.nblocks = (count + 255u) / 256u;
    sa.out_base = (uint64_t)(uintptr_t)out_base;
    sa.mark = h->d_sub_mark;
    sa.ctl = slot->d_sub_ctl;
    sa.segs = (uint32_t *)buf;
    sa.bsum = (unsigned long long *)(buf + ob);
    sa.runs = (RunDesc *)(buf + orr);
    sa.status = status;
    SegArgs a = seg_args(h, c, sa.runs, count, 0, 1u << kSubsetLoBits, lo, slot->d_sub_ctl->counter);
    a.nseg_dev = &slot->d_sub_ctl->nseg;
    a.polys_hi = hi;
    a.lo_bits = kSubsetLoBits;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1u, (uint64_t)h->n_cu * c.waves / (c.block / 64u));

    if (h->timing && hipEventRecord(h->ev0, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
    const hipError_t e = launch_subset(sa, a, grid, c.block, seg_kernel_store(c), h->d_state, st);
    if (e != hipSuccess) return hip_error(e, "subset kernels");
    if (h->timing) {
        if (hipEventRecord(h->ev1, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
        h->ev_pending = true;
    }
    return CPRNG_OK;
}

namespace cprng_impl {

int prepare_request_tables(cprng_t *h, uint64_t max_len)
{
    int rc = ensure_common(h);
    if (rc) return rc;
    const SegCfg c = resolve_seg_cfg(h, max_len, max_len);
    // Every chunk length request_chunk() can pick for a run of max_len.
    for (uint32_t chunk = c.chunk;; chunk /= 2) {
        const uint32_t *d = nullptr;
        uint32_t kcap = 0;
        rc = request_table(h, chunk, segments_of(max_len, 0, chunk), &d, &kcap);
        if (rc || chunk <= kMinRequestChunk || h->tuning.chunk) return rc;
    }
}

}  // namespace cprng_impl
