// serve.cpp -- continuous-batching request server over a V0 handle.
//
// Clients are the handle's streams; their generator states stay resident in
// device memory.  Results are carved out of one device arena whose size is
// the admission budget (first-fit, 256-byte granules, neighbours coalesced on
// release).  Each poll collects finished batches (HIP events), admits waiting
// requests in arrival order, and launches one batch per idle HIP stream.  A
// client with a request on the GPU is not admitted again until that batch
// completes, so every launch touches each stream at most once and batches on
// different HIP streams touch disjoint streams (the requirement of
// cprng_generate_requests for overlapping launches).
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.h"

using namespace cprng_impl;

namespace {

constexpr uint64_t kGranule = 256;
constexpr uint64_t kAgingNs = 20ull * 1000 * 1000;      // 20 ms: stop letting others pass
constexpr uint64_t kStallNs = 10ull * 1000 * 1000 * 1000;  // replay gives up after 10 s idle

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Pending {
    uint64_t tag, length, t_submit;
    uint32_t client;
};

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<cprng_completion_t> reqs;
};

}  // namespace

struct cprng_server {
    cprng_t *h = nullptr;
    uint8_t *arena = nullptr;
    uint64_t arena_bytes = 0;
    std::map<uint64_t, uint64_t> free_blocks;          // offset -> bytes
    std::unordered_map<uint64_t, uint64_t> used;       // offset -> bytes
    uint64_t bytes_in_use = 0;
    std::vector<Pending> waiting;                      // arrival order
    std::vector<uint8_t> on_gpu;                       // per client
    std::vector<uint32_t> blocked;                     // per client: pass stamp
    uint32_t pass = 0;
    std::vector<Lane> lanes;
    std::deque<cprng_completion_t> done;
    uint32_t max_batch = 1024;
    uint64_t in_flight = 0;
    std::vector<cprng_request_t> scratch;

    bool alloc(uint64_t bytes, uint64_t *off)
    {
        const uint64_t need = (bytes + kGranule - 1) / kGranule * kGranule;
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const uint64_t rest = it->second - need;
            const uint64_t roff = it->first + need;
            free_blocks.erase(it);
            if (rest) free_blocks[roff] = rest;
            used[*off] = need;
            bytes_in_use += need;
            return true;
        }
        return false;
    }

    bool release(uint64_t off)
    {
        auto u = used.find(off);
        if (u == used.end()) return false;
        uint64_t len = u->second;
        used.erase(u);
        bytes_in_use -= len;
        auto next = free_blocks.lower_bound(off);
        if (next != free_blocks.end() && off + len == next->first) {
            len += next->second;
            next = free_blocks.erase(next);
        }
        if (next != free_blocks.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return true;
            }
        }
        free_blocks[off] = len;
        return true;
    }
};

namespace {

int collect(cprng_server *s)
{
    for (Lane &l : s->lanes) {
        if (!l.busy) continue;
        const hipError_t e = hipEventQuery(l.done);
        if (e == hipErrorNotReady) continue;
        const uint64_t t = now_ns();
        for (cprng_completion_t c : l.reqs) {
            c.t_done_ns = t;
            if (e != hipSuccess) c.status = CPRNG_E_HIP;
            s->on_gpu[c.client] = 0;
            s->done.push_back(c);
        }
        s->in_flight -= l.reqs.size();
        l.reqs.clear();
        l.busy = false;
        if (e != hipSuccess) return hip_error(e, "request batch");
    }
    return CPRNG_OK;
}

int admit_and_launch(cprng_server *s)
{
    for (Lane &l : s->lanes) {
        if (l.busy || s->waiting.empty()) continue;
        const uint64_t t = now_ns();
        ++s->pass;
        bool stop = false;
        std::vector<Pending> kept;
        kept.reserve(s->waiting.size());
        s->scratch.clear();
        for (const Pending &p : s->waiting) {
            if (stop || l.reqs.size() >= s->max_batch || s->on_gpu[p.client] || s->blocked[p.client] == s->pass) {
                s->blocked[p.client] = s->pass;     // keeps this client's order
                kept.push_back(p);
                continue;
            }
            uint64_t off = 0;
            if (!s->alloc(p.length * 4u, &off)) {
                s->blocked[p.client] = s->pass;
                kept.push_back(p);
                if (t - p.t_submit > kAgingNs) stop = true;   // reserve the budget for it
                continue;
            }
            s->on_gpu[p.client] = 1;
            cprng_completion_t c{};
            c.tag = p.tag;
            c.client = p.client;
            c.status = CPRNG_OK;
            c.length = p.length;
            c.out = reinterpret_cast<uint32_t *>(s->arena + off);
            c.t_submit_ns = p.t_submit;
            c.t_admit_ns = t;
            l.reqs.push_back(c);
            cprng_request_t q{};
            q.stream = p.client;
            q.length = p.length;
            q.out = c.out;
            s->scratch.push_back(q);
        }
        s->waiting.swap(kept);
        if (l.reqs.empty()) continue;
        int rc = cprng_generate_requests(s->h, s->scratch.data(), (uint32_t)s->scratch.size(),
                                         (cprng_stream_t)l.stream);
        if (rc == CPRNG_OK && hipEventRecord(l.done, l.stream) != hipSuccess)
            rc = set_error(CPRNG_E_HIP, "hipEventRecord");
        if (rc != CPRNG_OK) {
            // Fail the batch's requests; their results still belong to the caller.
            for (cprng_completion_t c : l.reqs) {
                c.status = rc;
                c.t_done_ns = now_ns();
                s->on_gpu[c.client] = 0;
                s->done.push_back(c);
            }
            l.reqs.clear();
            return rc;
        }
        s->in_flight += l.reqs.size();
        l.busy = true;
    }
    return CPRNG_OK;
}

}  // namespace

extern "C" {

uint64_t cprng_now_ns(void) { return now_ns(); }

int cprng_server_create(cprng_t *h, const cprng_server_params_t *params, cprng_server_t **out)
{
    if (!h || !out) return set_error(CPRNG_E_INVAL, "NULL argument");
    *out = nullptr;
    if (params && params->struct_size < sizeof(cprng_server_params_t))
        return set_error(CPRNG_E_INVAL, "cprng_server_params_t.struct_size too small");
    if (h->variant != CPRNG_V0_PLAIN) return set_error(CPRNG_E_UNSUPPORTED, "the server needs a V0 handle");
    uint32_t nstreams = params && params->n_gpu_streams ? params->n_gpu_streams : 2u;
    uint64_t budget = params && params->budget_bytes ? params->budget_bytes : (64ull << 30);
    const uint32_t max_batch = params && params->max_batch ? params->max_batch : 1024u;
    if (nstreams > 16) return set_error(CPRNG_E_INVAL, "n_gpu_streams must be <= 16");
    budget = budget / kGranule * kGranule;
    if (budget < kGranule) return set_error(CPRNG_E_INVAL, "budget too small");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != h->device) (void)hipSetDevice(h->device);
    std::unique_ptr<cprng_server> s(new cprng_server());
    s->h = h;
    s->max_batch = max_batch;
    s->on_gpu.assign(h->ns, 0);
    s->blocked.assign(h->ns, 0);
    int rc = CPRNG_OK;
    if (hipMalloc(&s->arena, budget) != hipSuccess) rc = set_error(CPRNG_E_NOMEM, "hipMalloc result arena");
    // Build the jump tables for the largest request that fits the budget (at
    // most 2^26 outputs, 256 MiB; larger ones extend the tables on first use),
    // so that no batch pays for them.
    if (!rc) rc = prepare_request_tables(h, std::min<uint64_t>(budget / 4, 1ull << 26));
    if (!rc) {
        s->arena_bytes = budget;
        s->free_blocks[0] = budget;
        s->lanes.resize(nstreams);
        for (Lane &l : s->lanes) {
            if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess) {
                rc = set_error(CPRNG_E_HIP, "server stream/event creation");
                break;
            }
        }
    }
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    if (rc) {
        cprng_server_destroy(s.release());
        return rc;
    }
    *out = s.release();
    return CPRNG_OK;
}

int cprng_server_submit(cprng_server_t *s, uint32_t client, uint64_t length, uint64_t tag, uint64_t t_submit_ns)
{
    if (!s) return set_error(CPRNG_E_INVAL, "NULL server");
    if (client >= s->h->ns) return set_error(CPRNG_E_INVAL, "client id out of range");
    if (length == 0 || length > s->arena_bytes / 4) return set_error(CPRNG_E_INVAL, "length must be in 1 .. budget/4");
    s->waiting.push_back(Pending{tag, length, t_submit_ns ? t_submit_ns : now_ns(), client});
    return CPRNG_OK;
}

int cprng_server_poll(cprng_server_t *s, cprng_completion_t *done, uint32_t max_done, uint32_t *n_done)
{
    if (!s || !n_done || (!done && max_done)) return set_error(CPRNG_E_INVAL, "NULL argument");
    *n_done = 0;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != s->h->device) (void)hipSetDevice(s->h->device);
    int rc = collect(s);
    if (!rc) rc = admit_and_launch(s);
    if (!rc) rc = collect(s);
    if (prev >= 0 && prev != s->h->device) (void)hipSetDevice(prev);
    while (*n_done < max_done && !s->done.empty()) {
        done[(*n_done)++] = s->done.front();
        s->done.pop_front();
    }
    return rc;
}

int cprng_server_release(cprng_server_t *s, uint32_t *out)
{
    if (!s || !out) return set_error(CPRNG_E_INVAL, "NULL argument");
    const uint8_t *p = reinterpret_cast<const uint8_t *>(out);
    if (p < s->arena || p >= s->arena + s->arena_bytes) return set_error(CPRNG_E_INVAL, "not a result of this server");
    if (!s->release((uint64_t)(p - s->arena))) return set_error(CPRNG_E_INVAL, "result not in use");
    return CPRNG_OK;
}

int cprng_server_stats(const cprng_server_t *s, uint64_t *waiting, uint64_t *in_flight, uint64_t *bytes_in_use)
{
    if (!s) return set_error(CPRNG_E_INVAL, "NULL server");
    if (waiting) *waiting = s->waiting.size();
    if (in_flight) *in_flight = s->in_flight;
    if (bytes_in_use) *bytes_in_use = s->bytes_in_use;
    return CPRNG_OK;
}

static int replay_impl(cprng_server_t *s, const uint64_t *arrival_ns, const uint32_t *client,
                       const uint64_t *length, uint32_t count, int release_results, const uint8_t *keep,
                       cprng_completion_t *results);

int cprng_server_replay(cprng_server_t *s, const uint64_t *arrival_ns, const uint32_t *client,
                        const uint64_t *length, uint32_t count, int release_results, cprng_completion_t *results)
{
    return replay_impl(s, arrival_ns, client, length, count, release_results, nullptr, results);
}

int cprng_server_replay_keep(cprng_server_t *s, const uint64_t *arrival_ns, const uint32_t *client,
                             const uint64_t *length, uint32_t count, const uint8_t *keep,
                             cprng_completion_t *results)
{
    if (count && !keep) return set_error(CPRNG_E_INVAL, "NULL keep mask");
    return replay_impl(s, arrival_ns, client, length, count, 1, keep, results);
}

static int replay_impl(cprng_server_t *s, const uint64_t *arrival_ns, const uint32_t *client,
                       const uint64_t *length, uint32_t count, int release_results, const uint8_t *keep,
                       cprng_completion_t *results)
{
    if (!s || (count && (!arrival_ns || !client || !length || !results)))
        return set_error(CPRNG_E_INVAL, "NULL argument");
    for (uint32_t i = 0; i < count; ++i) {
        if (i && arrival_ns[i] < arrival_ns[i - 1]) return set_error(CPRNG_E_INVAL, "arrivals must be non-decreasing");
        if (client[i] >= s->h->ns || length[i] == 0 || length[i] > s->arena_bytes / 4)
            return set_error(CPRNG_E_INVAL, "bad request in trace");
    }
    std::vector<cprng_completion_t> buf(512);
    const uint64_t t0 = now_ns();
    uint32_t next = 0, finished = 0;
    uint64_t last_progress = t0;
    while (finished < count) {
        const uint64_t t = now_ns();
        bool progress = false;
        while (next < count && t0 + arrival_ns[next] <= t) {
            int rc = cprng_server_submit(s, client[next], length[next], next, t0 + arrival_ns[next]);
            if (rc) return rc;
            ++next;
            progress = true;
        }
        uint32_t n = 0;
        int rc = cprng_server_poll(s, buf.data(), (uint32_t)buf.size(), &n);
        for (uint32_t k = 0; k < n; ++k) {
            const cprng_completion_t &c = buf[k];
            results[c.tag] = c;
            ++finished;
            if (release_results && !(keep && keep[c.tag])) (void)cprng_server_release(s, c.out);
        }
        if (rc) return rc;
        if (n) progress = true;
        if (progress) {
            last_progress = t;
        } else if (s->in_flight == 0 && !s->waiting.empty() && t - last_progress > kStallNs) {
            return set_error(CPRNG_E_NOMEM, "replay stalled: waiting requests never fit the budget");
        } else if (s->in_flight == 0 && s->waiting.empty() && next < count) {
            // Idle until the next arrival; sleep most of the gap, spin the rest.
            const uint64_t due = t0 + arrival_ns[next];
            if (due > t + 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(due - t - 100000));
        }
    }
    return CPRNG_OK;
}

void cprng_server_destroy(cprng_server_t *s)
{
    if (!s) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != s->h->device) (void)hipSetDevice(s->h->device);
    for (Lane &l : s->lanes) {
        if (l.stream) (void)hipStreamSynchronize(l.stream);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.stream) (void)hipStreamDestroy(l.stream);
    }
    if (s->arena) (void)hipFree(s->arena);
    if (prev >= 0 && prev != s->h->device) (void)hipSetDevice(prev);
    delete s;
}

}  // extern "C"
