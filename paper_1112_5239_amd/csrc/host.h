// host.h -- host-side pieces of the library: seeding, combination arrays,
// GF(2) jump polynomials, error reporting and the handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "cprng.h"
#include "internal.h"

namespace cprng_impl {

// ---- errors ---------------------------------------------------------------
int set_error(int status, const std::string &detail);
int hip_error(hipError_t e, const char *what);

// ---- seeding (seed.cpp) ---------------------------------------------------
// Words per stream of a variant (V0 5, V1 23, V2 6).
int words_per_stream(int variant);
// Fill AoS words (n_streams x words) for streams [first, first+count).
void seed_streams(int variant, bool w32, uint64_t sigma, uint64_t first, uint64_t count,
                  uint32_t *aos);
// The same from an explicit SplitMix64 start counter per stream.
void seed_streams_at(int variant, bool w32, const uint64_t *counters, uint64_t count, uint32_t *aos);
// Default combination arrays for a group of C streams (C >= 3).
bool default_combs(uint32_t C, uint32_t *comb1, uint32_t *comb2);
// Default 16 arrangement arrays of the BBS variant (out: 16*C entries).
bool default_bbs_combs(uint32_t C, uint32_t *out);

// ---- GF(2) jump polynomials (gf2.cpp) ------------------------------------
// Elements of GF(2)[X]/(q) with q the annihilating polynomial of the V0
// one-step map on (xor128 words, x); deg q <= 129, so 3 64-bit words.
struct JPoly {
    uint64_t w[3];
};
// Initialise (idempotent, thread-safe): computes q and self-checks it.
bool jump_init(std::string *why);
JPoly jump_mul(const JPoly &a, const JPoly &b);
JPoly jump_xpow(uint64_t J);          // X^J mod q
JPoly jump_one();
// Pack into the kernel's 5 x 32-bit coefficient words (coefficients 0..128).
void jump_pack(const JPoly &p, uint32_t out[5]);
// Packed table of X^(k*chunk) mod q, k = 0..kcap-1, at index k (5 words
// each).  Cached per process and extended on demand.
void jump_table(uint32_t chunk, uint32_t kcap, std::vector<uint32_t> &out);
// Make sure request batches of runs up to max_len outputs find their jump
// table on the device without rebuilding it (segments.cpp).
int prepare_request_tables(cprng_t *h, uint64_t max_len);

// ---- ragged / request plans (segments.cpp, groupjump.cpp) -----------------
struct RaggedPlan;
struct ChunkPlan;
struct ChunkBufs;
// Launch configuration of the chunk kernels of batched V1/V2/V4 calls.
struct ChunkCfg {
    uint64_t chunk = 0;       // outputs per chunk, a multiple of 64; 0 = automatic
    uint32_t round = 64;      // words per lane per store round: 32, 64 or 128
    uint32_t wg_waves = 4;    // waves per workgroup: 1 or 4
    uint32_t parts = 2;       // V1 aggregate pass: lanes per chunk (1, 2 or 4)
};
void destroy_plans(cprng_t *h);

// One launch of the V0 chunk kernels over batched uneven streams, planned on
// the host: the runs (longest first) with their segment numbering, the
// streams to commit, the jump-table rows needed and the launch configuration.
struct V0Launch {
    std::vector<RunDesc> runs;
    std::vector<uint32_t> ids;
    uint64_t nseg = 0, max_seg = 0;
    uint32_t kcap = 0;
    uint32_t chunk = 0, unroll = 0, waves = 0, block = 0, store = 0;
};
// Validate arguments (as cprng_generate_ragged) and plan the launch.  Needs
// a V0 handle; no device work, no device allocation.
int plan_ragged_v0(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, V0Launch &p);
// Enqueue the plan's kernels (queue reset, chunk kernel, commit) on st with
// the given device buffers: runs, commit ids, jump table (p.kcap rows of
// 5 words), 8 queue counters and end-state staging (5 x n_streams words).
hipError_t launch_ragged_v0(const cprng_t *h, const V0Launch &p, const RunDesc *d_runs, const uint32_t *d_ids,
                            const uint32_t *d_polys, uint32_t *d_counter, uint32_t *d_state_next, hipStream_t st);

// Work buffers of request batches on one HIP stream (batches on different
// streams may overlap on the device, so each stream has its own).
struct ReqSlot {
    hipStream_t stream = nullptr;
    uint32_t *d_counter = nullptr;      // work-queue counters
    bool counters_clean = true;         // zero (cleared by the last launch's commit)
    void *d_buf = nullptr;              // run descriptors and commit ids
    void *h_stage = nullptr;            // pinned staging of d_buf
    size_t buf_cap = 0;
    hipEvent_t ev_stage = nullptr;      // the previous upload has completed
    uint32_t index = 0;                 // slot number (top byte of its subset call epochs)
    // subset calls: control block and grow-only work buffers (segment counts,
    // block sums, run descriptors for sub_cap descriptors)
    SubsetCtl *d_sub_ctl = nullptr;
    void *d_sub_buf = nullptr;
    uint32_t sub_cap = 0;
};
void destroy_req_slots(cprng_t *h);

}  // namespace cprng_impl

// The handle.
struct cprng {
    int device = 0;
    uint32_t variant = 0;       // low byte
    uint32_t flags = 0;         // cprng_flags
    uint32_t ns = 0;
    uint32_t words = 0;
    uint32_t group = 0;         // V2
    uint8_t comb1[64] = {0};
    uint8_t comb2[64] = {0};
    uint8_t combs16[16][64] = {{0}};   // V3
    uint32_t *d_state = nullptr;        // SoA, words x ns
    uint32_t *d_state_next = nullptr;   // V0 segment kernels: end states
    uint32_t n_cu = 0;
    cprng_tuning_t tuning{};            // user / autotuned (0 = default)
    bool tuned_loaded = false;

    // timing
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool ev_pending = false;

    // segment machinery (V0)
    uint32_t *d_counter = nullptr;
    std::vector<cprng_impl::RaggedPlan *> plans;
    // requests: work buffers per HIP stream (grow-only)
    std::vector<cprng_impl::ReqSlot *> req_slots;
    // jump tables X^(h + k*chunk) for requests, per chunk length
    std::unordered_map<uint32_t, uint32_t> req_poly_kcap;
    std::unordered_map<uint32_t, uint32_t *> d_req_poly_tables;
    // subset calls: per-stream marks (epoch of the last call listing the
    // stream) and the two-level jump tables, per chunk length
    unsigned long long *d_sub_mark = nullptr;
    std::unordered_map<uint32_t, uint32_t *> d_sub_tables;

    // group jump-ahead (V2/V4 batched uneven runs): minimal polynomial of the
    // group's one-step map and grow-only work buffers
    std::vector<uint64_t> gj_q;
    int gj_deg = 0;
    uint32_t *d_gj_next = nullptr;      // end states of batched V1/V2/V4 calls
    size_t gj_next_cap = 0;
    // batched V1/V2/V4 calls: cached plans with captured graphs, and the
    // grow-only tables of one-off calls (request rounds)
    std::vector<cprng_impl::ChunkPlan *> chunk_plans;
    cprng_impl::ChunkBufs *chunk_direct = nullptr;
};
