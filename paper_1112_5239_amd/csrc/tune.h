// tune.h -- launch configuration defaults, the autotuner and its JSON cache.
#pragma once

#include <functional>
#include <string>
#include <utility>

#include "host.h"

namespace cprng_impl {

struct TuneEntry {
    uint32_t block = 0, unroll = 0, store = 0, chunk = 0, waves = 0, slots = 0, exchange = 0;
};

LaunchCfg default_cfg(uint32_t variant, bool w32, bool consume);
TuneEntry default_entry(uint32_t variant, bool consume);
// Dynamic LDS per block that caps residency at `waves_per_cu` waves per CU
// (0 = no cap); LDS modes only, limited to 64 KiB per block.
uint32_t lds_for_waves(uint32_t block, uint32_t waves_per_cu);
std::string tune_key_generate(const cprng_t *h, uint64_t n);
std::string tune_key_ragged(const cprng_t *h, uint64_t total, uint64_t max_len);
void tune_cache_load(cprng_t *h);
bool tune_cache_lookup(const cprng_t *h, uint64_t n, TuneEntry *e);
bool tune_cache_lookup_key(const std::string &key, TuneEntry *e);
void tune_cache_store(const std::string &key, const TuneEntry &e);

int generate_with(cprng_t *h, uint32_t *out, uint64_t n, hipStream_t st, LaunchCfg c);
// The library's default launch configuration of cprng_generate for this
// handle and n (no cache entry, no explicit tuning), as a cache entry too.
std::pair<LaunchCfg, TuneEntry> default_generate(cprng_t *h, uint64_t n);
// Candidate selection of the autotuners.  run(i) enqueues candidate i once on
// st.  Screening: each candidate is run once untimed, then timed over enough
// back-to-back runs to cover about 2 ms.  Confirmation: the four fastest and
// candidate default_idx are run once more untimed, then timed in 5 rounds that
// alternate between them (so slow drifts of the clock hit all of them alike);
// the lowest median wins, and default_idx is kept unless another candidate
// is more than 1% faster.  after_screen(i, kept) is told which candidates
// take part in the confirmation (to release the others' resources).
int tune_select(size_t n_cand, size_t default_idx, hipStream_t st, const std::function<int(size_t)> &run,
                const std::function<void(size_t, bool)> &after_screen, size_t *best);
// The handle's stream states, copied aside on the device before tuning and
// put back afterwards, so that tuning leaves the streams where they were.
struct StateBackup {
    uint32_t *d = nullptr;
    size_t words = 0;
    int save(const cprng_t *h, hipStream_t st);
    int restore(cprng_t *h, hipStream_t st);
    ~StateBackup();
};
// True for V2/V4 handles whose arrays are the pattern the DPP exchange implements.
bool dpp_pattern(const cprng_t *h);
// Kernel arguments of a handle, and the per-call timing events (api.cpp).
void fill_gen_args(const cprng_t *h, GenArgs &a);
int timing_begin(cprng_t *h, hipStream_t st);
int timing_end(cprng_t *h, hipStream_t st);
// Batched uneven runs of V2/V4 through the group jump-ahead, and of V1
// through per-generator jumps and an aggregate pass (groupjump.cpp).
int group_minpoly(cprng_t *h);
void group_jump_rows(const cprng_t *h, uint64_t chunk, uint32_t rows, std::vector<uint32_t> &out);
// Launch configuration of the chunk kernels: explicit tuning, else the
// autotuner's cache entry for the shape class, else the defaults.
ChunkCfg resolve_chunk_cfg(const cprng_t *h, uint64_t total, uint64_t max_len);
// One batched call with configuration cfg.  cached: the call's tables and a
// captured graph are kept per (lengths, offsets, out, cfg) and replayed;
// otherwise they are built for this call only.
int ragged_chunked(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st,
                   const ChunkCfg &cfg, bool cached);
// The chunk length a call with these lengths and cfg uses (cfg.chunk, or
// the automatic one).
int chunk_for(cprng_t *h, const uint64_t *lengths, const ChunkCfg &cfg, uint64_t *chunk);
int ragged_groups(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st);
int ragged_v1(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st,
              bool cached);
int autotune_chunked(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st,
                     uint64_t total, uint64_t max_len);
void destroy_group_buffers(cprng_t *h);

}  // namespace cprng_impl
