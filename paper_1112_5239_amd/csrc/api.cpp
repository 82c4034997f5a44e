// api.cpp -- C ABI of the chaotic-iteration PRNG library (lifecycle, plain
// generation, consumption, state, tuning, timing, probes).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "host.h"
#include "tune.h"

using namespace cprng_impl;

namespace cprng_impl {

static thread_local std::string g_last_error;

int set_error(int status, const std::string &detail)
{
    g_last_error = detail;
    return status;
}

int hip_error(hipError_t e, const char *what)
{
    return set_error(CPRNG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace cprng_impl

#define HIP_TRY(call, what)                                    \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return hip_error(_e, what);      \
    } while (0)

namespace {

// Make the handle's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

void fill_args(const cprng_t *h, GenArgs &a)
{
    std::memset(&a, 0, sizeof a);
    a.state = h->d_state;
    a.ns = h->ns;
    a.group = h->group ? h->group : 1;
    std::memcpy(a.comb1, h->comb1, 64);
    std::memcpy(a.comb2, h->comb2, 64);
    std::memcpy(a.combs16, h->combs16, sizeof a.combs16);
    const bool xor64 = (h->flags & CPRNG_F_V1_XOR64) != 0;
    a.xs_b = xor64 ? 7u : 17u;
    a.xs_c = xor64 ? 17u : 5u;
}

int begin_timing(cprng_t *h, hipStream_t st)
{
    if (!h->timing) return CPRNG_OK;
    HIP_TRY(hipEventRecord(h->ev0, st), "hipEventRecord");
    return CPRNG_OK;
}

int end_timing(cprng_t *h, hipStream_t st)
{
    if (!h->timing) return CPRNG_OK;
    HIP_TRY(hipEventRecord(h->ev1, st), "hipEventRecord");
    h->ev_pending = true;
    return CPRNG_OK;
}

int create_impl(const cprng_params_t *p, cprng_t **out)
{
    if (!p || !out) return set_error(CPRNG_E_INVAL, "NULL params or output handle");
    *out = nullptr;
    if (p->struct_size < sizeof(cprng_params_t))
        return set_error(CPRNG_E_INVAL, "cprng_params_t.struct_size too small");
    const uint32_t var = p->variant & 0xffu;
    const uint32_t flags = p->variant & ~0xffu;
    if (words_per_stream((int)var) < 0) return set_error(CPRNG_E_INVAL, "unknown variant");
    if (flags & ~(uint32_t)(CPRNG_F_INTERLEAVED | CPRNG_F_V1_W32 | CPRNG_F_V1_XOR64 | CPRNG_F_SEED_PER_STREAM))
        return set_error(CPRNG_E_INVAL, "unknown flag bits");
    if ((flags & CPRNG_F_SEED_PER_STREAM) && !p->seeds)
        return set_error(CPRNG_E_INVAL, "CPRNG_F_SEED_PER_STREAM needs the seeds array");
    if ((flags & CPRNG_F_V1_W32) && var != CPRNG_V1_NAIVE3)
        return set_error(CPRNG_E_INVAL, "CPRNG_F_V1_W32 applies to the V1 variant only");
    if ((flags & CPRNG_F_V1_XOR64) && (var != CPRNG_V1_NAIVE3 || (flags & CPRNG_F_V1_W32)))
        return set_error(CPRNG_E_INVAL, "CPRNG_F_V1_XOR64 applies to the V1 variant with 64-bit words only");
    if (p->n_streams == 0) return set_error(CPRNG_E_INVAL, "n_streams must be >= 1");

    std::unique_ptr<cprng> h(new cprng());
    h->variant = var;
    h->flags = flags;
    h->ns = p->n_streams;
    h->words = (uint32_t)words_per_stream((int)var);

    if (var == CPRNG_V2_SHMEM || var == CPRNG_V4_XOR64) {
        const uint32_t C = p->group ? p->group : 32u;
        if (!is_pow2(C) || C > 64)
            return set_error(CPRNG_E_UNSUPPORTED, "V2/V4 group size must be a power of two <= 64 (a group lies in one wave)");
        if (p->n_streams % C != 0) return set_error(CPRNG_E_INVAL, "V2/V4 need n_streams % group == 0");
        uint32_t c1[64], c2[64];
        if (p->comb1 || p->comb2) {
            if (!p->comb1 || !p->comb2) return set_error(CPRNG_E_INVAL, "give both comb1 and comb2");
            for (uint32_t j = 0; j < C; ++j) {
                if (p->comb1[j] >= C || p->comb2[j] >= C)
                    return set_error(CPRNG_E_INVAL, "combination entry out of range");
                c1[j] = p->comb1[j];
                c2[j] = p->comb2[j];
            }
        } else if (!default_combs(C, c1, c2)) {
            return set_error(CPRNG_E_INVAL, "no default combination arrays for this group size (need C >= 3)");
        }
        h->group = C;
        for (uint32_t j = 0; j < 64; ++j) {
            h->comb1[j] = (uint8_t)c1[j % C];
            h->comb2[j] = (uint8_t)c2[j % C];
        }
    }

    if (var == CPRNG_V3_BBS) {
        const uint32_t C = p->group ? p->group : 32u;
        if (!is_pow2(C) || C < 4 || C > 64)
            return set_error(CPRNG_E_UNSUPPORTED, "V3 group size must be a power of two in [4, 64] (a group lies in one wave)");
        if (p->n_streams % C != 0) return set_error(CPRNG_E_INVAL, "V3 needs n_streams % group == 0");
        if (p->comb1 || p->comb2) return set_error(CPRNG_E_UNSUPPORTED, "V3 uses the library's arrangement arrays");
        uint32_t arr[16 * 64];
        if (!default_bbs_combs(C, arr)) return set_error(CPRNG_E_INVAL, "no arrangement arrays for this group size");
        h->group = C;
        for (uint32_t a = 0; a < 16; ++a)
            for (uint32_t j = 0; j < 64; ++j) h->combs16[a][j] = (uint8_t)arr[a * C + j % C];
    }

    int dev = p->device;
    if (dev < 0) HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    h->device = dev;
    DeviceGuard g(dev);
    if (!g.ok) return set_error(CPRNG_E_HIP, "hipSetDevice failed");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    h->n_cu = (uint32_t)prop.multiProcessorCount;

    // Seed on the host, pack SoA, upload.
    const uint64_t nwords = (uint64_t)h->ns * h->words;
    std::vector<uint32_t> aos(nwords), soa(nwords);
    if (flags & CPRNG_F_SEED_PER_STREAM)
        seed_streams_at((int)var, (flags & CPRNG_F_V1_W32) != 0, p->seeds, h->ns, aos.data());
    else
        seed_streams((int)var, (flags & CPRNG_F_V1_W32) != 0, p->seed, 0, h->ns, aos.data());
    for (uint64_t s = 0; s < h->ns; ++s)
        for (uint32_t k = 0; k < h->words; ++k) soa[k * (uint64_t)h->ns + s] = aos[s * h->words + k];
    if (hipMalloc(&h->d_state, nwords * sizeof(uint32_t)) != hipSuccess)
        return set_error(CPRNG_E_NOMEM, "hipMalloc of the stream states failed");
    HIP_TRY(hipMemcpy(h->d_state, soa.data(), nwords * sizeof(uint32_t), hipMemcpyHostToDevice),
            "hipMemcpy state");
    HIP_TRY(hipEventCreate(&h->ev0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&h->ev1), "hipEventCreate");
    *out = h.release();
    return CPRNG_OK;
}

// Stream-major generate with few streams.  The defaults of default_entry()
// suit 2^18 streams and more; fewer streams leave CUs idle and each wave's
// latency exposed.  Measured on MI355X at 1,024 outputs per stream: up to one
// wave per CU, one-wave blocks storing their own quads beat the LDS tiles
// (1,024 streams: V0 0.016 vs 0.033 ms, V1 0.063 vs 0.081, V2 0.040 vs
// 0.063); beyond that, one-wave LDS tiles of 32 steps for V0 up to six waves
// per CU (65,600 streams: 0.042 vs 0.082 ms; even at 98,304) and for V2/V4
// up to four (65,536: V2 0.064 vs 0.071 ms), and for V1 the direct stores up
// to six (98,304: 0.150 vs 0.160 ms against the large-shape default of rounds
// of 32 with no residency cap; slower by 131,072).  The BBS variant keeps its
// defaults.
void small_shape_defaults(const cprng_t *h, LaunchCfg &c, TuneEntry &e)
{
    if (h->variant == CPRNG_V3_BBS || (h->flags & CPRNG_F_INTERLEAVED)) return;
    const uint64_t ns = h->ns, cu = h->n_cu ? h->n_cu : 256u;
    const bool v0 = h->variant == CPRNG_V0_PLAIN, v1 = h->variant == CPRNG_V1_NAIVE3;
    if (ns <= cu * 64u || (v1 && ns <= cu * 384u)) {
        c.block = 64; c.unroll = 32; c.store = ST_DIRECT;
    } else if (ns <= cu * (v0 ? 384u : 256u) && !v1) {
        c.block = 64; c.unroll = 32; c.store = ST_LDS;
    } else {
        return;
    }
    e.block = c.block; e.unroll = c.unroll; e.store = c.store; e.waves = 0;
}

// The default entry of a stream-major generate call on this handle.
TuneEntry default_generate_entry(const cprng_t *h)
{
    LaunchCfg c = default_cfg(h->variant, (h->flags & CPRNG_F_V1_W32) != 0, false);
    TuneEntry e = default_entry(h->variant, false);
    small_shape_defaults(h, c, e);
    return e;
}

// Launch configuration of a generate / consume call: the library's defaults,
// then the autotuner's entry for the shape class, then cprng_set_tuning's
// fields.  defaults_only: the defaults alone.
LaunchCfg resolve_cfg(cprng_t *h, uint64_t n, bool consume, bool defaults_only = false)
{
    if (!h->tuned_loaded) {
        tune_cache_load(h);
        h->tuned_loaded = true;
    }
    if (!consume && (h->flags & CPRNG_F_INTERLEAVED)) {
        // Interleaved layout: LDS tiles of K steps x block streams, spread
        // over the XCDs in bands.  Measured on MI355X at 2^20 streams x 1024:
        // 1,024 streams x 16 steps, two tile buffers (128 KiB of LDS),
        // non-temporal stores, V2/V4 exchange through the LDS word buffer
        // (as fast as cross-lane reads with the default arrays, and faster
        // with others, e.g. 0.68 vs 0.76 ms with the DPP arrays); V1,
        // VALU-bound, 256 x 32 with one buffer; V3, VALU-bound, 512 x 16
        // with one buffer and the LDS word exchange.  Direct store modes
        // select the per-lane dword kernel.
        LaunchCfg c{1024, 16, ST_ILV_TILE_NT, 0, 2, XCH_LDS, 0};
        if (h->variant == CPRNG_V1_NAIVE3) {
            c.block = 256;
            c.unroll = 32;
            c.slots = 1;
        } else if (h->variant == CPRNG_V3_BBS) {
            c.block = 512;
            c.slots = 1;
            c.exchange = XCH_LDS;
        }
        // With few streams the tiles leave most CUs idle; per-lane dword
        // stores in one-wave blocks of 32 steps are faster: V0 up to five
        // waves' worth of streams per CU (1,024 streams: 0.022 vs 0.068 ms;
        // 65,600: 0.044 vs 0.070; slower by 98,304), V1, V2 and V4 up to
        // eight (1,024: V2 0.055 vs 0.111 ms, V1 0.067 vs 0.080; 131,072: V2
        // 0.114 vs 0.123, V1 0.187 vs 0.192; slower by 196,608).  BBS keeps
        // its tiles, of 256 streams up to four waves' worth per CU (1,024
        // streams: 0.274 vs 0.308 ms; 65,536: 0.294 vs 0.325; equal beyond).
        const uint64_t ilv_cu = h->n_cu ? h->n_cu : 256u;
        if (h->variant == CPRNG_V3_BBS && (uint64_t)h->ns <= ilv_cu * 256u) c.block = 256;
        if (h->variant != CPRNG_V3_BBS &&
            (uint64_t)h->ns <= ilv_cu * (h->variant == CPRNG_V0_PLAIN ? 320u : 512u)) {
            c.block = 64;
            c.unroll = 32;
            c.store = ST_INTERLEAVED;
            c.slots = 1;
        }
        if (defaults_only) return c;
        TuneEntry e;
        if (tune_cache_lookup(h, n, &e) && e.store) {       // the autotuner's pick for this shape class
            c.block = e.block;
            c.unroll = e.unroll;
            c.store = e.store;
            c.slots = e.slots ? e.slots : 1;
            if (e.exchange) c.exchange = e.exchange;
            c.grid = h->n_cu * e.waves;
        }
        if (h->tuning.streams_per_lane) c.slots = h->tuning.streams_per_lane;
        if (h->tuning.store == ST_DIRECT || h->tuning.store == ST_DIRECT_NT) c.store = ST_INTERLEAVED;
        if (h->tuning.store == ST_LDS || h->tuning.store == ST_PIPE) c.store = ST_ILV_TILE;
        if (h->tuning.store == ST_LDS_NT || h->tuning.store == ST_PIPE_NT) c.store = ST_ILV_TILE_NT;
        if (h->tuning.store == 5) c.store = ST_ILV_QUAD;
        if (h->tuning.store == 6) c.store = ST_ILV_QUAD_NT;
        if (c.store == ST_ILV_QUAD || c.store == ST_ILV_QUAD_NT) c.block = 256;
        if (h->tuning.block) c.block = h->tuning.block;
        if (h->tuning.unroll) c.unroll = h->tuning.unroll;
        if (h->tuning.exchange) c.exchange = h->tuning.exchange;
        // waves_per_cu: persistent workgroups per CU (a multiple of 8 overall
        // keeps each workgroup's tiles in its XCD's band); 0 = one per tile
        if (h->tuning.waves_per_cu) c.grid = h->n_cu * h->tuning.waves_per_cu;
        return c;
    }
    LaunchCfg c = default_cfg(h->variant, (h->flags & CPRNG_F_V1_W32) != 0, consume);
    TuneEntry e = default_entry(h->variant, consume);
    if (!consume) small_shape_defaults(h, c, e);
    if (defaults_only) {
        c.lds_bytes = (c.store == ST_PIPE || c.store == ST_PIPE_NT) ? 0u : lds_for_waves(c.block, consume ? 0u : e.waves);
        return c;
    }
    if (!consume && tune_cache_lookup(h, n, &e)) {
        c.block = e.block;
        c.unroll = e.unroll;
        c.store = e.store;
        c.slots = e.slots ? e.slots : 1;
        if (e.exchange) c.exchange = e.exchange;
    }
    if (h->tuning.streams_per_lane) c.slots = h->tuning.streams_per_lane;
    if (h->tuning.exchange) c.exchange = h->tuning.exchange;
    if (h->tuning.block) c.block = h->tuning.block;
    if (h->tuning.unroll) c.unroll = h->tuning.unroll;
    if (h->tuning.store && !consume) c.store = h->tuning.store;
    const uint32_t wpc = h->tuning.waves_per_cu ? h->tuning.waves_per_cu : (consume ? 0u : e.waves);
    if (c.store == ST_PIPE || c.store == ST_PIPE_NT) {
        // persistent: waves per CU sets the grid, one wave per workgroup
        c.block = 64;
        c.grid = h->n_cu * (wpc ? wpc : 2u);
        c.lds_bytes = 0;
    } else {
        c.lds_bytes = lds_for_waves(c.block, wpc);
    }
    return c;
}

}  // namespace

namespace cprng_impl {

void fill_gen_args(const cprng_t *h, GenArgs &a) { fill_args(h, a); }

std::pair<LaunchCfg, TuneEntry> default_generate(cprng_t *h, uint64_t n)
{
    const LaunchCfg c = resolve_cfg(h, n, false, true);
    TuneEntry e;
    e.block = c.block;
    e.unroll = c.unroll;
    e.store = c.store;
    e.slots = c.slots;
    e.exchange = c.exchange;
    e.waves = (h->flags & CPRNG_F_INTERLEAVED) ? (h->n_cu ? c.grid / h->n_cu : 0u) : default_generate_entry(h).waves;
    return {c, e};
}
int timing_begin(cprng_t *h, hipStream_t st) { return begin_timing(h, st); }
int timing_end(cprng_t *h, hipStream_t st) { return end_timing(h, st); }

bool dpp_pattern(const cprng_t *h)
{
    if ((h->variant != CPRNG_V2_SHMEM && h->variant != CPRNG_V4_XOR64) || h->group != kDppGroup) return false;
    for (uint32_t j = 0; j < 64; ++j) {
        const uint32_t r = j % kDppGroup;
        if (h->comb1[j] != (r + kDppOff1) % kDppGroup || h->comb2[j] != (r + kDppOff2) % kDppGroup) return false;
    }
    return true;
}

int generate_with(cprng_t *h, uint32_t *out, uint64_t n, hipStream_t st, LaunchCfg c)
{
    GenArgs a;
    fill_args(h, a);
    a.out = out;
    a.n = n;
    // The DPP exchange implements one pair of arrays; any other handle gets
    // the cross-lane reads, which produce the same words.
    if (c.exchange == XCH_DPP && !dpp_pattern(h)) c.exchange = XCH_BPERM;
    // The BBS variant's arrays differ per thread, so the two-steps-per-read
    // exchange (which follows a neighbour's neighbours) does not apply.
    if (h->variant == CPRNG_V3_BBS && c.exchange == XCH_BPERM2) c.exchange = XCH_BPERM;
    // The BBS variant is ALU-bound: its kernels are built for K <= 32 only.
    if (h->variant == CPRNG_V3_BBS && c.unroll > 32) c.unroll = 32;
    if (h->flags & CPRNG_F_INTERLEAVED) {
        const bool tile_ok = ((uintptr_t)out % 16u) == 0 && (h->ns % 4u) == 0;
        const bool quad = c.store == ST_ILV_QUAD || c.store == ST_ILV_QUAD_NT;
        // The quad-lane kernel covers the 32-bit-word variants V0, V2, V4; the
        // others take the LDS tiles.
        const bool quad_var = h->variant == CPRNG_V0_PLAIN || h->variant == CPRNG_V2_SHMEM ||
                              h->variant == CPRNG_V4_XOR64;
        if (quad && !quad_var) {
            c.store = c.store == ST_ILV_QUAD_NT ? ST_ILV_TILE_NT : ST_ILV_TILE;
            c.block = 256;
        }
        if (!tile_ok || (c.store != ST_ILV_TILE && c.store != ST_ILV_TILE_NT && c.store != ST_ILV_QUAD &&
                         c.store != ST_ILV_QUAD_NT))
            c.store = ST_INTERLEAVED;
        if (c.store == ST_ILV_QUAD || c.store == ST_ILV_QUAD_NT) {
            // 64, 128 or 256 threads, each holding four streams
            if (c.block > 256) c.block = 256;
            if (c.block != 64 && c.block != 128) c.block = 256;
        } else if (c.store == ST_INTERLEAVED) {
            if (c.block > 256) c.block = 256;
            if (c.unroll > 32) c.unroll = 32;
        } else {
            // block: 256, 512 or 1024 streams; the tiles (+ the V2 exchange
            // buffer) must fit a workgroup's LDS
            uint32_t b = 256;
            while (b < c.block && b < 1024) b *= 2;
            c.block = b;
            if (c.unroll < 8) c.unroll = 8;
            if (c.unroll > 64) c.unroll = 64;
            if (c.exchange < XCH_BPERM || c.exchange > XCH_BPERM2) c.exchange = XCH_BPERM;
            if (c.slots != 2) c.slots = 1;      // 2: double-buffered tiles
            const uint32_t extra = (has_exchange(h->variant) && c.exchange == XCH_LDS) ? 1u : 0u;
            if (c.block == 1024 && c.unroll > 32) c.unroll = 32;
            while ((uint64_t)(c.slots * c.unroll + extra) * c.block * 4u > kMaxLdsBytes) {
                if (c.unroll > 8) c.unroll /= 2;
                else if (c.block > 256) c.block /= 2;
                else c.slots = 1;
            }
        }
    } else {
        if (c.block > 256) c.block = 256;
        // Rows off the 128-byte lines take the LDS tiles, whose launch then
        // stores line-aligned pieces: the per-lane quads need n % 4 == 0 and a
        // 16-byte aligned base, and the pipelined tiles would split lines.
        const bool aligned = ((uintptr_t)out % 16u) == 0 && (n % 4u) == 0;
        const bool on_lines = ((uintptr_t)out % 128u) == 0 && (n % 32u) == 0;
        if (!aligned || (!on_lines && (c.store == ST_PIPE || c.store == ST_PIPE_NT))) c.store = ST_LDS_NT;
    }
    if (c.store == ST_LDS || c.store == ST_LDS_NT) {
        // LDS tiles hold K >= 16 words per row; block/64 waves x 64 rows x K
        // words must fit a workgroup's LDS (160 KiB on gfx950).
        if (c.unroll < 16) c.unroll = 16;
        if (c.slots != 1 && c.slots != 2 && c.slots != 4) c.slots = 1;
        if (c.exchange < XCH_BPERM || c.exchange > XCH_BPERM2) c.exchange = XCH_BPERM;
        // tile (+ the exchange buffer) per block must fit the LDS
        const uint32_t extra = (has_exchange(h->variant) && c.exchange == XCH_LDS) ? 1u : 0u;
        while (c.block > 64 && (uint64_t)c.block * c.slots * (c.unroll + extra) * 4u > kMaxLdsBytes) c.block -= 64;
        while (c.slots > 1 && (uint64_t)c.block * c.slots * (c.unroll + extra) * 4u > kMaxLdsBytes) c.slots /= 2;
        if ((uint64_t)c.block * c.slots * (c.unroll + extra) * 4u > kMaxLdsBytes) c.unroll /= 2;
    }
    if ((c.store == ST_PIPE || c.store == ST_PIPE_NT) && n >= (1ull << 26)) c.store = ST_LDS;   // 32-bit block offsets
    if (c.store == ST_PIPE || c.store == ST_PIPE_NT) {
        // two tiles (+ the exchange buffer) per wave must fit the LDS
        c.block = 64;
        if (c.unroll < 16) c.unroll = 16;
        if (c.unroll > 256) c.unroll = 256;
        if (c.exchange < XCH_BPERM || c.exchange > XCH_BPERM2) c.exchange = XCH_BPERM;
        const uint32_t extra = (has_exchange(h->variant) && c.exchange == XCH_LDS) ? 64u : 0u;
        if ((uint64_t)2 * 64 * c.unroll * 4u + extra * 4u > kMaxLdsBytes) c.unroll /= 2;
        if (!c.grid) c.grid = h->n_cu * 2u;
    }
    int rc = begin_timing(h, st);
    if (rc) return rc;
    HIP_TRY(launch_generate(a, (int)h->variant, (h->flags & CPRNG_F_V1_W32) != 0, c, st),
            "generate kernel launch");
    return end_timing(h, st);
}

}  // namespace cprng_impl

extern "C" {

int cprng_create(const uint64_t *seeds, uint32_t n_streams, uint32_t variant, cprng_t **out)
{
    if (!seeds) return set_error(CPRNG_E_INVAL, "seeds is NULL");
    cprng_params_t p;
    std::memset(&p, 0, sizeof p);
    p.struct_size = sizeof p;
    p.variant = variant;
    p.n_streams = n_streams;
    p.seed = seeds[0];
    p.device = -1;
    if (variant & CPRNG_F_SEED_PER_STREAM) p.seeds = seeds;
    return create_impl(&p, out);
}

int cprng_create_ex(const cprng_params_t *params, cprng_t **out) { return create_impl(params, out); }

void cprng_destroy(cprng_t *h)
{
    if (!h) return;
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    destroy_plans(h);
    if (h->d_state) (void)hipFree(h->d_state);
    if (h->d_state_next) (void)hipFree(h->d_state_next);
    if (h->d_counter) (void)hipFree(h->d_counter);
    destroy_req_slots(h);
    destroy_group_buffers(h);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

int cprng_generate(cprng_t *h, uint32_t *out, uint64_t n_per_stream, cprng_stream_t stream)
{
    if (!h) return set_error(CPRNG_E_INVAL, "NULL handle");
    if (n_per_stream == 0) return CPRNG_OK;
    if (!out) return set_error(CPRNG_E_INVAL, "out is NULL");
    if ((uintptr_t)out % 4u) return set_error(CPRNG_E_INVAL, "out must be 4-byte aligned");
    DeviceGuard g(h->device);
    if (!g.ok) return set_error(CPRNG_E_HIP, "hipSetDevice failed");
    const LaunchCfg c = resolve_cfg(h, n_per_stream, false);
    return generate_with(h, out, n_per_stream, (hipStream_t)stream, c);
}

int cprng_consume_qc(cprng_t *h, uint64_t *counts, uint64_t n_per_stream, cprng_stream_t stream)
{
    if (!h) return set_error(CPRNG_E_INVAL, "NULL handle");
    if (!counts) return set_error(CPRNG_E_INVAL, "counts is NULL");
    if (n_per_stream % 2u) return set_error(CPRNG_E_INVAL, "n_per_stream must be even (pairs)");
    if ((uintptr_t)counts % 8u) return set_error(CPRNG_E_INVAL, "counts must be 8-byte aligned");
    DeviceGuard g(h->device);
    if (!g.ok) return set_error(CPRNG_E_HIP, "hipSetDevice failed");
    GenArgs a;
    fill_args(h, a);
    a.counts = counts;
    a.n = n_per_stream;
    LaunchCfg c = resolve_cfg(h, n_per_stream, true);
    if (c.exchange == XCH_DPP && !dpp_pattern(h)) c.exchange = XCH_BPERM;
    int rc = begin_timing(h, (hipStream_t)stream);
    if (rc) return rc;
    HIP_TRY(launch_consume(a, (int)h->variant, (h->flags & CPRNG_F_V1_W32) != 0, c, (hipStream_t)stream),
            "consume kernel launch");
    return end_timing(h, (hipStream_t)stream);
}

int cprng_state_words(const cprng_t *h)
{
    if (!h) return set_error(CPRNG_E_INVAL, "NULL handle");
    return (int)h->words;
}

size_t cprng_state_bytes(const cprng_t *h)
{
    if (!h) return 0;
    return (size_t)h->ns * h->words * sizeof(uint32_t);
}

uint32_t cprng_n_streams(const cprng_t *h) { return h ? h->ns : 0u; }
uint32_t cprng_variant(const cprng_t *h) { return h ? (h->variant | h->flags) : 0u; }

int cprng_get_state(cprng_t *h, uint32_t *host_words, size_t n_words)
{
    if (!h || !host_words) return set_error(CPRNG_E_INVAL, "NULL argument");
    const uint64_t nw = (uint64_t)h->ns * h->words;
    if (n_words != nw) return set_error(CPRNG_E_INVAL, "n_words must be n_streams * state_words");
    DeviceGuard g(h->device);
    std::vector<uint32_t> soa(nw);
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    HIP_TRY(hipMemcpy(soa.data(), h->d_state, nw * sizeof(uint32_t), hipMemcpyDeviceToHost), "hipMemcpy state");
    for (uint64_t s = 0; s < h->ns; ++s)
        for (uint32_t k = 0; k < h->words; ++k) host_words[s * h->words + k] = soa[k * (uint64_t)h->ns + s];
    return CPRNG_OK;
}

int cprng_set_state(cprng_t *h, const uint32_t *host_words, size_t n_words)
{
    if (!h || !host_words) return set_error(CPRNG_E_INVAL, "NULL argument");
    const uint64_t nw = (uint64_t)h->ns * h->words;
    if (n_words != nw) return set_error(CPRNG_E_INVAL, "n_words must be n_streams * state_words");
    const bool w32 = (h->flags & CPRNG_F_V1_W32) != 0;
    for (uint64_t s = 0; s < h->ns; ++s) {
        const uint32_t *w = host_words + s * h->words;
        if (h->variant == CPRNG_V1_NAIVE3) {
            if ((w[0] | w[1]) == 0) return set_error(CPRNG_E_INVAL, "xorshift word is zero");
            uint32_t or2 = 0, or3 = 0;
            for (int k = 2; k < 10; ++k) or2 |= w[k];
            for (int k = 10; k < 20; ++k) or3 |= w[k];
            if (!or2 || !or3) return set_error(CPRNG_E_INVAL, "xor128 or xorwow words all zero");
            if (w32)
                for (int k = 1; k < 22; k += 2)
                    if (w[k]) return set_error(CPRNG_E_INVAL, "32-bit-word V1 state has a nonzero high half");
        } else if (h->variant == CPRNG_V3_BBS) {
            for (int k = 0; k < 8; ++k)
                if (w[k] >= 65536u) return set_error(CPRNG_E_INVAL, "BBS slot state must be below 2^16");
        } else if (h->variant == CPRNG_V4_XOR64) {
            if ((w[0] | w[1]) == 0) return set_error(CPRNG_E_INVAL, "xor64 word is zero");
        } else if ((w[0] | w[1] | w[2] | w[3]) == 0) {
            return set_error(CPRNG_E_INVAL, "xor128 words all zero");
        }
    }
    DeviceGuard g(h->device);
    std::vector<uint32_t> soa(nw);
    for (uint64_t s = 0; s < h->ns; ++s)
        for (uint32_t k = 0; k < h->words; ++k) soa[k * (uint64_t)h->ns + s] = host_words[s * h->words + k];
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    HIP_TRY(hipMemcpy(h->d_state, soa.data(), nw * sizeof(uint32_t), hipMemcpyHostToDevice), "hipMemcpy state");
    return CPRNG_OK;
}

int cprng_default_bbs_combs(uint32_t C, uint32_t *out)
{
    if (!out) return set_error(CPRNG_E_INVAL, "NULL argument");
    if (C < 4 || C > 64 || !is_pow2(C)) return set_error(CPRNG_E_INVAL, "C must be a power of two in [4, 64]");
    if (!default_bbs_combs(C, out)) return set_error(CPRNG_E_INVAL, "no arrangement arrays found");
    return CPRNG_OK;
}

int cprng_default_combs(uint32_t C, uint32_t *comb1, uint32_t *comb2)
{
    if (!comb1 || !comb2) return set_error(CPRNG_E_INVAL, "NULL argument");
    if (C < 3 || C > 64 || !is_pow2(C)) return set_error(CPRNG_E_INVAL, "C must be a power of two in [4, 64]");
    if (!default_combs(C, comb1, comb2)) return set_error(CPRNG_E_INVAL, "no combination arrays found");
    return CPRNG_OK;
}

int cprng_set_tuning(cprng_t *h, const cprng_tuning_t *t)
{
    if (!h || !t) return set_error(CPRNG_E_INVAL, "NULL argument");
    if (t->block && (t->block % 64 || t->block > 1024))
        return set_error(CPRNG_E_INVAL, "block must be a multiple of 64, <= 1024 (above 256: interleaved tiles)");
    if (t->unroll && t->unroll != 8 && t->unroll != 16 && t->unroll != 32 && t->unroll != 64 &&
        t->unroll != 128 && t->unroll != 256)
        return set_error(CPRNG_E_INVAL, "unroll must be 8, 16, 32, 64, 128 or 256 (above 32: LDS store modes)");
    if (t->store > 8) return set_error(CPRNG_E_INVAL, "store mode must be 0..8");
    if ((t->store == 5 || t->store == 6) && !(h->flags & CPRNG_F_INTERLEAVED))
        return set_error(CPRNG_E_INVAL, "store modes 5 and 6 apply to interleaved handles");
    if (t->chunk && (t->chunk % 64 || t->chunk > (1u << 24))) return set_error(CPRNG_E_INVAL, "chunk must be a multiple of 64, <= 2^24");
    if (t->waves_per_cu > 32) return set_error(CPRNG_E_INVAL, "waves_per_cu must be <= 32");
    if (t->streams_per_lane && t->streams_per_lane != 1 && t->streams_per_lane != 2 && t->streams_per_lane != 4)
        return set_error(CPRNG_E_INVAL, "streams_per_lane must be 1, 2 or 4");
    if (t->exchange > 4) return set_error(CPRNG_E_INVAL, "exchange must be 0..4");
    h->tuning = *t;
    return CPRNG_OK;
}

int cprng_get_tuning(const cprng_t *h, cprng_tuning_t *t)
{
    if (!h || !t) return set_error(CPRNG_E_INVAL, "NULL argument");
    *t = h->tuning;
    return CPRNG_OK;
}

static int tuning_source(const cprng_t *h, bool cached)
{
    const cprng_tuning_t &t = h->tuning;
    if (t.block || t.unroll || t.store || t.chunk || t.waves_per_cu || t.streams_per_lane || t.exchange) return 2;
    return cached ? 1 : 0;
}

int cprng_resolved_tuning(cprng_t *h, uint64_t n_per_stream, cprng_tuning_t *out, int *source)
{
    if (!h || !out) return set_error(CPRNG_E_INVAL, "NULL argument");
    const LaunchCfg c = resolve_cfg(h, n_per_stream, false);
    TuneEntry e;
    const bool cached = tune_cache_lookup(h, n_per_stream, &e);
    std::memset(out, 0, sizeof *out);
    out->block = c.block;
    out->unroll = c.unroll;
    out->store = c.store;
    out->streams_per_lane = c.slots;
    out->exchange = c.exchange;
    if (h->flags & CPRNG_F_INTERLEAVED)
        out->waves_per_cu = h->n_cu ? c.grid / h->n_cu : 0;
    else if (c.store == ST_PIPE || c.store == ST_PIPE_NT)
        out->waves_per_cu = h->n_cu ? c.grid / h->n_cu : 0;
    else
        out->waves_per_cu = h->tuning.waves_per_cu ? h->tuning.waves_per_cu : (cached ? e.waves : default_generate_entry(h).waves);
    if (source) *source = tuning_source(h, cached);
    return CPRNG_OK;
}

int cprng_enable_timing(cprng_t *h, int on)
{
    if (!h) return set_error(CPRNG_E_INVAL, "NULL handle");
    h->timing = on != 0;
    h->ev_pending = false;
    return CPRNG_OK;
}

double cprng_last_kernel_ms(cprng_t *h)
{
    if (!h || !h->ev_pending) return -1.0;
    DeviceGuard g(h->device);
    if (hipEventSynchronize(h->ev1) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev0, h->ev1) != hipSuccess) return -1.0;
    return (double)ms;
}

int cprng_probe_fill(uint32_t *dst, uint64_t n_words, uint32_t value, cprng_stream_t stream)
{
    if (!dst || (uintptr_t)dst % 16u) return set_error(CPRNG_E_INVAL, "dst must be 16-byte aligned");
    HIP_TRY(launch_fill(dst, n_words, value, (hipStream_t)stream), "fill kernel launch");
    return CPRNG_OK;
}

int cprng_probe_copy(uint32_t *dst, const uint32_t *src, uint64_t n_words, cprng_stream_t stream)
{
    if (!dst || !src || (uintptr_t)dst % 16u || (uintptr_t)src % 16u)
        return set_error(CPRNG_E_INVAL, "dst and src must be 16-byte aligned");
    HIP_TRY(launch_copy(dst, src, n_words, (hipStream_t)stream), "copy kernel launch");
    return CPRNG_OK;
}

int cprng_probe_valu(uint32_t kind, uint32_t *out, uint32_t n_threads, uint32_t iters, cprng_stream_t stream)
{
    if (!out || n_threads == 0 || n_threads % 256) return set_error(CPRNG_E_INVAL, "n_threads must be a positive multiple of 256");
    if (kind > 4)
        return set_error(CPRNG_E_INVAL, "kind must be 0 (xor), 1 (shift), 2 (f32 mul/add), 3 (64-bit shift) or 4 (64-bit add)");
    HIP_TRY(launch_valu_probe(kind, out, n_threads, iters, (hipStream_t)stream), "VALU probe launch");
    return CPRNG_OK;
}

const char *cprng_strerror(int status)
{
    switch (status) {
    case CPRNG_OK: return "ok";
    case CPRNG_E_INVAL: return "invalid argument";
    case CPRNG_E_NOMEM: return "out of memory";
    case CPRNG_E_HIP: return "HIP runtime error";
    case CPRNG_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *cprng_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
