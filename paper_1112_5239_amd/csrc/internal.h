// internal.h -- shared declarations between the host runtime and the gfx950
// kernels of the chaotic-iteration PRNG library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cprng.h"

namespace cprng_impl {

// LDS a gfx950 workgroup may allocate (the whole 160 KiB of a CU).
constexpr uint32_t kMaxLdsBytes = 160u * 1024u;

// Moduli of the eight BBS slots of Algorithm 5 (Section 9.1): products of two
// primes = 3 mod 4 near 256, each below 2^16 so a square of a state below
// 2^16 fits 32 bits.
constexpr uint32_t kBbsModuli[8] = {251u * 239u, 251u * 227u, 251u * 223u, 251u * 211u,
                                    239u * 227u, 239u * 223u, 239u * 211u, 227u * 223u};

// True for the variants that mix neighbours' words (group size C).
constexpr bool has_exchange(uint32_t variant)
{
    return variant == CPRNG_V2_SHMEM || variant == CPRNG_V3_BBS || variant == CPRNG_V4_XOR64;
}

// Store modes of the plain generate kernel.
enum StoreMode : int {
    ST_DIRECT = 1,        // each lane stores its own stream's 16-byte quads
    ST_LDS = 2,           // tile transposed through LDS, full lines per store
    ST_DIRECT_NT = 3,     // as ST_DIRECT with non-temporal stores
    ST_LDS_NT = 4,        // as ST_LDS with non-temporal stores
    ST_INTERLEAVED = 5,   // out[i * n_streams + s], one dword per lane
    ST_PIPE = 7,          // persistent waves, double-buffered LDS tiles, stores overlapped
    ST_PIPE_NT = 8,       // as ST_PIPE with non-temporal stores
    ST_ILV_TILE = 9,      // interleaved layout through a K x block LDS tile, 16-byte stores
    ST_ILV_TILE_NT = 10,  // as ST_ILV_TILE with non-temporal stores
    ST_ILV_QUAD = 11,     // interleaved layout, four consecutive streams per lane, direct 16-byte stores
    ST_ILV_QUAD_NT = 12   // as ST_ILV_QUAD with non-temporal stores
};

// Neighbour-exchange implementations of the V2 variant (tiled kernel).
enum ExchangeMode : int {
    XCH_BPERM = 1,        // two cross-lane reads (ds_bpermute) per step
    XCH_LDS = 2,          // per-wave LDS word buffer: one write, two reads per step
    XCH_BPERM2 = 3,       // two steps per round of eight cross-lane reads
    XCH_DPP = 4           // two DPP row rotations per step (one fixed pattern, groups of 16)
};

// The combination arrays the DPP exchange implements: within each row of 16
// lanes, stream j reads streams (j + 1) mod 16 and (j + 4) mod 16 (a DPP
// row_ror:r hands lane i the value of lane (i - r) mod 16 of its row).
constexpr uint32_t kDppGroup = 16, kDppOff1 = 1, kDppOff2 = 4;

// Kernel arguments of the plain generate / consume kernels.
struct GenArgs {
    uint32_t *state;       // SoA: word k of stream s at state[k * ns + s]
    uint32_t *out;         // outputs (generate)
    uint64_t *counts;      // hit counts (consume)
    uint64_t n;            // outputs per stream
    uint32_t ns;           // number of streams
    uint32_t group;        // V2/V3/V4 group size C (divides 64)
    uint32_t xs_b, xs_c;   // V1: right and second left shift of the first generator
    uint8_t comb1[64];     // V2/V4: comb1[j mod C]
    uint8_t comb2[64];
    uint8_t combs16[16][64];   // V3: arrangement array a, entry j mod C
};

// One chunk of a group's run (V2/V4 batched uneven runs): the group's C
// streams generate steps [start, start + len) from the state reached by the
// jump polynomial of row `row`; the last chunk writes the end states.
struct GroupItem {
    uint32_t group;
    uint32_t row;
    uint64_t start;
    uint64_t len;
    uint32_t last;
    uint32_t pad;
};

struct GroupJumpArgs {
    GenArgs g;                  // the call's start states, ns, group, arrays
    uint32_t *state_next;       // end states (groups with a last chunk)
    const GroupItem *items;
    uint32_t n_items;
    uint32_t row_words;         // 32-bit words per jump row
    uint32_t deg;               // degree of the group's minimal polynomial
    uint32_t round;             // words per lane per store round: 32, 64 or 128
    uint32_t wg_waves;          // waves per workgroup: 1 or 4
    const uint32_t *rows;       // row r: coefficients of X^(r * chunk) mod q
    uint32_t *out;
    const uint64_t *offsets;    // per stream
};

// One chunk of a V1 run: stream `stream` generates steps [start, start +
// len); `row` selects the jump polynomials of J = start (= row * chunk);
// items of a stream are consecutive, its chunk 0 at index `first`.
struct V1Item {
    uint32_t stream;
    uint32_t row;
    uint64_t start;
    uint64_t len;
    uint32_t last;
    uint32_t first;
};

struct V1ChunkArgs {
    GenArgs g;                  // the call's start states, ns, first generator's shifts
    uint32_t *state_next;       // end states (streams with a last chunk)
    const V1Item *items;
    uint32_t n_items;
    uint32_t row_words;         // 32-bit words per row: xorshift | xor128 | xorwow polynomials
    uint32_t deg1, deg2, deg3;  // degrees of the three minimal polynomials
    uint32_t off2, off3;        // word offsets of the xor128 and xorwow polynomials in a row
    const uint32_t *rows;
    uint32_t *agg;              // per chunk: xor of its strategy words, then (after the
                                // scan) the xor of those of the stream's earlier chunks
    uint32_t *out;
    const uint64_t *offsets;    // per stream
    uint64_t chunk;             // length of a full chunk
    uint32_t sum_row;           // row of sum_{i=1..chunk} X^i (xorshift and xor128 parts)
    uint32_t round;             // generating pass: words per lane per store round (32, 64, 128)
    uint32_t wg_waves;          // generating pass: waves per workgroup (1 or 4)
    const uint32_t *order;      // aggregate pass: the chunks that are not a stream's last
    uint32_t n_agg;             // entries of order
    uint32_t parts;             // aggregate pass: lanes per chunk (1, 2 or 4)
    const uint32_t *sub_rows;   // xorwow polynomials X^(row * chunk + p * chunk / parts), row-major
                                // by (row, p), w3 words each
    uint32_t w3;                // 32-bit words per xorwow polynomial
    const uint32_t *sfirst;     // per stream: index of its first chunk (n_streams + 1 entries)
};

struct LaunchCfg {
    uint32_t block;        // threads per block
    uint32_t unroll;       // outputs per lane per round
    uint32_t store;        // StoreMode
    uint32_t lds_bytes;    // LDS modes: dynamic LDS per block (>= the tile; more caps occupancy)
    uint32_t slots;        // LDS modes: streams per lane (1, 2 or 4)
    uint32_t exchange;     // V2, LDS modes: ExchangeMode
    uint32_t grid;         // ST_PIPE modes: persistent workgroups (0: one per 64 streams)
};

// variant: 0 V0, 1 V1 (w32 selects 32-bit words), 2 V2.
hipError_t launch_generate(const GenArgs &a, int variant, int w32, const LaunchCfg &c,
                           hipStream_t st);
hipError_t launch_consume(const GenArgs &a, int variant, int w32, const LaunchCfg &c,
                          hipStream_t st);

// Per-variant generate / consume launches, each variant's kernels in a
// source file of their own (gen_v0.hip .. gen_v3.hip).
hipError_t launch_generate_v0(const GenArgs &a, const LaunchCfg &c, hipStream_t st);
hipError_t launch_generate_v1(const GenArgs &a, bool w32, const LaunchCfg &c, hipStream_t st);
hipError_t launch_generate_v2(const GenArgs &a, const LaunchCfg &c, hipStream_t st);
hipError_t launch_generate_v3(const GenArgs &a, const LaunchCfg &c, hipStream_t st);
hipError_t launch_consume_v0(const GenArgs &a, const LaunchCfg &c, hipStream_t st);
hipError_t launch_consume_v1(const GenArgs &a, bool w32, const LaunchCfg &c, hipStream_t st);
hipError_t launch_consume_v2(const GenArgs &a, const LaunchCfg &c, hipStream_t st);
hipError_t launch_consume_v3(const GenArgs &a, const LaunchCfg &c, hipStream_t st);
hipError_t launch_generate_v4(const GenArgs &a, const LaunchCfg &c, hipStream_t st);
hipError_t launch_consume_v4(const GenArgs &a, const LaunchCfg &c, hipStream_t st);
// Chunks of V1 runs: aggregate pass, then generating pass (groupjump.cpp
// plans them); w32 selects 32-bit words.
hipError_t launch_v1_chunks(const V1ChunkArgs &a, bool w32, hipStream_t st);
// Chunks of V2/V4 group runs (groupjump.cpp plans them).
hipError_t launch_group_chunks(const GroupJumpArgs &a, int variant, hipStream_t st);
hipError_t launch_group_chunks_v2(const GroupJumpArgs &a, hipStream_t st);
hipError_t launch_group_chunks_v4(const GroupJumpArgs &a, hipStream_t st);

// A run of consecutive outputs of one stream (a batched stream or a request)
// for the chunked kernels.  The run is cut into chunks ("segments"):
// segment 0 covers positions [0, min(len, head + chunk)), segment k >= 1
// covers [head + k*chunk, min(len, head + (k+1)*chunk)); `head` (0..63) makes
// every segment after the first start on a 256-byte boundary.  Segment k >= 1
// starts from the stream's state jumped ahead by k*chunk (polynomial at table
// index k) and then stepped `head` times.
struct RunDesc {
    uint64_t out;          // device address of the run's first output
    uint64_t len;          // outputs in the run (> 0)
    uint32_t stream;       // stream id
    uint32_t head;         // 0..63: outputs before the run's first 256-byte boundary
    uint32_t first_seg;    // global index of the run's segment 0
    uint32_t last;         // 1: the run ends the stream's work of this launch
};

struct SegArgs {
    const RunDesc *runs;   // sorted by first_seg
    uint32_t nrun;
    uint32_t nseg;         // total segments
    uint32_t chunk;        // outputs per segment (multiple of 64)
    uint32_t kcap;         // jump table entries (distances k * chunk, k < kcap)
    const uint32_t *polys; // kcap polynomials X^(k*chunk) mod q, 5 words each, bit i = coeff of X^i
    uint32_t ns;           // streams (SoA stride)
    const uint32_t *state; // current states (read only during the launch)
    uint32_t *state_next;  // end states of runs with `last`
    uint32_t *counter;     // work-queue counters, one per XCD (8 words, reset before each launch)
    uint32_t unroll;       // outputs per lane per round
    uint32_t persistent;   // 1: waves take grabs from the queues; 0: one grab per wave, by workgroup id
    // Device-planned launches (stream subsets): when set, the segment count
    // is read from *nseg_dev at kernel start instead of nseg.
    const uint32_t *nseg_dev;
    // Two-level jump table: when set, segment k jumps by (k mod 2^lo_bits) *
    // chunk with polys and by (k >> lo_bits) * 2^lo_bits * chunk with
    // polys_hi (the two maps commute), so k is bounded by 2^(2 lo_bits)
    // whatever the run lengths.
    const uint32_t *polys_hi;
    uint32_t lo_bits;
};

// Request batches small enough to travel in the kernel arguments: up to
// kInlineRuns runs and commit ids, read by the kernels through their
// kernel-argument segment, so no descriptor upload precedes the launch.
constexpr uint32_t kInlineRuns = 64;
struct SegInline {
    SegArgs a;                    // a.runs is ignored: the kernels use runs[]
    RunDesc runs[kInlineRuns];
    uint32_t ids[kInlineRuns];    // streams whose end states the commit copies back
    uint32_t n_ids;
};
// Tiled segment kernel (store ST_LDS / ST_LDS_NT, persistent) on an inline batch.
hipError_t launch_segments_inline(const SegInline &si, uint32_t grid, uint32_t store, hipStream_t st);
// Commit of an inline batch; also clears its 8 work-queue counters (si.a.counter).
hipError_t launch_commit_inline(const SegInline &si, uint32_t *state, hipStream_t st);

// Stream subsets described in device memory (cprng_generate_subset).
constexpr uint64_t kSubsetMaxLen = 1ull << 37;   // outputs per descriptor
constexpr uint32_t kSubsetLoBits = 13;           // jump table: 2 x 2^13 rows
constexpr uint32_t kSubsetMinChunk = 2048;       // (2^37 / 2048 = 2^26 segments per run)

// Per-call control block of a subset launch, in device memory.
struct SubsetCtl {
    unsigned long long epoch;  // this call's stream mark (unique per slot and call)
    uint32_t err;              // set when a descriptor is invalid
    uint32_t nseg;             // segments of the call (0 after an error)
    int32_t status;            // 0 or CPRNG_E_INVAL
    uint32_t pad[3];
    uint32_t counter[8];       // work-queue counters of the segment kernel
};

struct SubsetArgs {
    const uint32_t *ids;       // count stream ids (device)
    const uint64_t *lens;      // count lengths (device)
    const uint64_t *offs;      // count output offsets in uint32 elements (device)
    uint32_t count;
    uint32_t ns;
    uint32_t chunk;
    uint32_t nblocks;          // blocks of 256 descriptors
    uint64_t out_base;         // device address of the output base
    unsigned long long *mark;  // ns entries: the epoch of the last call that listed the stream
    SubsetCtl *ctl;
    uint32_t *segs;            // count: segments per descriptor
    unsigned long long *bsum;  // nblocks: segments per block, then their exclusive prefix
    RunDesc *runs;             // count run descriptors
    int32_t *status;           // caller's status word (device) or nullptr
};

// Plan a subset call on the device (check, count, scan, run list), then the
// segment kernel with a.nseg_dev / a.counter pointing into sa.ctl, then the
// commit of the listed streams' end states (skipped after an error).
hipError_t launch_subset(const SubsetArgs &sa, const SegArgs &a, uint32_t grid, uint32_t block, uint32_t store,
                         uint32_t *state, hipStream_t st);

// lds_min: dynamic LDS per workgroup at least this (caps residency).
hipError_t launch_segments(const SegArgs &a, uint32_t grid, uint32_t block, uint32_t store, uint32_t lds_min,
                           hipStream_t st);
// state[k * ns + ids[i]] = state_next[k * ns + ids[i]] for k < 5; with
// reset_counters, also clears those 8 work-queue counters for the next launch.
hipError_t launch_commit(uint32_t *state, const uint32_t *state_next, const uint32_t *ids,
                         uint32_t count, uint32_t ns, hipStream_t st, uint32_t *reset_counters = nullptr);
hipError_t launch_zero_u32(uint32_t *p, uint32_t count, hipStream_t st);

hipError_t launch_fill(uint32_t *dst, uint64_t n_words, uint32_t value, hipStream_t st);
hipError_t launch_valu_probe(uint32_t kind, uint32_t *out, uint32_t n_threads, uint32_t iters, hipStream_t st);
hipError_t launch_copy(uint32_t *dst, const uint32_t *src, uint64_t n_words, hipStream_t st);

}  // namespace cprng_impl
