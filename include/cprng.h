/*
 * cprng.h -- C ABI of the MI355X (gfx950) chaotic-iteration PRNG library.
 *
 * The library generates, for many independent streams at once, the
 * pseudorandom numbers of the chaotic-iteration generator of Bahi, Couturier,
 * Guyeux and Heam (arXiv 1112.5239): each stream keeps a 32-bit state x and
 * applies x <- x xor S for a strategy word S drawn from Marsaglia xor-like
 * generators (Section 4.2, Eq. "Oplus"; Section 5; Section 6).
 *
 * Conventions for every entry point:
 *  - Return value: CPRNG_OK (0) or a negative cprng_status.  Nothing throws
 *    across this boundary.  cprng_last_error() gives a human-readable detail
 *    of the last failure on the calling thread.
 *  - Pointers documented "device" are HIP device addresses (for example a
 *    torch tensor's data_ptr()); "host" pointers are ordinary host memory.
 *    The caller owns every buffer it passes; the handle owns only its own
 *    device state and work lists.
 *  - Calls that take a stream are asynchronous on that HIP stream (NULL = the
 *    null stream).  A handle's state advances in stream order; calls on one
 *    handle must be ordered on one stream and a handle is not thread-safe.
 *  - Outputs are 32-bit unsigned integers.  Unless CPRNG_F_INTERLEAVED is
 *    set, output i of stream s of one call is out[s * n_per_stream + i].
 *  - Successive calls continue the streams: two calls of a and b outputs give
 *    the same numbers as one call of a + b.
 */
#ifndef CPRNG_H
#define CPRNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t is a pointer to this opaque type in the HIP runtime. */
typedef struct ihipStream_t *cprng_stream_t;

typedef struct cprng cprng_t;

/* Variant in the low byte of `variant`, flags above it. */
enum cprng_variant {
    /* Eq. (Oplus) with one xor128 (32-bit words) as the strategy (Section 5,
     * first idea; the construction X of Section 8).  5 state words/stream. */
    CPRNG_V0_PLAIN = 0,
    /* Listing 1 / Algorithm 3 (Section 6.1): xorshift(13,17,5), xor128 and
     * xorwow on 64-bit words; S is the xor of their six 32-bit halves.
     * 23 state words/stream. */
    CPRNG_V1_NAIVE3 = 1,
    /* Algorithm 4 (Section 6.2): one xor128 per stream mixed with the previous
     * words of two other streams of its group of C streams, chosen by two
     * combination arrays.  6 state words/stream.  Needs n_streams % C == 0. */
    CPRNG_V2_SHMEM = 2,
    /* Algorithm 5 (Section 9.1): the strategy word is assembled from eight
     * Blum-Blum-Shub generators x <- x^2 mod M (M = p*q < 2^16, p, q prime and
     * 3 mod 4; four bits from each, then two shifts of 0..3 bits filled from
     * second outputs of BBS1 and BBS2) and mixed as in Algorithm 4 with two
     * streams of the group chosen, once per call, from 16 arrangement arrays
     * by the low three bits of BBS1's and BBS2's states; at the end of a call
     * with outputs the eight BBS states rotate (slot k to k+1, 8 to 1).
     * 10 state words/stream: BBS slots 1..8 (each < 2^16), x, previous word.
     * Needs n_streams % C == 0.  Library arrangement arrays only. */
    CPRNG_V3_BBS = 3,
    /* Algorithm 4 with Marsaglia's xor64 as each stream's generator (the
     * generator Section 7 names for its optimized versions): 64-bit word y,
     * y ^= y << 13, y ^= y >> 7, y ^= y << 17; the stream's word is the xor of
     * y's two 32-bit halves, mixed with two streams of its group as in V2.
     * 4 state words/stream: y (low, high), x, previous word.  Needs
     * n_streams % C == 0; combination arrays as for V2. */
    CPRNG_V4_XOR64 = 4
};

enum cprng_flags {
    /* Output i of stream s goes to out[i * n_streams + s]. */
    CPRNG_F_INTERLEAVED = 1u << 8,
    /* V1 only: the three generators use 32-bit words (high halves are 0). */
    CPRNG_F_V1_W32 = 1u << 9,
    /* Seeds hold n_streams entries: stream s's SplitMix64 counter starts at
     * seeds[s] (the single-seed rule is the case seeds[s] = sigma*2^32 + s). */
    CPRNG_F_SEED_PER_STREAM = 1u << 10,
    /* V1 only, 64-bit words: Listing 1's first generator is xor64 (triple
     * 13, 7, 17) instead of Algorithm 2's triple (13, 17, 5) on the 64-bit
     * word.  Same state layout and seeding. */
    CPRNG_F_V1_XOR64 = 1u << 11
};

enum cprng_status {
    CPRNG_OK = 0,
    CPRNG_E_INVAL = -1,        /* bad argument (NULL pointer, size, variant) */
    CPRNG_E_NOMEM = -2,        /* device or host allocation failed */
    CPRNG_E_HIP = -3,          /* a HIP runtime call or launch failed */
    CPRNG_E_UNSUPPORTED = -4   /* valid request that this build does not do */
};

/* Parameters of cprng_create_ex().  Zero-initialise, then set fields. */
typedef struct cprng_params {
    uint32_t struct_size;      /* sizeof(cprng_params_t) */
    uint32_t variant;          /* cprng_variant | cprng_flags */
    uint32_t n_streams;        /* >= 1 */
    uint32_t group;            /* V2/V3 group size C; 0 = 32.  A power of two in [4, 64]. */
    uint64_t seed;             /* base seed sigma */
    const uint32_t *comb1;     /* host, `group` entries in [0,C); NULL = default */
    const uint32_t *comb2;     /* host, `group` entries in [0,C); NULL = default */
    int32_t device;            /* HIP device ordinal; -1 = current device */
    uint32_t reserved;
    const uint64_t *seeds;     /* host, n_streams entries with CPRNG_F_SEED_PER_STREAM
                                  (seed is then ignored); NULL otherwise */
} cprng_params_t;

/* ------------------------------------------------------------------------ */
/* Lifecycle.                                                                */
/* ------------------------------------------------------------------------ */

/* Create a generator of n_streams streams on the current HIP device.
 * seeds: host, one uint64 base seed sigma (n_streams seeds with
 * CPRNG_F_SEED_PER_STREAM in variant).  Stream s is initialised from
 * SplitMix64 draws whose counter starts at sigma*2^32 + s (the paper seeds
 * per-thread parameters on the host with ISAAC, Section 6.1); generator
 * words that would all be zero are redrawn.  V2 uses group size 32 and the
 * library's default combination arrays.  The state lives in device memory
 * owned by the handle.  Errors: E_INVAL (NULL, n_streams == 0, unknown
 * variant, V2 with n_streams % 32 != 0), E_NOMEM, E_HIP. */
int cprng_create(const uint64_t *seeds, uint32_t n_streams, uint32_t variant, cprng_t **out);

/* As cprng_create with explicit group size, combination arrays and device.
 * Combination arrays follow Algorithm 4: stream j of a group mixes the
 * previous words of streams comb1[j mod C] and comb2[j mod C] of its group. */
int cprng_create_ex(const cprng_params_t *params, cprng_t **out);

/* Wait for the handle's pending work, free its device memory and the handle.
 * NULL is a no-op. */
void cprng_destroy(cprng_t *h);

/* ------------------------------------------------------------------------ */
/* Hot path.                                                                 */
/* ------------------------------------------------------------------------ */

/* Generate n_per_stream outputs for every stream into out (device,
 * n_streams * n_per_stream uint32, 4-byte aligned).  In the stream-major
 * layout, rows that start off 128-byte lines (n_per_stream % 32 != 0 or a
 * base not 128-byte aligned) are stored in line-aligned pieces through LDS
 * tiles whatever the store mode asked.  Each output is the new
 * state x after one chaotic iteration x <- x xor S (Section 4.2), with S as
 * the variant defines it; the state is written back at the end, as the GPU
 * kernels of Section 6 do.  n_per_stream == 0 is a no-op.
 * Errors: E_INVAL, E_HIP. */
int cprng_generate(cprng_t *h, uint32_t *out, uint64_t n_per_stream, cprng_stream_t stream);

/* In-kernel consumption (numbers used directly after generation, as in the
 * storage-free runs of Section 7): advance every stream by n_per_stream
 * outputs without storing them.  Outputs 2k and 2k+1 of a stream form a pair
 * (r1, r2) mapped to binary32 u = (r1 >> 8) * 2^-24, v = (r2 >> 8) * 2^-24;
 * the pair is a hit iff fl(fl(u*u) + fl(v*v)) < 1 (round to nearest even, no
 * fused multiply-add).  counts (device, n_streams uint64) receives each
 * stream's hit count for this call (overwritten).  n_per_stream must be even.
 * Errors: E_INVAL, E_HIP. */
int cprng_consume_qc(cprng_t *h, uint64_t *counts, uint64_t n_per_stream, cprng_stream_t stream);

/* Batched uneven streams (V0, V1, and the exchange variants V2 and V4).  Stream
 * s writes its next lengths[s] outputs to out[offsets[s] .. offsets[s] +
 * lengths[s]) (device, 4-byte aligned, no other alignment needed); offsets
 * == NULL means the exclusive prefix sum of lengths.  lengths/offsets: host,
 * n_streams entries each.  Long streams are split into chunks that start
 * from a jumped-ahead state: the strategy generator and the x chain are
 * linear over GF(2), so the state after J steps is a polynomial in the
 * one-step map (x^J modulo the minimal polynomial), and the x chain is the
 * prefix-xor of the strategy words (construction X of Section 8).
 * V0: one hipGraph launch of a persistent kernel; the graph is built on the
 * first call with a given (lengths, offsets, out) and replayed afterwards.
 * V2/V4: the C streams of a group advance together (Algorithm 4), so lengths
 * must be equal within each group; the jump is taken by the whole group (its
 * one-step map on all C states is linear; its minimal polynomial is found
 * once per handle); chunk length from tuning.chunk (0 = automatic); the call
 * waits for earlier work on `stream` before reusing its buffers and then
 * launches a state copy, the chunk kernel and the commit.
 * V1: the three generators jump by their own polynomials (xorwow's Weyl
 * counter by J * 362437); x does not (xorwow's d + v is not linear), so an
 * aggregate pass xors each chunk's strategy words and each chunk starts from
 * x_0 xor the aggregates of the chunks before it; same buffers, copies and
 * waits as V2/V4.  Results equal those of each stream (V0, V1) or group
 * (V2/V4) generated alone.  Errors: E_INVAL (unequal lengths within a group),
 * E_UNSUPPORTED (V3, interleaved flag), E_NOMEM, E_HIP. */
int cprng_generate_ragged(cprng_t *h, uint32_t *out, const uint64_t *lengths,
                          const uint64_t *offsets, cprng_stream_t stream);

/* Bytes of the per-GPU device array cprng_generate_ragged_noalloc works in. */
#define CPRNG_NOALLOC_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): cprng_generate_ragged
 * on a V0 handle, with the same arguments and the same results, allocating no
 * device memory.  The work buffers of its kernels -- 8 queue counters, the run
 * descriptors (32 bytes per stream with a nonzero length), the commit list (4
 * bytes per such stream), the jump table (20 bytes per row; rows = the
 * smallest power of two, at least 64, above the longest run's chunk count)
 * and the end states (20 bytes per stream of the handle), each rounded up to
 * 256 bytes after 256 bytes of counters -- live in one file-scope device array
 * of CPRNG_NOALLOC_SCRATCH_BYTES (16 MiB) per GPU, held until the process
 * ends.  The call plans on the host, copies the descriptors into the array in
 * order on `stream`, resets the counters with a kernel and launches the chunk
 * and commit kernels directly (no graph).  The array keeps the last call's
 * contents, so calls that overlap on one GPU (any handles, on different
 * streams or threads) race on it: order them on one stream.  Errors: as
 * cprng_generate_ragged; E_UNSUPPORTED for handles other than V0; E_INVAL
 * when the buffers would exceed the array (the detail gives the sizes). */
int cprng_generate_ragged_noalloc(cprng_t *h, uint32_t *out, const uint64_t *lengths,
                                  const uint64_t *offsets, cprng_stream_t stream);

/* Host-only self-test of the jump-ahead used by cprng_generate_ragged (no
 * device work, no handle).  variant: CPRNG_V2_SHMEM or CPRNG_V4_XOR64 (a
 * group of C streams, comb1/comb2 host arrays of C entries or NULL for the
 * library's defaults) or CPRNG_V1_NAIVE3 with its flags (C, comb1, comb2
 * unused).  Finds the minimal polynomials as a handle would, then checks on
 * random states that the jump polynomial X^J mod q reproduces J steps of the
 * map (for V1 also the closed-form sum of the first J outputs).  Returns
 * CPRNG_OK, E_INVAL for bad arguments, E_HIP when a check fails. */
int cprng_jump_selftest(uint32_t variant, uint32_t C, const uint32_t *comb1, const uint32_t *comb2,
                        uint64_t J);

/* One request of cprng_generate_requests(). */
typedef struct cprng_request {
    uint32_t stream;           /* stream id < n_streams */
    uint32_t reserved;
    uint64_t length;           /* outputs to produce (0 allowed) */
    uint32_t *out;             /* device, 4-byte aligned, `length` uint32 */
} cprng_request_t;

/* Serve a batch of requests (V0 and V1): request r receives the next
 * `length` outputs of its stream; several requests of one stream are served
 * in array order, one after the other.  Streams without a request keep their
 * state.  reqs: host, count entries.  Same chunking and jump-ahead as
 * cprng_generate_ragged: V0 in one kernel launch per call; V1 as one batched
 * uneven call per round, round j serving the j-th request of every stream
 * (so it waits for earlier work on `stream` like that call).  Errors:
 * E_INVAL, E_UNSUPPORTED (V2, V3, V4: their streams advance by groups),
 * E_NOMEM, E_HIP. */
int cprng_generate_requests(cprng_t *h, const cprng_request_t *reqs, uint32_t count,
                            cprng_stream_t stream);

/* Serve a subset of the streams described in device memory (V0): descriptor
 * k makes stream ids[k] write its next lens[k] outputs to out_base +
 * out_offsets[k] (offsets in uint32 elements); streams not listed keep their
 * state.  This is the per-thread generation of Algorithms 3 and 4 restricted
 * to the listed streams, each with its own length, and it equals generating
 * each listed stream alone.  ids (uint32), lens and out_offsets (uint64):
 * device, count entries each, written by the caller's own kernels if it
 * likes -- the host never reads them.  The descriptors are checked, counted
 * and cut into chunks on the device (the same jumped-ahead chunks as
 * cprng_generate_ragged, from a two-level jump table), so the call does no
 * host round trip and, once a call of at least `count` descriptors has been
 * made on `stream`, allocates nothing (it can then be captured in a hipGraph
 * and replayed with new descriptor contents).  Lengths are at most 2^37; ids
 * must be distinct within a call.  status: optional device int32 that
 * receives, in stream order, 0 or CPRNG_E_INVAL when a descriptor is
 * invalid (id >= n_streams, repeated id, length > 2^37); an invalid call
 * writes no output and changes no state.  A call with count 0 does nothing
 * and leaves status untouched.  Calls on different HIP streams
 * must list disjoint streams.  ids, lens and out_offsets must stay valid
 * until the call has run.  Chunk length: tuning.chunk (at least 2048), else
 * 2048.  Errors (host side): E_INVAL (NULL or misaligned pointers, count >
 * n_streams, chunk below 2048), E_UNSUPPORTED (V1 .. V4), E_NOMEM, E_HIP. */
int cprng_generate_subset(cprng_t *h, const uint32_t *ids, const uint64_t *lens,
                          const uint64_t *out_offsets, uint32_t count, uint32_t *out_base,
                          int32_t *status, cprng_stream_t stream);

/* ------------------------------------------------------------------------ */
/* State (checkpoint / resume).                                              */
/* ------------------------------------------------------------------------ */

/* 32-bit words of state per stream: V0 5 {x128 x,y,z,w, x}, V2 6 {x128
 * x,y,z,w, x, previous mixed word}, V1 23 {xorshift lo,hi; xor128 x,y,z,w
 * as lo,hi; xorwow x,y,z,w,v,d as lo,hi; x}, V3 10 {BBS slots 1..8, x,
 * previous mixed word}, V4 4 {xor64 lo,hi, x, previous mixed word}.
 * Returns < 0 on a bad handle. */
int cprng_state_words(const cprng_t *h);

/* Bytes of all stream states (n_streams * state_words * 4); 0 on a bad
 * handle. */
size_t cprng_state_bytes(const cprng_t *h);

/* Copy all states to / from host memory, stream after stream, each stream's
 * words in the order above (host, n_streams * state_words uint32).  These
 * calls synchronise the device.  set_state rejects generator words that are
 * all zero (E_INVAL).  Errors: E_INVAL, E_HIP. */
int cprng_get_state(cprng_t *h, uint32_t *host_words, size_t n_words);
int cprng_set_state(cprng_t *h, const uint32_t *host_words, size_t n_words);

/* Versioned checkpoint images.  The kernels write every stream's state back
 * at the end of a call (the internal variables stored after the loop of
 * Algorithms 3 and 4), so the device state between calls is a complete
 * checkpoint.  An image is a 256-byte header -- magic "CPRNGCKP", format
 * version 1, header size, the handle's variant and flags, n_streams, state
 * words per stream, group size, the combination arrays (V2/V4), payload size,
 * a 64-bit FNV-1a hash of the payload and one of the header -- followed by the
 * states in cprng_get_state's order; integers little-endian.
 * cprng_checkpoint_bytes: the image size for h (0 on a bad handle).
 * cprng_checkpoint_save: write h's image to host_buf (host, exactly that many
 * bytes; synchronises the device like cprng_get_state).
 * cprng_checkpoint_load: restore an image saved from a handle of the same
 * variant, flags, stream count, group size and arrays (the seed may differ);
 * every header field, both hashes and the state rules of cprng_set_state are
 * checked first, and a failing check leaves h unchanged.  Errors: E_INVAL
 * (NULL, wrong size, bad magic, version, hash or a field that does not match
 * h), E_HIP. */
size_t cprng_checkpoint_bytes(const cprng_t *h);
int cprng_checkpoint_save(cprng_t *h, void *host_buf, size_t bytes);
int cprng_checkpoint_load(cprng_t *h, const void *host_buf, size_t bytes);

/* ------------------------------------------------------------------------ */
/* Introspection and tuning.                                                 */
/* ------------------------------------------------------------------------ */

uint32_t cprng_n_streams(const cprng_t *h);
uint32_t cprng_variant(const cprng_t *h);

/* Library's default V2 combination arrays for group size C (3 <= C <= 64,
 * C dividing 64): two permutations of [0,C) with comb1[j] != j,
 * comb2[j] != j and comb1[j] != comb2[j].  comb1/comb2: host, C entries. */
int cprng_default_combs(uint32_t C, uint32_t *comb1, uint32_t *comb2);

/* The library's 16 arrangement arrays of the BBS variant for group size C (a
 * power of two in [4, 64]): permutations of [0,C) without fixed points; array
 * a at out[a*C .. a*C+C-1] (host, 16*C entries).  Errors: E_INVAL. */
int cprng_default_bbs_combs(uint32_t C, uint32_t *out);

/* Kernel configuration used by the hot-path entry points.  Zero fields mean
 * "autotuned / default".  store: 0 auto, 1 per-lane direct, 2 LDS-transposed,
 * 3 direct non-temporal, 4 LDS-transposed non-temporal, 7 persistent
 * pipelined (waves_per_cu one-wave workgroups per CU take 64-stream blocks in
 * address order; two LDS tiles so each round's stores overlap the next
 * round's generation), 8 as 7 with non-temporal stores.  Handles created with
 * CPRNG_F_INTERLEAVED take 0/2/7 (LDS tiles of unroll steps x block streams,
 * each step's block stored as one contiguous run; needs n_streams % 4 == 0 and
 * a 16-byte aligned output, else the per-lane path runs), 4/8 (the same,
 * non-temporal), 1/3 (per-lane dword stores) or 5/6 (V0, V2, V4: four
 * consecutive streams per lane, whose words of each step are stored as one
 * 16-byte store with no LDS tile; 6 non-temporal; block = 64, 128 or 256
 * threads per tile of 4 x block streams; V1 and V3 take the tiles instead;
 * other handles reject 5/6).  The chunk kernels of
 * cprng_generate_ragged / cprng_generate_requests take 1 (per-lane), 2/4
 * (LDS tiles, persistent waves fed by one work queue per XCD) or 7/8 (LDS
 * tiles, one workgroup per 64 chunks banded over the XCDs; waves_per_cu then
 * caps residency, 0 = none). */
typedef struct cprng_tuning {
    uint32_t block;            /* threads per block: 64, 128, 192 or 256; the interleaved
                                  layout's tiles take 256, 512 or 1024 (streams per tile);
                                  batched runs of V1, V2 and V4 (chunk kernels): 64 or
                                  256 (the default; the V2/V4 kernel takes 64 with
                                  unroll 128) */
    uint32_t unroll;           /* outputs per stream per round: 8, 16, 32 (direct);
                                  16..256, powers of two (LDS-transposed; chunk
                                  kernels 32..256); 16..128 (pipelined); the
                                  V3 (BBS) kernels are built for 8..32 only and
                                  larger values are lowered to 32; batched runs of
                                  V1, V2 and V4: words per store round = the output's
                                  aligned lines those rounds store, 32, 64 or 128
                                  (defaults: V1 64, V2/V4 32) */
    uint32_t store;            /* store mode, see above */
    uint32_t chunk;            /* ragged/requests: outputs per chunk (multiple of 64) */
    uint32_t waves_per_cu;     /* ragged/requests (store 1/2/4) and pipelined generate:
                                  persistent waves per CU (0 = default); LDS-transposed
                                  generate and ragged store 7/8: residency cap (0 = none);
                                  interleaved tiles: persistent workgroups per CU, each
                                  taking tiles of its XCD's band in turn (0 = one
                                  workgroup per tile, the default) */
    uint32_t streams_per_lane; /* LDS-transposed generate: 1, 2 or 4 streams per lane;
                                  batched V1 runs: lanes per chunk of the aggregate
                                  pass, 1, 2 (the default) or 4;
                                  interleaved tiles: 2 = two tile buffers, so each
                                  round's stores overlap the next round's steps */
    uint32_t exchange;         /* V2/V3/V4 tile kernels (stream-major, pipelined,
                                  interleaved) and consumption: 1 cross-lane reads,
                                  2 LDS word buffer, 3 two steps per read round
                                  (V2 only), 4 DPP row rotations.  4 applies to
                                  V2/V4 handles created with group 16,
                                  comb1[j] = (j + 1) % 16 and
                                  comb2[j] = (j + 4) % 16 (the pattern two DPP
                                  rotations of a 16-lane row implement; tile
                                  kernels and consumption only); other handles
                                  and kernels use 1.  Every choice gives the same
                                  words. */
    uint32_t reserved;
} cprng_tuning_t;

int cprng_set_tuning(cprng_t *h, const cprng_tuning_t *t);
int cprng_get_tuning(const cprng_t *h, cprng_tuning_t *t);

/* Autotuner (the batched-launch configurations of the hot path, Sections 6
 * and 7 give none for this hardware).  Times each candidate configuration of
 * cprng_generate for n_per_stream on this handle with HIP events on `stream`
 * (median of three launches after a warm-up), keeps the fastest in a
 * process-wide table keyed by device architecture, variant, word-width flags,
 * layout and the power-of-two classes of n_streams and n_per_stream, and
 * rewrites the JSON cache file named by $CPRNG_TUNE_CACHE if set (read once
 * per process, at the first lookup).  Later calls of any handle of the same
 * class use the entry unless cprng_set_tuning overrides it.  Candidates:
 * stream-major -- per-lane stores and LDS tiles of several widths, streams
 * per lane, residency caps, exchange implementations; interleaved -- LDS
 * tiles of 256/512/1024 streams x 8/16/32 steps, one or two tile buffers,
 * exchange through cross-lane reads or the LDS word buffer, one workgroup per
 * tile or 1/2 persistent workgroups per CU, and (V0, V2, V4) the
 * four-streams-per-lane kernel.  The stream states are copied aside before
 * tuning and put back after it, so the call leaves the streams where they
 * were; scratch (device, 16-byte aligned, n_streams * n_per_stream words) is
 * overwritten.  Synchronises `stream`.  Errors: E_INVAL (NULL, misaligned,
 * stream-major n % 4 != 0, interleaved n_streams % 4 != 0), E_NOMEM, E_HIP. */
int cprng_autotune(cprng_t *h, uint32_t *scratch, uint64_t n_per_stream, cprng_stream_t stream);

/* Same for cprng_generate_ragged with the given lengths and offsets (keyed by
 * variant, flags and the classes of n_streams, total and longest length).
 * V0: chunk length, store mode and round, persistent waves per CU.  V1, V2,
 * V4: store round (32/64/128 words), workgroup shape (1 or 4 waves), chunk
 * length (automatic, half or twice the automatic one) and (V1) lanes per
 * chunk of the aggregate pass.  States are restored as above; `out` is
 * overwritten.  Errors as cprng_generate_ragged. */
int cprng_autotune_ragged(cprng_t *h, uint32_t *out, const uint64_t *lengths,
                          const uint64_t *offsets, cprng_stream_t stream);

/* The launch configuration the next cprng_generate of n_per_stream would use
 * on this handle, before the per-call adjustments to alignment and LDS size
 * (fields as cprng_tuning_t; store holds the internal mode: 9/10 interleaved
 * tiles (10 non-temporal), 11/12 four streams per lane; waves_per_cu of the
 * interleaved layout = persistent workgroups per CU).  *source (may be NULL):
 * 0 defaults, 1 the autotuner's entry for this shape class, 2 cprng_set_tuning.
 * No device work.  Errors: E_INVAL. */
int cprng_resolved_tuning(cprng_t *h, uint64_t n_per_stream, cprng_tuning_t *out, int *source);

/* Same for cprng_generate_ragged with these lengths: V0 chunk, unroll,
 * waves_per_cu, block, store; V1/V2/V4 chunk (the automatic length resolved),
 * unroll = store round, block = 64 * waves per workgroup, streams_per_lane =
 * V1's aggregate lanes per chunk.  May compute the group's jump polynomial on
 * the host.  Errors: E_INVAL, E_UNSUPPORTED (BBS, interleaved handles). */
int cprng_resolved_tuning_ragged(cprng_t *h, const uint64_t *lengths, cprng_tuning_t *out, int *source);

/* Average device time in milliseconds of the last kernel launched by the
 * most recent hot-path call on this handle, when timing is enabled with
 * cprng_enable_timing(h, 1) (events recorded on the call's stream around the
 * kernel).  Returns < 0 if unavailable. */
int cprng_enable_timing(cprng_t *h, int on);
double cprng_last_kernel_ms(cprng_t *h);

/* ------------------------------------------------------------------------ */
/* Serving loop (continuous batching over a V0 handle's resident streams).   */
/*                                                                           */
/* Each client is one stream of the handle, whose state stays in device      */
/* memory.  A request (client, length) receives that client's next `length`  */
/* outputs, in the order the client's requests were submitted.  Results live */
/* in a device arena of `budget_bytes` owned by the server: a request is     */
/* admitted when its result fits in the free part of the arena (and the      */
/* client has no request on the GPU), and its memory returns to the budget   */
/* when the caller releases the result.  Admitted requests are launched in   */
/* batches (cprng_generate_requests) on up to `n_gpu_streams` HIP streams,   */
/* so a batch can start while earlier ones still run; a client appears in at */
/* most one batch in flight.  Results are identical whatever the mix of      */
/* requests they were served with.  Not thread-safe: one thread drives it.   */
/* ------------------------------------------------------------------------ */
typedef struct cprng_server cprng_server_t;

typedef struct cprng_server_params {
    uint32_t struct_size;      /* sizeof(cprng_server_params_t) */
    uint32_t n_gpu_streams;    /* concurrent batches (HIP streams, 1..16); 0 = 2 */
    uint64_t budget_bytes;     /* result arena = admission budget; 0 = 64 GiB */
    uint32_t max_batch;        /* requests per batch; 0 = 1024 */
    uint32_t reserved;
} cprng_server_params_t;

typedef struct cprng_completion {
    uint64_t tag;              /* caller's tag from cprng_server_submit */
    uint32_t client;           /* stream id */
    int32_t status;            /* CPRNG_OK, or the error of the batch */
    uint64_t length;           /* outputs */
    uint32_t *out;             /* device, in the arena; valid until released */
    uint64_t t_submit_ns;      /* cprng_now_ns() clock: submitted (as given), */
    uint64_t t_admit_ns;       /* admitted and launched, */
    uint64_t t_done_ns;        /* completion observed by cprng_server_poll */
} cprng_completion_t;

/* Steady monotonic clock in nanoseconds (the clock of cprng_completion_t). */
uint64_t cprng_now_ns(void);

/* Create a server over h (V0 only; h must outlive the server).  Allocates the
 * arena.  Errors: E_INVAL, E_UNSUPPORTED (not V0), E_NOMEM, E_HIP. */
int cprng_server_create(cprng_t *h, const cprng_server_params_t *params, cprng_server_t **out);

/* Queue a request of `length` outputs (1 .. budget/4) for `client`; t_submit_ns
 * is its arrival time on cprng_now_ns()'s clock (0 = now).  Never blocks.
 * Errors: E_INVAL (client out of range, length 0 or larger than the budget). */
int cprng_server_submit(cprng_server_t *s, uint32_t client, uint64_t length, uint64_t tag,
                        uint64_t t_submit_ns);

/* Make progress without blocking: collect finished batches, admit waiting
 * requests in arrival order (a request that does not fit lets later ones of
 * other clients pass, unless it has waited more than 20 ms), launch batches
 * on free HIP streams, and return up to max_done completions (host array).
 * *n_done receives their number.  Errors: E_INVAL, E_HIP. */
int cprng_server_poll(cprng_server_t *s, cprng_completion_t *done, uint32_t max_done, uint32_t *n_done);

/* Return a completed result's memory to the budget.  Errors: E_INVAL. */
int cprng_server_release(cprng_server_t *s, uint32_t *out);

/* Requests waiting for admission, requests on the GPU, arena bytes in use
 * (admitted and not yet released).  Any pointer may be NULL. */
int cprng_server_stats(const cprng_server_t *s, uint64_t *waiting, uint64_t *in_flight,
                       uint64_t *bytes_in_use);

/* Drive the server through a trace in real time: request i (client[i],
 * length[i]) arrives at start + arrival_ns[i] (non-decreasing); the call
 * submits each request at its arrival time, polls until every request has
 * completed, and writes request i's completion to results[i] (host, count
 * entries; tag = i).  With release_results != 0 each result is released as
 * soon as it completes (its `out` is then no longer valid).
 * Errors: E_INVAL, E_HIP. */
int cprng_server_replay(cprng_server_t *s, const uint64_t *arrival_ns, const uint32_t *client,
                        const uint64_t *length, uint32_t count, int release_results,
                        cprng_completion_t *results);

/* As cprng_server_replay with release_results = 1, except that result i is
 * kept (not released; the caller releases it) when keep[i] != 0 (host, count
 * entries): a replay that checks a sample of the results after the run.
 * Errors as cprng_server_replay; E_INVAL for a NULL keep with count > 0. */
int cprng_server_replay_keep(cprng_server_t *s, const uint64_t *arrival_ns, const uint32_t *client,
                             const uint64_t *length, uint32_t count, const uint8_t *keep,
                             cprng_completion_t *results);

/* Wait for the server's batches and free it.  NULL is a no-op. */
void cprng_server_destroy(cprng_server_t *s);

/* ------------------------------------------------------------------------ */
/* Measurement probes (not part of the generator).                           */
/* ------------------------------------------------------------------------ */

/* Fill dst (device, n_words uint32, 16-byte aligned) with `value` using
 * coalesced 16-byte stores: the store-only bandwidth reference. */
int cprng_probe_fill(uint32_t *dst, uint64_t n_words, uint32_t value, cprng_stream_t stream);

/* Copy n_words uint32 from src to dst (device, 16-byte aligned): the copy
 * kernel used to calibrate hardware byte counters. */
int cprng_probe_copy(uint32_t *dst, const uint32_t *src, uint64_t n_words, cprng_stream_t stream);

/* VALU issue-rate probe: n_threads lanes (a multiple of 256) each run `iters`
 * iterations of 32 instructions of one class -- kind 0 v_xor_b32, 1
 * v_lshlrev_b32, 2 v_mul_f32/v_add_f32, 3 v_lshlrev_b64, 4 v_lshl_add_u64 --
 * on 8 registers (pairs for the 64-bit kinds) with no dependency closer than
 * four instructions, then write one word to out (device, n_threads uint32).
 * Errors: E_INVAL (kind > 4, n_threads not a positive multiple of 256, out
 * NULL), E_HIP. */
int cprng_probe_valu(uint32_t kind, uint32_t *out, uint32_t n_threads, uint32_t iters, cprng_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Errors.                                                                   */
/* ------------------------------------------------------------------------ */
const char *cprng_strerror(int status);
const char *cprng_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CPRNG_H */
