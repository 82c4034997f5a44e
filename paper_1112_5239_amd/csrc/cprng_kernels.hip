// cprng_kernels.hip -- gfx950 kernels of the chaotic-iteration PRNG: the chunk
// kernels of batched uneven streams and requests, the probes, and the launch
// entry points.  The generate / consume kernels are in gen_kernels.inc,
// instantiated per variant in gen_v0.hip .. gen_v3.hip.
//
// Every kernel keeps one stream per lane with its whole generator state in
// VGPRs, applies the chaotic iteration x <- x xor S (Section 4.2, Eq. Oplus)
// once per output and writes the state back at the end, as the GPU kernels of
// Section 6 (Algorithms 3 and 4) do.  The work is integer ALU plus stores:
// there is no dense contraction, so no MFMA.  The hot path is bound by HBM
// writes (generate) or by the VALU (consume, and the three-generator
// variant).
//
// Neighbour exchange (Algorithm 4): the paper's shared-memory array is
// replaced by ds_bpermute_b32, which reads another lane's register.  All 64
// lanes are read in one instruction before any lane updates its word, which
// is exactly "every thread reads the previous step's words" -- race-free with
// no barrier, as long as a group of C streams lies within one wave (C | 64).

#include "internal.h"

#pragma clang fp contract(off)

namespace cprng_impl {
namespace {

#include "device_common.inc"

// ------------------------------------------------------------------------
// Segments of V0 streams (batched uneven streams, requests).  Each lane takes
// one segment from a work queue (64 per wave and grab), jumps the stream's
// 160-bit state (xor128 words and x) ahead by the segment's start position,
// then generates and stores its outputs.
//
// Jump: the map v -> A'v (one xor128 step, then x ^= new w) is linear over
// GF(2), so A'^J v = sum_k c_k A'^k v with sum_k c_k X^k = X^J mod q(X),
// q the polynomial annihilating A' (degree <= 129).  The host supplies the
// coefficients c_k; the lane walks k = 0..128, accumulating A'^k v where
// c_k = 1.
// ------------------------------------------------------------------------
__device__ __forceinline__ void jump_v0(X128 &g, uint32_t &x, const uint32_t *poly)
{
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
#pragma unroll 1
    for (int w = 0; w < 5; ++w) {
        const uint32_t pw = poly[w];
        const int nb = (w < 4) ? 32 : 1;     // coefficients 0..128
#pragma unroll 4
        for (int b = 0; b < nb; ++b) {
            const uint32_t m = 0u - ((pw >> b) & 1u);
            a0 ^= g.x & m;
            a1 ^= g.y & m;
            a2 ^= g.z & m;
            a3 ^= g.w & m;
            a4 ^= x & m;
            x ^= x128_next(g);
        }
    }
    g.x = a0; g.y = a1; g.z = a2; g.w = a3;
    x = a4;
}

// Work queues of the chunk kernels (persistent launches): one per XCD.  The
// segments form grabs of 64 (the last may be short); queue x holds the
// contiguous run of grabs that xcd_tile gives XCD x, and its counter
// a.counter[x] counts the grabs taken.  A wave takes one grab at a time from
// its own XCD's queue (workgroup b runs on XCD b % 8) and, once that is empty,
// from the others in turn.  Each XCD thus writes one band of the output in
// order, and small launches still take whole grabs.  Returns false when every
// queue is empty.
__device__ __forceinline__ bool grab_segments(const SegArgs &a, uint32_t lane, uint32_t &qi, uint32_t &base,
                                              uint32_t &end)
{
    if (!a.persistent) {
        // One grab per wave: wave w of workgroup b takes the 64 segments of
        // tile xcd_tile(b) * (waves per workgroup) + w.
        if (qi) return false;
        qi = 8u;
        const uint32_t wpb = blockDim.x >> 6;
        base = (xcd_tile(blockIdx.x, gridDim.x) * wpb + (threadIdx.x >> 6)) * 64u;
        end = (a.nseg - base) < 64u ? a.nseg : base + 64u;
        return base < a.nseg;
    }
    const uint32_t grabs = (a.nseg + 63u) >> 6;
    const uint32_t per = grabs >> 3, extra = grabs & 7u;
    while (qi < 8u) {
        const uint32_t x = (blockIdx.x + qi) & 7u;
        const uint32_t lo = x * per + (x < extra ? x : extra);
        const uint32_t count = per + (x < extra ? 1u : 0u);
        uint32_t off = 0;
        if (lane == 0) off = atomicAdd(a.counter + x, 1u);
        off = (uint32_t)__builtin_amdgcn_readfirstlane((int)off);
        if (off < count) {
            base = (lo + off) * 64u;
            end = (a.nseg - base) < 64u ? a.nseg : base + 64u;
            return true;
        }
        ++qi;
    }
    return false;
}

// Segment idx -> its run, position, length, head and jump polynomial.
struct Seg {
    gu32 *out;             // first output of the segment
    uint32_t len, head, stream, last;
    const uint32_t *poly;  // nullptr: no jump (segment 0); else X^(k*chunk) mod q
    const uint32_t *poly2; // two-level tables: the second factor of the jump, or nullptr
    uint32_t skip;         // steps after the jump: the run's head
    uint64_t pos;          // start position within the run
};

__device__ __forceinline__ Seg decode_segment(const SegArgs &a, uint32_t idx)
{
    // Binary search for the run with first_seg <= idx < next run's first_seg.
    uint32_t lo = 0, hi = a.nrun;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.runs[mid].first_seg <= idx) lo = mid;
        else hi = mid;
    }
    const RunDesc r = a.runs[lo];
    const uint32_t k = idx - r.first_seg;
    Seg s;
    s.stream = r.stream;
    const uint64_t seg0 = (uint64_t)r.head + a.chunk;
    uint64_t len;
    if (k == 0) {
        s.pos = 0;
        len = r.len < seg0 ? r.len : seg0;
        s.head = r.head;
        s.poly = nullptr;
        s.poly2 = nullptr;
        s.skip = 0;
    } else {
        // position head + k*chunk: jump by k*chunk, then step head times
        s.pos = seg0 + (uint64_t)(k - 1) * a.chunk;
        const uint64_t left = r.len - s.pos;
        len = left < a.chunk ? left : a.chunk;
        s.head = 0;
        if (a.polys_hi) {
            const uint32_t klo = k & ((1u << a.lo_bits) - 1u), khi = k >> a.lo_bits;
            s.poly = klo ? a.polys + 5ull * klo : nullptr;
            s.poly2 = khi ? a.polys_hi + 5ull * khi : nullptr;
        } else {
            s.poly = a.polys + 5ull * k;
            s.poly2 = nullptr;
        }
        s.skip = r.head;
    }
    s.len = (uint32_t)len;
    s.out = gptr(r.out) + s.pos;
    s.last = (r.last && s.pos + len == r.len) ? 1u : 0u;
    return s;
}

template <int K>
__global__ __launch_bounds__(256) void k_segments(SegArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t ns = a.ns;
    if (a.nseg_dev) a.nseg = (uint32_t)__builtin_amdgcn_readfirstlane((int)*a.nseg_dev);
    uint32_t qi = 0, base = 0, end = 0;
    while (grab_segments(a, lane, qi, base, end)) {
        const uint32_t idx = base + lane;
        if (idx < end) {
            const Seg d = decode_segment(a, idx);
            const uint32_t *p = a.state + d.stream;
            X128 g{p[0], p[ns], p[2 * ns], p[3 * ns]};
            uint32_t x = p[4 * ns];
            if (d.poly) jump_v0(g, x, d.poly);
            if (d.poly2) jump_v0(g, x, d.poly2);
            for (uint32_t i = 0; i < d.skip; ++i) x ^= x128_next(g);
            gu32 *o = d.out;
            const uint32_t len = d.len;
            uint32_t i = 0;
            const uint32_t head = d.head < len ? d.head : len;
            for (; i < head; ++i) {
                x ^= x128_next(g);
                o[i] = x;
            }
            for (; i + K <= len; i += K) {
                uint32_t v[K];
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    x ^= x128_next(g);
                    v[j] = x;
                }
#pragma unroll
                for (int q = 0; q < K / 4; ++q)
                    gstore4<false>(o + i + 4 * q, v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
            }
            for (; i + 4 <= len; i += 4) {
                uint32_t v0, v1, v2, v3;
                x ^= x128_next(g); v0 = x;
                x ^= x128_next(g); v1 = x;
                x ^= x128_next(g); v2 = x;
                x ^= x128_next(g); v3 = x;
                gstore4<false>(o + i, v0, v1, v2, v3);
            }
            for (; i < len; ++i) {
                x ^= x128_next(g);
                o[i] = x;
            }
            if (d.last) {
                uint32_t *q = a.state_next + d.stream;
                q[0] = g.x; q[ns] = g.y; q[2 * ns] = g.z; q[3 * ns] = g.w;
                q[4 * ns] = x;
            }
        }
    }
}

// Tiled variant of k_segments: one wave per workgroup (each wave runs its
// own number of rounds, so barriers must stay wave-local).  After a grab of
// 64 segments the wave stores, in each round, every segment's next K outputs
// through an LDS tile as in k_generate_tile.  Store instruction j of a round
// covers rows j*RPI .. j*RPI+RPI-1 (RPI = 64/(K/4) rows of K words); the rows
// a lane serves are the same in every round, so their base addresses and
// lengths are read once per grab into registers.  Rounds in which every row
// is full take a branch-free store loop; the last rounds of short segments
// store whole quads, then the final partial quad word by word.  Rows start
// 256-byte aligned after the run's head (0..63 outputs stored singly by
// segment 0), so full rounds write whole lines.
template <int K, bool NT>
__device__ __forceinline__ void segments_tile(SegArgs a, uint32_t *lds)
{
    constexpr int QPR = K / 4;               // quads per row
    constexpr int RPI = 64 / QPR;            // rows per store instruction
    static_assert(QPR <= 64 && 64 % QPR == 0, "K must divide 256");
    uint32_t *tile = lds;                    // 64 rows x K words, quad-swizzled
    uint64_t *mbase = reinterpret_cast<uint64_t *>(lds + 64 * K);   // per row: base after head
    uint32_t *mlen = lds + 64 * K + 128;     // per row: outputs after head
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t q = lane % QPR;           // quad a lane stores
    const uint32_t rsub = lane / QPR;        // row within an instruction's RPI rows
    const uint64_t ns = a.ns;
    if (a.nseg_dev) a.nseg = (uint32_t)__builtin_amdgcn_readfirstlane((int)*a.nseg_dev);
    uint32_t qi = 0, base = 0, end = 0;
    while (grab_segments(a, lane, qi, base, end)) {
        const uint32_t idx = base + lane;
        X128 g{0u, 0u, 0u, 0u};
        uint32_t x = 0, rem = 0, stream = 0, last = 0;
        uint64_t obase = 0;
        if (idx < end) {
            const Seg d = decode_segment(a, idx);
            const uint32_t *p = a.state + d.stream;
            g = X128{p[0], p[ns], p[2 * ns], p[3 * ns]};
            x = p[4 * ns];
            if (d.poly) jump_v0(g, x, d.poly);
            if (d.poly2) jump_v0(g, x, d.poly2);
            for (uint32_t i = 0; i < d.skip; ++i) x ^= x128_next(g);
            const uint32_t head = d.head < d.len ? d.head : d.len;
            for (uint32_t i = 0; i < head; ++i) {
                x ^= x128_next(g);
                d.out[i] = x;
            }
            obase = (uint64_t)(uintptr_t)(d.out + head);
            rem = d.len - head;
            stream = d.stream;
            last = d.last;
        }
        mbase[lane] = obase;
        mlen[lane] = rem;
        __syncthreads();
        uint64_t rb[QPR];
        uint32_t rl[QPR];
#pragma unroll
        for (int j = 0; j < QPR; ++j) {
            rb[j] = mbase[j * RPI + rsub] + 16u * q;
            rl[j] = mlen[j * RPI + rsub];
        }
        uint32_t done = 0;                   // outputs per row stored so far (uniform)
        uint32_t *row = tile + lane * K;
        while (__ballot(rem > 0u) != 0ull) {
            const uint32_t cnt = rem < (uint32_t)K ? rem : (uint32_t)K;
            if (cnt == (uint32_t)K) {
#pragma unroll
                for (int qq = 0; qq < QPR; ++qq) {
                    uint32_t v0, v1, v2, v3;
                    x ^= x128_next(g); v0 = x;
                    x ^= x128_next(g); v1 = x;
                    x ^= x128_next(g); v2 = x;
                    x ^= x128_next(g); v3 = x;
                    store4<false>(row + 4 * (qq ^ (lane & (QPR - 1))), v0, v1, v2, v3);
                }
            } else {
                for (uint32_t j = 0; j < cnt; ++j) {
                    x ^= x128_next(g);
                    row[4 * ((j >> 2) ^ (lane & (QPR - 1))) + (j & 3u)] = x;
                }
            }
            __syncthreads();
            const bool all_full = __ballot(cnt != (uint32_t)K) == 0ull;
            if (all_full) {
#pragma unroll
                for (int j = 0; j < QPR; ++j) {
                    const uint32_t r = j * RPI + rsub;
                    uint32_t x0, x1, x2, x3;
                    load4(tile + r * K + 4 * (q ^ (r & (QPR - 1))), x0, x1, x2, x3);
                    gstore4<NT>(gptr(rb[j] + 4ull * done), x0, x1, x2, x3);
                }
            } else {
#pragma unroll
                for (int j = 0; j < QPR; ++j) {
                    const uint32_t r = j * RPI + rsub;
                    const uint32_t left = rl[j] > done ? rl[j] - done : 0u;
                    const uint32_t cr = left < (uint32_t)K ? left : (uint32_t)K;
                    if (4 * q < cr) {
                        const uint32_t *src = tile + r * K + 4 * (q ^ (r & (QPR - 1)));
                        gu32 *dst = gptr(rb[j] + 4ull * done);
                        if (4 * q + 4 <= cr) {
                            uint32_t x0, x1, x2, x3;
                            load4(src, x0, x1, x2, x3);
                            gstore4<NT>(dst, x0, x1, x2, x3);
                        } else {
                            for (uint32_t e = 0; e < cr - 4 * q; ++e) dst[e] = src[e];
                        }
                    }
                }
            }
            __syncthreads();
            done += (uint32_t)K;
            rem -= cnt;
        }
        if (last) {
            uint32_t *st = a.state_next + stream;
            st[0] = g.x; st[ns] = g.y; st[2 * ns] = g.z; st[3 * ns] = g.w;
            st[4 * ns] = x;
        }
    }
}

template <int K, bool NT>
__global__ __launch_bounds__(64) void k_segments_tile(SegArgs a)
{
    HIP_DYNAMIC_SHARED(uint32_t, lds);
    segments_tile<K, NT>(a, lds);
}

// The same with the run descriptors in the kernel arguments (small request
// batches): they are read through the kernel-argument segment, so no upload
// precedes the launch.
template <int K, bool NT>
__global__ __launch_bounds__(64) void k_segments_tile_inline(SegInline s)
{
    HIP_DYNAMIC_SHARED(uint32_t, lds);
    const SegInline *p = (const SegInline *)__builtin_amdgcn_kernarg_segment_ptr();
    SegArgs a = p->a;
    a.runs = p->runs;
    segments_tile<K, NT>(a, lds);
}

// Commit of an inline batch (ids in the kernel arguments, at most 64), which
// also clears the batch's work-queue counters for the next launch.
__global__ __launch_bounds__(64) void k_commit_inline(SegInline s, uint32_t *state)
{
    const SegInline *p = (const SegInline *)__builtin_amdgcn_kernarg_segment_ptr();
    const uint32_t i = threadIdx.x;
    if (i < 8u) p->a.counter[i] = 0u;
    if (i >= p->n_ids) return;
    const uint64_t id = p->ids[i], ns = p->a.ns;
#pragma unroll
    for (int k = 0; k < 5; ++k) state[k * ns + id] = p->a.state_next[k * ns + id];
}

// Copies the listed streams' end states back; with `reset` set, thread 0
// also clears the 8 work-queue counters for the next launch on the stream
// (after the segment kernel that used them has finished, in stream order).
__global__ void k_commit(uint32_t *state, const uint32_t *state_next, const uint32_t *ids,
                         uint32_t count, uint32_t ns, uint32_t *reset)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (reset && i < 8u) reset[i] = 0u;
    if (i >= count) return;
    const uint64_t id = ids[i];
#pragma unroll
    for (int k = 0; k < 5; ++k) state[k * (uint64_t)ns + id] = state_next[k * (uint64_t)ns + id];
}

// ------------------------------------------------------------------------
// Stream subsets described in device memory (ids, lengths and output offsets
// that the caller's kernels may have written).  Three small kernels turn the
// descriptors into the run list of the segment kernels above with no host
// round trip:
//   k_subset_count  checks each descriptor and counts its segments, with one
//                   sum per block of 256 descriptors;
//   k_subset_scan   (one workgroup) turns the block sums into offsets,
//                   decides the call's status, resets the work-queue
//                   counters and moves to the next call epoch;
//   k_subset_runs   writes the run descriptors.
// A repeated stream id is caught with a per-stream mark: each descriptor
// swaps the call's epoch into its stream's mark, and a swap that returns that
// same epoch means another descriptor of the call named the stream first.
// After an error the segment count is 0 and the commit is skipped, so no
// output is written and no state changes.
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t subset_head(uint64_t addr) { return (64u - (uint32_t)((addr >> 2) & 63u)) & 63u; }

__global__ __launch_bounds__(256) void k_subset_count(SubsetArgs a)
{
    __shared__ unsigned long long part[4];
    const uint32_t t = threadIdx.x, lane = t & 63u;
    const uint32_t i = blockIdx.x * 256u + t;
    uint32_t nseg = 0;
    bool bad = false;
    if (i < a.count) {
        const uint32_t id = a.ids[i];
        const uint64_t len = a.lens[i];
        if (id >= a.ns || len > kSubsetMaxLen) {
            bad = true;
        } else {
            const unsigned long long ep = a.ctl->epoch;
            if (atomicExch(a.mark + id, ep) == ep) bad = true;
            if (len) {
                const uint64_t seg0 = (uint64_t)subset_head(a.out_base + 4ull * a.offs[i]) + a.chunk;
                nseg = len <= seg0 ? 1u : (uint32_t)(1u + (len - seg0 + a.chunk - 1u) / a.chunk);
            }
        }
        a.segs[i] = nseg;
    }
    if (bad) atomicOr(&a.ctl->err, 1u);
    unsigned long long v = nseg;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    if (lane == 0) part[t >> 6] = v;
    __syncthreads();
    if (t == 0) a.bsum[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ __launch_bounds__(1024) void k_subset_scan(SubsetArgs a)
{
    __shared__ unsigned long long wsum[16];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    unsigned long long carry = 0;
    for (uint32_t base = 0; base < a.nblocks; base += 1024u) {
        const uint32_t i = base + t;
        const unsigned long long v = i < a.nblocks ? a.bsum[i] : 0ull;
        unsigned long long inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned long long o = __shfl_up(inc, d);
            if (lane >= (uint32_t)d) inc += o;
        }
        if (lane == 63u) wsum[w] = inc;
        __syncthreads();
        unsigned long long before = 0, total = 0;
        for (uint32_t k = 0; k < 16u; ++k) {
            if (k < w) before += wsum[k];
            total += wsum[k];
        }
        if (i < a.nblocks) a.bsum[i] = carry + before + inc - v;
        carry += total;
        __syncthreads();
    }
    if (t == 0) {
        const bool ok = a.ctl->err == 0u && carry < (1ull << 31);
        const int32_t st = ok ? 0 : (int32_t)CPRNG_E_INVAL;
        a.ctl->nseg = ok ? (uint32_t)carry : 0u;
        a.ctl->status = st;
        if (a.status) *a.status = st;
        a.ctl->err = 0u;
        a.ctl->epoch = a.ctl->epoch + 1ull;
    }
    if (t < 8u) a.ctl->counter[t] = 0u;
}

__global__ __launch_bounds__(256) void k_subset_runs(SubsetArgs a)
{
    if (a.ctl->status != 0) return;
    __shared__ uint32_t part[4];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const uint32_t i = blockIdx.x * 256u + t;
    // With the status clear the call has fewer than 2^31 segments, so every
    // prefix below fits 32 bits.
    const uint32_t v = i < a.count ? a.segs[i] : 0u;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d);
        if (lane >= (uint32_t)d) inc += o;
    }
    if (lane == 63u) part[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t k = 0; k < w; ++k) before += part[k];
    if (i < a.count) {
        RunDesc r;
        r.out = a.out_base + 4ull * a.offs[i];
        r.len = a.lens[i];
        r.stream = a.ids[i];
        r.head = subset_head(r.out);
        r.first_seg = (uint32_t)a.bsum[blockIdx.x] + before + inc - v;
        r.last = 1u;
        a.runs[i] = r;
    }
}

__global__ __launch_bounds__(256) void k_subset_commit(SubsetArgs a, uint32_t *state, const uint32_t *state_next)
{
    if (a.ctl->status != 0) return;
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= a.count || a.lens[i] == 0) return;
    const uint64_t id = a.ids[i], ns = a.ns;
#pragma unroll
    for (int k = 0; k < 5; ++k) state[k * ns + id] = state_next[k * ns + id];
}

__global__ void k_zero_u32(uint32_t *p, uint32_t count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// ------------------------------------------------------------------------
// Probes: store-only fill and copy with 16-byte accesses (grid-stride).
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill(uint32_t *dst, uint64_t nq, uint32_t value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride)
        store4<false>(dst + 4 * q, value, value, value, value);
}

__global__ __launch_bounds__(256) void k_copy(uint32_t *dst, const uint32_t *src, uint64_t nq)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride) {
        uint32_t a0, a1, a2, a3;
        load4(src + 4 * q, a0, a1, a2, a3);
        store4<false>(dst + 4 * q, a0, a1, a2, a3);
    }
}

// VALU issue-rate probe: each iteration issues 32 instructions of one class
// on 8 registers per lane, ordered (inline assembly, so the compiler keeps
// the order) so that every instruction depends only on one issued four or
// more instructions earlier.  KIND 0: v_xor_b32; 1: v_lshlrev_b32; 2:
// v_mul_f32 / v_add_f32; 3: v_lshlrev_b64; 4: v_lshl_add_u64 (64-bit add).
// On gfx950 the classes issue at different rates, which the ALU rooflines of
// the consumption kernel and of the 64-bit-word variant are weighted by.
#define CPRNG_PROBE_ROUND(OP)                                                              \
    OP " %0, %0, %1\n" OP " %2, %2, %3\n" OP " %4, %4, %5\n" OP " %6, %6, %7\n"            \
    OP " %1, %1, %2\n" OP " %3, %3, %4\n" OP " %5, %5, %6\n" OP " %7, %7, %0\n"
#define CPRNG_PROBE_SHL64                                                                  \
    "v_lshlrev_b64 %0, 3, %1\n v_lshlrev_b64 %2, 3, %3\n v_lshlrev_b64 %4, 3, %5\n"       \
    "v_lshlrev_b64 %6, 3, %7\n v_lshlrev_b64 %1, 3, %2\n v_lshlrev_b64 %3, 3, %4\n"       \
    "v_lshlrev_b64 %5, 3, %6\n v_lshlrev_b64 %7, 3, %0\n"
#define CPRNG_PROBE_ADD64                                                                  \
    "v_lshl_add_u64 %0, %0, 0, %1\n v_lshl_add_u64 %2, %2, 0, %3\n"                          \
    "v_lshl_add_u64 %4, %4, 0, %5\n v_lshl_add_u64 %6, %6, 0, %7\n"                          \
    "v_lshl_add_u64 %1, %1, 0, %2\n v_lshl_add_u64 %3, %3, 0, %4\n"                          \
    "v_lshl_add_u64 %5, %5, 0, %6\n v_lshl_add_u64 %7, %7, 0, %0\n"
template <int KIND>
__global__ __launch_bounds__(256) void k_valu_probe(uint32_t *out, uint32_t iters)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (KIND >= 3) {
        uint64_t b0 = gid, b1 = gid + 1, b2 = gid + 2, b3 = gid + 3, b4 = gid + 4, b5 = gid + 5, b6 = gid + 6,
                 b7 = gid + 7;
        for (uint32_t i = 0; i < iters; ++i) {
            if constexpr (KIND == 3)
                asm volatile(CPRNG_PROBE_SHL64 CPRNG_PROBE_SHL64 CPRNG_PROBE_SHL64 CPRNG_PROBE_SHL64
                             : "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3), "+v"(b4), "+v"(b5), "+v"(b6), "+v"(b7));
            else
                asm volatile(CPRNG_PROBE_ADD64 CPRNG_PROBE_ADD64 CPRNG_PROBE_ADD64 CPRNG_PROBE_ADD64
                             : "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3), "+v"(b4), "+v"(b5), "+v"(b6), "+v"(b7));
        }
        const uint64_t r = b0 ^ b1 ^ b2 ^ b3 ^ b4 ^ b5 ^ b6 ^ b7;
        out[gid] = (uint32_t)r ^ (uint32_t)(r >> 32);
        return;
    }
    uint32_t a0 = gid, a1 = gid + 1, a2 = gid + 2, a3 = gid + 3, a4 = gid + 4, a5 = gid + 5, a6 = gid + 6,
             a7 = gid + 7;
    for (uint32_t i = 0; i < iters; ++i) {
        if constexpr (KIND == 0)
            asm volatile(CPRNG_PROBE_ROUND("v_xor_b32") CPRNG_PROBE_ROUND("v_xor_b32")
                         CPRNG_PROBE_ROUND("v_xor_b32") CPRNG_PROBE_ROUND("v_xor_b32")
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7));
        else if constexpr (KIND == 1)
            asm volatile(CPRNG_PROBE_ROUND("v_lshlrev_b32") CPRNG_PROBE_ROUND("v_lshlrev_b32")
                         CPRNG_PROBE_ROUND("v_lshlrev_b32") CPRNG_PROBE_ROUND("v_lshlrev_b32")
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7));
        else
            asm volatile(CPRNG_PROBE_ROUND("v_mul_f32") CPRNG_PROBE_ROUND("v_add_f32")
                         CPRNG_PROBE_ROUND("v_mul_f32") CPRNG_PROBE_ROUND("v_add_f32")
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7));
    }
    out[gid] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}
#undef CPRNG_PROBE_ROUND
#undef CPRNG_PROBE_SHL64
#undef CPRNG_PROBE_ADD64

__global__ void k_tail_words(uint32_t *dst, const uint32_t *src, uint64_t begin, uint64_t end, uint32_t value)
{
    const uint64_t i = begin + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i < end) dst[i] = src ? src[i] : value;
}


}  // namespace

hipError_t launch_generate(const GenArgs &a, int variant, int w32, const LaunchCfg &c, hipStream_t st)
{
    const uint32_t max_block = (c.store == ST_ILV_TILE || c.store == ST_ILV_TILE_NT) ? 1024u : 256u;
    if (c.block == 0 || c.block % 64 != 0 || c.block > max_block) return hipErrorInvalidValue;
    switch (variant) {
    case 0: return launch_generate_v0(a, c, st);
    case 1: return launch_generate_v1(a, w32 != 0, c, st);
    case 2: return launch_generate_v2(a, c, st);
    case 3: return launch_generate_v3(a, c, st);
    case 4: return launch_generate_v4(a, c, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_consume(const GenArgs &a, int variant, int w32, const LaunchCfg &c, hipStream_t st)
{
    if (c.block == 0 || c.block % 64 != 0 || c.block > 256) return hipErrorInvalidValue;
    switch (variant) {
    case 0: return launch_consume_v0(a, c, st);
    case 1: return launch_consume_v1(a, w32 != 0, c, st);
    case 2: return launch_consume_v2(a, c, st);
    case 3: return launch_consume_v3(a, c, st);
    case 4: return launch_consume_v4(a, c, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_segments(const SegArgs &a, uint32_t grid, uint32_t block, uint32_t store, uint32_t lds_min,
                           hipStream_t st)
{
    if (grid == 0) return hipErrorInvalidValue;
    if (store == ST_LDS || store == ST_LDS_NT) {
        const bool nt = store == ST_LDS_NT;
        size_t lds = (size_t)64 * a.unroll * 4 + 64 * 12;
        if (lds < lds_min) lds = lds_min;
#define SEG_TILE(K)                                                                              \
    do {                                                                                         \
        if (nt) hipLaunchKernelGGL((k_segments_tile<K, true>), dim3(grid), dim3(64), lds, st, a);  \
        else hipLaunchKernelGGL((k_segments_tile<K, false>), dim3(grid), dim3(64), lds, st, a);    \
    } while (0)
        switch (a.unroll) {
        case 32: SEG_TILE(32); break;
        case 64: SEG_TILE(64); break;
        case 128: SEG_TILE(128); break;
        case 256: SEG_TILE(256); break;                 // 64 KiB tile + row data (gfx950: 160 KiB per workgroup)
        default: return hipErrorInvalidValue;
        }
#undef SEG_TILE
        return hipGetLastError();
    }
    if (block == 0 || block % 64 != 0 || block > 256) return hipErrorInvalidValue;
    switch (a.unroll) {
    case 8: hipLaunchKernelGGL((k_segments<8>), dim3(grid), dim3(block), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_segments<16>), dim3(grid), dim3(block), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_segments<32>), dim3(grid), dim3(block), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_subset(const SubsetArgs &sa, const SegArgs &a, uint32_t grid, uint32_t block, uint32_t store,
                         uint32_t *state, hipStream_t st)
{
    if (sa.count == 0 || sa.nblocks != (sa.count + 255u) / 256u || !a.nseg_dev || !a.persistent)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_subset_count, dim3(sa.nblocks), dim3(256), 0, st, sa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_subset_scan, dim3(1), dim3(1024), 0, st, sa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_subset_runs, dim3(sa.nblocks), dim3(256), 0, st, sa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_segments(a, grid, block, store, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_subset_commit, dim3(sa.nblocks), dim3(256), 0, st, sa, state, a.state_next);
    return hipGetLastError();
}

hipError_t launch_segments_inline(const SegInline &si, uint32_t grid, uint32_t store, hipStream_t st)
{
    if (grid == 0 || si.n_ids > kInlineRuns || si.a.nrun > kInlineRuns || (store != ST_LDS && store != ST_LDS_NT))
        return hipErrorInvalidValue;
    const bool nt = store == ST_LDS_NT;
    const size_t lds = (size_t)64 * si.a.unroll * 4 + 64 * 12;
#define SEG_TILE_INLINE(K)                                                                                   \
    do {                                                                                                     \
        if (nt) hipLaunchKernelGGL((k_segments_tile_inline<K, true>), dim3(grid), dim3(64), lds, st, si);    \
        else hipLaunchKernelGGL((k_segments_tile_inline<K, false>), dim3(grid), dim3(64), lds, st, si);      \
    } while (0)
    switch (si.a.unroll) {
    case 32: SEG_TILE_INLINE(32); break;
    case 64: SEG_TILE_INLINE(64); break;
    case 128: SEG_TILE_INLINE(128); break;
    case 256: SEG_TILE_INLINE(256); break;
    default: return hipErrorInvalidValue;
    }
#undef SEG_TILE_INLINE
    return hipGetLastError();
}

hipError_t launch_commit_inline(const SegInline &si, uint32_t *state, hipStream_t st)
{
    if (si.n_ids > kInlineRuns) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_commit_inline, dim3(1), dim3(64), 0, st, si, state);
    return hipGetLastError();
}

hipError_t launch_commit(uint32_t *state, const uint32_t *state_next, const uint32_t *ids,
                         uint32_t count, uint32_t ns, hipStream_t st, uint32_t *reset_counters)
{
    if (count == 0 && !reset_counters) return hipSuccess;
    const uint32_t grid = count ? (count + 255) / 256 : 1u;
    hipLaunchKernelGGL(k_commit, dim3(grid), dim3(256), 0, st, state, state_next, ids, count, ns, reset_counters);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t count, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

static uint32_t probe_grid(uint64_t nq)
{
    uint64_t g = (nq + 255) / 256;
    const uint64_t cap = 256ull * 64;          // plenty of waves for 256 CUs
    if (g > cap) g = cap;
    return (uint32_t)(g ? g : 1);
}

hipError_t launch_valu_probe(uint32_t kind, uint32_t *out, uint32_t n_threads, uint32_t iters, hipStream_t st)
{
    if (n_threads == 0 || n_threads % 256) return hipErrorInvalidValue;
    switch (kind) {
    case 0: hipLaunchKernelGGL(k_valu_probe<0>, dim3(n_threads / 256), dim3(256), 0, st, out, iters); break;
    case 1: hipLaunchKernelGGL(k_valu_probe<1>, dim3(n_threads / 256), dim3(256), 0, st, out, iters); break;
    case 2: hipLaunchKernelGGL(k_valu_probe<2>, dim3(n_threads / 256), dim3(256), 0, st, out, iters); break;
    case 3: hipLaunchKernelGGL(k_valu_probe<3>, dim3(n_threads / 256), dim3(256), 0, st, out, iters); break;
    case 4: hipLaunchKernelGGL(k_valu_probe<4>, dim3(n_threads / 256), dim3(256), 0, st, out, iters); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_group_chunks(const GroupJumpArgs &a, int variant, hipStream_t st)
{
    switch (variant) {
    case 2: return launch_group_chunks_v2(a, st);
    case 4: return launch_group_chunks_v4(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fill(uint32_t *dst, uint64_t n_words, uint32_t value, hipStream_t st)
{
    const uint64_t nq = n_words / 4;
    if (nq) hipLaunchKernelGGL(k_fill, dim3(probe_grid(nq)), dim3(256), 0, st, dst, nq, value);
    if (n_words % 4)
        hipLaunchKernelGGL(k_tail_words, dim3(1), dim3(64), 0, st, dst, (const uint32_t *)nullptr,
                           nq * 4, n_words, value);
    return hipGetLastError();
}

hipError_t launch_copy(uint32_t *dst, const uint32_t *src, uint64_t n_words, hipStream_t st)
{
    const uint64_t nq = n_words / 4;
    if (nq) hipLaunchKernelGGL(k_copy, dim3(probe_grid(nq)), dim3(256), 0, st, dst, src, nq);
    if (n_words % 4)
        hipLaunchKernelGGL(k_tail_words, dim3(1), dim3(64), 0, st, dst, src, nq * 4, n_words, 0u);
    return hipGetLastError();
}

}  // namespace cprng_impl

