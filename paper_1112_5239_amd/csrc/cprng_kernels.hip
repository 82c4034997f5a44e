// cprng_kernels.hip -- gfx950 kernels of the chaotic-iteration PRNG.
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

// ------------------------------------------------------------------------
// Strategy generators.
// ------------------------------------------------------------------------
struct X128 {
    uint32_t x, y, z, w;
};

// Marsaglia xor128 on 32-bit words (the xor-like generator of Algorithm 4).
__device__ __forceinline__ uint32_t x128_next(X128 &g)
{
    uint32_t t = g.x ^ (g.x << 11);
    g.x = g.y;
    g.y = g.z;
    g.z = g.w;
    g.w = (g.w ^ (g.w >> 19)) ^ (t ^ (t >> 8));
    return g.w;
}

// The three generators of Listing 1 on words of type T (uint64_t: the
// listing's 64-bit generators; uint32_t: the 32-bit-word option).
template <typename T>
struct Naive3 {
    T a;                     // xorshift (13,17,5), Algorithm 2's triple
    T b0, b1, b2, b3;        // xor128
    T c0, c1, c2, c3, c4, d; // xorwow (d: Weyl counter)
};

template <typename T>
__device__ __forceinline__ uint32_t naive3_strategy(Naive3<T> &g)
{
    T a = g.a;
    a ^= a << 13;
    a ^= a >> 17;
    a ^= a << 5;
    g.a = a;

    T t = g.b0 ^ (g.b0 << 11);
    g.b0 = g.b1;
    g.b1 = g.b2;
    g.b2 = g.b3;
    g.b3 = (g.b3 ^ (g.b3 >> 19)) ^ (t ^ (t >> 8));

    T u = g.c0 ^ (g.c0 >> 2);
    g.c0 = g.c1;
    g.c1 = g.c2;
    g.c2 = g.c3;
    g.c3 = g.c4;
    g.c4 = (g.c4 ^ (g.c4 << 4)) ^ (u ^ (u << 1));
    g.d += (T)362437u;

    // S = xor of the low and high halves of the three outputs.
    T f = a ^ g.b3 ^ (T)(g.d + g.c4);
    if constexpr (sizeof(T) == 8)
        return (uint32_t)f ^ (uint32_t)(f >> 32);
    else
        return (uint32_t)f;
}

// ------------------------------------------------------------------------
// Per-variant stream state held in registers.  SoA in memory: word k of
// stream s is state[k * ns + s].
// ------------------------------------------------------------------------
template <int VAR, typename T>
struct Stream;

template <typename T>
struct Stream<0, T> {                       // V0 PLAIN
    X128 g;
    uint32_t x;
    __device__ void load(const GenArgs &a, uint32_t s)
    {
        const uint32_t *p = a.state + s;
        const uint64_t ns = a.ns;
        g.x = p[0]; g.y = p[ns]; g.z = p[2 * ns]; g.w = p[3 * ns];
        x = p[4 * ns];
    }
    __device__ void save(const GenArgs &a, uint32_t s) const
    {
        uint32_t *p = a.state + s;
        const uint64_t ns = a.ns;
        p[0] = g.x; p[ns] = g.y; p[2 * ns] = g.z; p[3 * ns] = g.w;
        p[4 * ns] = x;
    }
    __device__ void init_exchange(const GenArgs &, uint32_t) {}
    __device__ __forceinline__ uint32_t next()
    {
        x ^= x128_next(g);
        return x;
    }
    __device__ __forceinline__ void next2(uint32_t &r0, uint32_t &r1)
    {
        r0 = next();
        r1 = next();
    }
};

template <typename T>
struct Stream<2, T> {                       // V2 SHMEM (Algorithm 4)
    X128 g;
    uint32_t x, t;                          // t: this stream's previous mixed word
    int a1, a2;                             // byte addresses of lanes o1(j), o2(j)
    int a11, a21, a12, a22;                 // lanes o1(o1(j)), o2(o1(j)), o1(o2(j)), o2(o2(j))
    __device__ void load(const GenArgs &a, uint32_t s)
    {
        const uint32_t *p = a.state + s;
        const uint64_t ns = a.ns;
        g.x = p[0]; g.y = p[ns]; g.z = p[2 * ns]; g.w = p[3 * ns];
        x = p[4 * ns];
        t = p[5 * ns];
    }
    __device__ void save(const GenArgs &a, uint32_t s) const
    {
        uint32_t *p = a.state + s;
        const uint64_t ns = a.ns;
        p[0] = g.x; p[ns] = g.y; p[2 * ns] = g.z; p[3 * ns] = g.w;
        p[4 * ns] = x;
        p[5 * ns] = t;
    }
    __device__ void init_exchange(const GenArgs &a, uint32_t lane)
    {
        // o = threadIdx - offset + comb[offset], offset = threadIdx mod C,
        // within the wave (the group never straddles a wave since C | 64).
        const uint32_t m = a.group - 1;
        const uint32_t gb = lane & ~m;
        const uint32_t o1 = gb + a.comb1[lane & m];
        const uint32_t o2 = gb + a.comb2[lane & m];
        a1 = (int)(o1 << 2);
        a2 = (int)(o2 << 2);
        a11 = (int)((gb + a.comb1[o1 & m]) << 2);
        a21 = (int)((gb + a.comb2[o1 & m]) << 2);
        a12 = (int)((gb + a.comb1[o2 & m]) << 2);
        a22 = (int)((gb + a.comb2[o2 & m]) << 2);
    }
    __device__ __forceinline__ uint32_t next()
    {
        const uint32_t u = x128_next(g);
        const uint32_t n1 = (uint32_t)__builtin_amdgcn_ds_bpermute(a1, (int)t);
        const uint32_t n2 = (uint32_t)__builtin_amdgcn_ds_bpermute(a2, (int)t);
        t = u ^ n1 ^ n2;
        x ^= t;
        return x;
    }
    // One step with the exchange through a per-wave LDS buffer xb[64]: every
    // lane writes its previous word, then reads the two words it mixes.  LDS
    // executes one wave's instructions in order, so all writes of the step
    // land before any read; comb1/comb2 permute each group of consecutive
    // words, so the reads are bank-conflict-free.
    __device__ __forceinline__ uint32_t next_lds(uint32_t *xb, uint32_t lane)
    {
        const uint32_t u = x128_next(g);
        xb[lane] = t;
        __builtin_amdgcn_wave_barrier();
        const uint32_t n1 = xb[a1 >> 2];
        const uint32_t n2 = xb[a2 >> 2];
        __builtin_amdgcn_wave_barrier();
        t = u ^ n1 ^ n2;
        x ^= t;
        return x;
    }
    // Two steps with one round of cross-lane reads:
    //   t1 = u1 ^ t[o1] ^ t[o2]
    //   t2 = u2 ^ t1[o1] ^ t1[o2]
    //      = u2 ^ u1[o1] ^ u1[o2] ^ t[o1(o1)] ^ t[o2(o1)] ^ t[o1(o2)] ^ t[o2(o2)]
    // (all reads see the words of the step before, as in next()).
    __device__ __forceinline__ void next2(uint32_t &r0, uint32_t &r1)
    {
        const uint32_t u1 = x128_next(g);
        const uint32_t u2 = x128_next(g);
        const uint32_t p1 = (uint32_t)__builtin_amdgcn_ds_bpermute(a1, (int)t);
        const uint32_t p2 = (uint32_t)__builtin_amdgcn_ds_bpermute(a2, (int)t);
        const uint32_t p11 = (uint32_t)__builtin_amdgcn_ds_bpermute(a11, (int)t);
        const uint32_t p21 = (uint32_t)__builtin_amdgcn_ds_bpermute(a21, (int)t);
        const uint32_t p12 = (uint32_t)__builtin_amdgcn_ds_bpermute(a12, (int)t);
        const uint32_t p22 = (uint32_t)__builtin_amdgcn_ds_bpermute(a22, (int)t);
        const uint32_t q1 = (uint32_t)__builtin_amdgcn_ds_bpermute(a1, (int)u1);
        const uint32_t q2 = (uint32_t)__builtin_amdgcn_ds_bpermute(a2, (int)u1);
        const uint32_t t1 = u1 ^ p1 ^ p2;
        const uint32_t t2 = u2 ^ q1 ^ q2 ^ p11 ^ p21 ^ p12 ^ p22;
        x ^= t1;
        r0 = x;
        x ^= t2;
        r1 = x;
        t = t2;
    }
};

template <typename T>
struct Stream<1, T> {                       // V1 NAIVE3 (Listing 1, Algorithm 3)
    Naive3<T> g;
    uint32_t x;
    __device__ static T ld(const uint32_t *p, uint64_t ns, int k)
    {
        if constexpr (sizeof(T) == 8)
            return (T)p[(2 * k) * ns] | ((T)p[(2 * k + 1) * ns] << 32);
        else
            return (T)p[(2 * k) * ns];
    }
    __device__ static void st(uint32_t *p, uint64_t ns, int k, T v)
    {
        p[(2 * k) * ns] = (uint32_t)v;
        if constexpr (sizeof(T) == 8)
            p[(2 * k + 1) * ns] = (uint32_t)(v >> 32);
        else
            p[(2 * k + 1) * ns] = 0u;
    }
    __device__ void load(const GenArgs &a, uint32_t s)
    {
        const uint32_t *p = a.state + s;
        const uint64_t ns = a.ns;
        g.a = ld(p, ns, 0);
        g.b0 = ld(p, ns, 1); g.b1 = ld(p, ns, 2); g.b2 = ld(p, ns, 3); g.b3 = ld(p, ns, 4);
        g.c0 = ld(p, ns, 5); g.c1 = ld(p, ns, 6); g.c2 = ld(p, ns, 7); g.c3 = ld(p, ns, 8);
        g.c4 = ld(p, ns, 9); g.d = ld(p, ns, 10);
        x = p[22 * ns];
    }
    __device__ void save(const GenArgs &a, uint32_t s) const
    {
        uint32_t *p = a.state + s;
        const uint64_t ns = a.ns;
        st(p, ns, 0, g.a);
        st(p, ns, 1, g.b0); st(p, ns, 2, g.b1); st(p, ns, 3, g.b2); st(p, ns, 4, g.b3);
        st(p, ns, 5, g.c0); st(p, ns, 6, g.c1); st(p, ns, 7, g.c2); st(p, ns, 8, g.c3);
        st(p, ns, 9, g.c4); st(p, ns, 10, g.d);
        p[22 * ns] = x;
    }
    __device__ void init_exchange(const GenArgs &, uint32_t) {}
    __device__ __forceinline__ uint32_t next()
    {
        x ^= naive3_strategy(g);
        return x;
    }
    __device__ __forceinline__ void next2(uint32_t &r0, uint32_t &r1)
    {
        r0 = next();
        r1 = next();
    }
};

// ------------------------------------------------------------------------
// Stores.
// ------------------------------------------------------------------------
template <bool NT>
__device__ __forceinline__ void store4(uint32_t *p, uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 v = {a, b, c, d};
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
    else
        *reinterpret_cast<u32x4 *>(p) = v;
}

__device__ __forceinline__ void load4(const uint32_t *p, uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 v = *reinterpret_cast<const u32x4 *>(p);
    a = v.x; b = v.y; c = v.z; d = v.w;
}

// Pointers rebuilt from integers default to the generic (flat) address
// space; these keep chunk outputs in the global address space.
typedef __attribute__((address_space(1))) uint32_t gu32;

__device__ __forceinline__ gu32 *gptr(uint64_t addr) { return (gu32 *)(uintptr_t)addr; }

template <bool NT>
__device__ __forceinline__ void gstore4(gu32 *p, uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) u32x4 gu32x4;
    u32x4 v = {a, b, c, d};
    if constexpr (NT)
        __builtin_nontemporal_store(v, (gu32x4 *)p);
    else
        *(gu32x4 *)p = v;
}

// Workgroup -> tile map for the 8 XCDs of the chip.  Workgroups are handed
// to the XCDs round-robin (workgroup b runs on XCD b % 8); this bijection of
// [0, nb) gives XCD x the contiguous run of tiles x*floor(nb/8) + min(x, nb%8)
// ... , so each XCD's L2 and its stores sweep one band of the output in
// order instead of every XCD touching every eighth tile.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb)
{
    const uint32_t x = b & 7u, local = b >> 3;
    const uint32_t per = nb >> 3, extra = nb & 7u;
    return x * per + (x < extra ? x : extra) + local;
}

// ------------------------------------------------------------------------
// Plain generate kernel: one lane per stream, K outputs per lane per round.
//   ST_DIRECT(_NT): lane stores its K outputs as K/4 aligned 16-byte quads.
//   ST_INTERLEAVED: out[i * ns + s]; 64 lanes write 256 contiguous bytes.
//   ST_GENERIC    : out[s * n + i] one dword at a time (any n, any alignment).
// Fast modes need n % 4 == 0 and a 16-byte aligned `out` (host checks).
// ------------------------------------------------------------------------
template <int VAR, typename T, int K, int MODE>
__global__ __launch_bounds__(256) void k_generate(GenArgs a)
{
    constexpr bool NT = (MODE == ST_DIRECT_NT);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    const uint64_t n = a.n;
    Stream<VAR, T> st;
    st.load(a, s);
    st.init_exchange(a, lane);
    if constexpr (MODE == ST_INTERLEAVED) {
        uint64_t i = 0;
        for (; i + K <= n; i += K) {
            uint32_t v[K];
#pragma unroll
            for (int j = 0; j < K; ++j) v[j] = st.next();
#pragma unroll
            for (int j = 0; j < K; ++j) a.out[(i + j) * a.ns + s] = v[j];
        }
        for (; i < n; ++i) a.out[i * a.ns + s] = st.next();
    } else if constexpr (MODE == ST_GENERIC) {
        uint32_t *o = a.out + (uint64_t)s * n;
        uint64_t i = 0;
        for (; i + K <= n; i += K) {
            uint32_t v[K];
#pragma unroll
            for (int j = 0; j < K; ++j) v[j] = st.next();
#pragma unroll
            for (int j = 0; j < K; ++j) o[i + j] = v[j];
        }
        for (; i < n; ++i) o[i] = st.next();
    } else {
        uint32_t *o = a.out + (uint64_t)s * n;
        uint64_t i = 0;
        for (; i + K <= n; i += K) {
            uint32_t v[K];
#pragma unroll
            for (int j = 0; j < K; ++j) v[j] = st.next();
#pragma unroll
            for (int q = 0; q < K / 4; ++q)
                store4<NT>(o + i + 4 * q, v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        }
        for (; i < n; i += 4) {              // n % 4 == 0
            uint32_t v0 = st.next(), v1 = st.next(), v2 = st.next(), v3 = st.next();
            store4<NT>(o + i, v0, v1, v2, v3);
        }
    }
    st.save(a, s);
}

// ------------------------------------------------------------------------
// Tiled generate kernel (stream-major output through LDS).
//
// A wave owns 64*S consecutive streams: lane l, slot k holds stream
// base + 64k + l, so each slot's 64 lanes hold whole groups of C | 64 streams
// and the exchange addresses are the same for every slot; the S streams of a
// lane are independent, which gives the exchange's cross-lane reads S-fold
// instruction-level parallelism.  Each round every stream writes its next K
// outputs into its LDS row (row 64k + l); then store instruction j covers
// quads j*64 .. j*64+63 of the row-major (64 S) x K tile, i.e. 64/(K/4) whole
// rows of K words (K >= 32: whole 128-byte lines; K = 256: a 1 KiB row).
// Quad q of row r lives at quad q ^ (r mod K/4) of the row, so the row writes
// (consecutive rows, same q) and the line reads (one row, consecutive q) hit
// distinct banks with no padding.  All lanes take part in the stores; streams
// past the end run on a zero state and are never stored (for V2 these are
// whole groups, so no live stream reads them).
// ------------------------------------------------------------------------
template <int VAR, typename T, int K, int S, bool NT, int XM>
__global__ __launch_bounds__(256) void k_generate_tile(GenArgs a)
{
    HIP_DYNAMIC_SHARED(uint32_t, lds);
    constexpr int QPR = K / 4;               // quads per row
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = ((uint64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
    const uint64_t base = wave * 64u * S;
    uint32_t *tile = lds + (threadIdx.x >> 6) * (64 * S * K);
    // V2 with the LDS exchange: 64 words per slot after all tiles of the block.
    uint32_t *xb = lds + (blockDim.x >> 6) * (64 * S * K) + (threadIdx.x >> 6) * (64 * S);
    const uint64_t n = a.n;

    Stream<VAR, T> st[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const uint64_t s = base + 64u * k + lane;
        if (s < a.ns) st[k].load(a, (uint32_t)s);
        else st[k] = Stream<VAR, T>{};
        st[k].init_exchange(a, lane);
    }
    uint64_t i = 0;
    for (; i + K <= n; i += K) {
#pragma unroll
        for (int q = 0; q < QPR; ++q) {
            uint32_t v[4][S];
            if constexpr (XM == XCH_LDS) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int k = 0; k < S; ++k) v[e][k] = st[k].next_lds(xb + 64 * k, lane);
            } else if constexpr (XM == XCH_BPERM2) {
#pragma unroll
                for (int e = 0; e < 4; e += 2)
#pragma unroll
                    for (int k = 0; k < S; ++k) st[k].next2(v[e][k], v[e + 1][k]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int k = 0; k < S; ++k) v[e][k] = st[k].next();
            }
#pragma unroll
            for (int k = 0; k < S; ++k)
                store4<false>(tile + (64 * k + lane) * K + 4 * (q ^ (lane & (QPR - 1))),
                              v[0][k], v[1][k], v[2][k], v[3][k]);
        }
        __syncthreads();
#pragma unroll 8
        for (int j = 0; j < S * QPR; ++j) {
            const uint32_t Q = j * 64 + lane;
            const uint32_t r = Q / QPR;
            const uint32_t q = Q % QPR;
            uint32_t x0, x1, x2, x3;
            load4(tile + r * K + 4 * (q ^ (r & (QPR - 1))), x0, x1, x2, x3);
            if (base + r < a.ns)
                store4<NT>(a.out + (base + r) * n + i + 4 * q, x0, x1, x2, x3);
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const uint64_t s = base + 64u * k + lane;
        if (s < a.ns) {
            uint32_t *o = a.out + s * n;
            for (uint64_t t = i; t < n; t += 4) {    // n % 4 == 0
                uint32_t v0 = st[k].next(), v1 = st[k].next(), v2 = st[k].next(), v3 = st[k].next();
                store4<NT>(o + t, v0, v1, v2, v3);
            }
            st[k].save(a, (uint32_t)s);
        }
    }
}

// ------------------------------------------------------------------------
// Persistent pipelined tile kernel (ST_PIPE, ST_PIPE_NT): one wave per
// workgroup and gridDim.x workgroups, which take 64-stream blocks in address
// order (block b, b + gridDim.x, ...), so the rows written at any moment are
// neighbours in memory and the set of open DRAM pages stays small with only
// a few waves per CU.  Two LDS tiles alternate: while round r is generated
// into one, round r-1 is stored from the other, one store instruction per
// generated quad, so a wave's VALU work overlaps its own stores.  Store
// instruction j of a round covers rows j*RPI .. j*RPI+RPI-1 (RPI = 64/(K/4)).
// ------------------------------------------------------------------------
template <int VAR, typename T, int K, bool NT, int XM>
__global__ __launch_bounds__(64) void k_generate_pipe(GenArgs a)
{
    HIP_DYNAMIC_SHARED(uint32_t, lds);
    constexpr int QPR = K / 4;
    constexpr int RPI = 64 / QPR;
    static_assert(K >= 16 && QPR <= 64 && 64 % QPR == 0, "K must divide 256");
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t q = lane % QPR;
    const uint32_t rsub = lane / QPR;
    uint32_t *xb = lds + 2 * 64 * K;         // V2 with the LDS exchange
    const uint64_t n = a.n;
    const uint64_t rounds = n / K;
    // The host launches this kernel only when a 64-stream block spans fewer
    // than 2^32 words (n < 2^26), so in-block offsets fit 32 bits and every
    // store is a uniform block base plus a 32-bit lane offset.
    const uint32_t jstride = (uint32_t)(RPI * n);  // words between store instructions' rows
    const uint32_t nblk = (a.ns + 63u) / 64u;
    for (uint32_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const uint64_t base = (uint64_t)blk * 64u;
        const uint64_t s = base + lane;
        Stream<VAR, T> st;
        if (s < a.ns) st.load(a, (uint32_t)s);
        else st = Stream<VAR, T>{};
        st.init_exchange(a, lane);
        const uint32_t nrows = (a.ns - base) < 64u ? (uint32_t)(a.ns - base) : 64u;
        gu32 *blk_out = gptr((uint64_t)(uintptr_t)(a.out + base * n));
        const uint32_t lane_off = rsub * (uint32_t)n + 4u * q;
        auto gen_quad = [&](uint32_t *buf, int qq) {
            uint32_t v[4];
            if constexpr (XM == XCH_LDS) {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = st.next_lds(xb, lane);
            } else if constexpr (XM == XCH_BPERM2) {
                st.next2(v[0], v[1]);
                st.next2(v[2], v[3]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = st.next();
            }
            store4<false>(buf + lane * K + 4 * (qq ^ (lane & (QPR - 1))), v[0], v[1], v[2], v[3]);
        };
        auto put_quad = [&](const uint32_t *buf, int j, uint32_t off) {
            const uint32_t r = j * RPI + rsub;
            uint32_t x0, x1, x2, x3;
            load4(buf + r * K + 4 * (q ^ (r & (QPR - 1))), x0, x1, x2, x3);
            gstore4<NT>(blk_out + (off + (uint32_t)j * jstride), x0, x1, x2, x3);
        };
        // A full block runs the pipelined rounds; the last block of a launch
        // whose stream count is not a multiple of 64 stores per lane (its
        // absent rows' lanes stay inactive; V2 groups are whole, so the
        // present lanes never read an absent lane's word).
        uint64_t t0 = 0;
        if (nrows == 64u && rounds) {
#pragma unroll
            for (int qq = 0; qq < QPR; ++qq) gen_quad(lds, qq);
            __syncthreads();
            for (uint64_t r = 1; r < rounds; ++r) {
                uint32_t *cur = lds + (r & 1u) * (64 * K);
                const uint32_t *prev = lds + ((r - 1) & 1u) * (64 * K);
                const uint32_t off = lane_off + (uint32_t)(r - 1) * K;
#pragma unroll
                for (int qq = 0; qq < QPR; ++qq) {
                    gen_quad(cur, qq);
                    put_quad(prev, qq, off);
                }
                __syncthreads();
            }
            const uint32_t *last = lds + ((rounds - 1) & 1u) * (64 * K);
            const uint32_t off = lane_off + (uint32_t)(rounds - 1) * K;
#pragma unroll
            for (int j = 0; j < QPR; ++j) put_quad(last, j, off);
            __syncthreads();
            t0 = rounds * K;
        }
        if (s < a.ns) {
            uint32_t *o = a.out + s * n;
            for (uint64_t t = t0; t < n; t += 4) {    // n % 4 == 0
                const uint32_t v0 = st.next(), v1 = st.next(), v2 = st.next(), v3 = st.next();
                store4<NT>(o + t, v0, v1, v2, v3);
            }
            st.save(a, (uint32_t)s);
        }
    }
}

// ------------------------------------------------------------------------
// Interleaved-layout tile kernel (ST_ILV_TILE, ST_ILV_TILE_NT), output
// out[i * ns + s].  A workgroup of B threads holds B consecutive streams.
// Each round every thread writes its next K outputs into column t of a K x B
// LDS tile; row k of the tile is step i + k of B neighbouring streams, i.e.
// 4B contiguous bytes of the output, and the rows are stored as 16-byte
// quads, 64 consecutive quads (1 KiB) per store instruction.  Tiles are
// spread over the XCDs in bands (xcd_tile): the workgroups of one XCD run in
// order over neighbouring tiles, so each XCD writes long contiguous fronts of
// every step row.  Needs ns % 4 == 0 and a 16-byte aligned output.
// ------------------------------------------------------------------------
template <int VAR, typename T, int K, int B, bool NT, int XM, bool DB>
__global__ __launch_bounds__(B) void k_generate_ilv(GenArgs a)
{
    HIP_DYNAMIC_SHARED(uint32_t, lds);
    constexpr int QR = B / 4;                // quads per tile row
    constexpr int NBUF = DB ? 2 : 1;         // DB: round r is generated while round r-1 is stored
    static_assert(B >= 256 && (B & (B - 1)) == 0 && K % 4 == 0, "B a power of two >= 256");
    const uint32_t t = threadIdx.x;
    const uint32_t lane = t & 63u;
    const uint64_t ns = a.ns;
    const uint64_t base = (uint64_t)xcd_tile(blockIdx.x, gridDim.x) * B;
    const uint64_t s = base + t;
    uint32_t *xb = lds + NBUF * K * B + (t & ~63u);   // V2 with the LDS exchange: 64 words per wave
    Stream<VAR, T> st;
    if (s < ns) st.load(a, (uint32_t)s);
    else st = Stream<VAR, T>{};
    st.init_exchange(a, lane);
    const uint32_t cq = t % QR;              // quad column this thread stores
    const uint32_t r0 = t / QR;              // its row among each group of B / QR = 4 rows
    const bool col_ok = base + 4u * cq < ns;
    const uint64_t n = a.n;
    gu32 *out = gptr((uint64_t)(uintptr_t)a.out) + base + 4u * cq;
    auto gen4 = [&](uint32_t *buf, int k0) {   // steps k0 .. k0+3 into column t
        uint32_t v[4];
        if constexpr (XM == XCH_LDS) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = st.next_lds(xb, lane);
        } else if constexpr (XM == XCH_BPERM2) {
            st.next2(v[0], v[1]);
            st.next2(v[2], v[3]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = st.next();
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) buf[(k0 + e) * B + t] = v[e];
    };
    auto put = [&](const uint32_t *buf, int j, uint64_t i) {   // rows 4j .. 4j+3 of the tile
        const uint32_t row = 4u * j + r0;
        uint32_t x0, x1, x2, x3;
        load4(buf + row * B + 4u * cq, x0, x1, x2, x3);
        if (col_ok) gstore4<NT>(out + (i + row) * ns, x0, x1, x2, x3);
    };
    uint64_t i = 0;
    if constexpr (DB) {
        const uint64_t rounds = n / K;
        if (rounds) {
#pragma unroll
            for (int k = 0; k < K; k += 4) gen4(lds, k);
            __syncthreads();
            for (uint64_t r = 1; r < rounds; ++r) {
                uint32_t *cur = lds + (r & 1u) * (K * B);
                const uint32_t *prev = lds + ((r - 1) & 1u) * (K * B);
#pragma unroll
                for (int j = 0; j < K / 4; ++j) {
                    gen4(cur, 4 * j);
                    put(prev, j, (r - 1) * K);
                }
                __syncthreads();
            }
            const uint32_t *last = lds + ((rounds - 1) & 1u) * (K * B);
#pragma unroll
            for (int j = 0; j < K / 4; ++j) put(last, j, (rounds - 1) * K);
            i = rounds * K;
        }
    } else {
        for (; i + K <= n; i += K) {
#pragma unroll
            for (int k = 0; k < K; k += 4) gen4(lds, k);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < K / 4; ++j) put(lds, j, i);
            __syncthreads();
        }
    }
    if (s < ns) {                            // whole V2 groups: present lanes read present lanes only
        for (; i < n; ++i) a.out[i * ns + s] = st.next();
        st.save(a, (uint32_t)s);
    }
}

// ------------------------------------------------------------------------
// Consumption kernel: pairs of outputs -> binary32 point in [0,1)^2 -> hit
// count of the unit quarter circle.  Products and the sum are rounded one by
// one (contraction is off for this file).
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t qc_hit(uint32_t r1, uint32_t r2)
{
    const float u = (float)(r1 >> 8) * 0x1p-24f;
    const float v = (float)(r2 >> 8) * 0x1p-24f;
    const float uu = u * u;
    const float vv = v * v;
    const float sum = uu + vv;
    return sum < 1.0f ? 1u : 0u;
}

template <int VAR, typename T, int K>
__global__ __launch_bounds__(256) void k_consume(GenArgs a)
{
    static_assert(K % 2 == 0, "pairs");
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    Stream<VAR, T> st;
    st.load(a, s);
    st.init_exchange(a, lane);
    const uint64_t n = a.n;
    uint64_t total = 0;
    uint64_t i = 0;
    while (i < n) {
        const uint64_t lim = (n - i > (1ull << 30)) ? i + (1ull << 30) : n;
        uint32_t c = 0;
        for (; i + K <= lim; i += K) {
#pragma unroll
            for (int j = 0; j < K; j += 2) {
                const uint32_t r1 = st.next();
                const uint32_t r2 = st.next();
                c += qc_hit(r1, r2);
            }
        }
        for (; i < lim; i += 2) {
            const uint32_t r1 = st.next();
            const uint32_t r2 = st.next();
            c += qc_hit(r1, r2);
        }
        total += c;
    }
    a.counts[s] = total;
    st.save(a, s);
}

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
        s.skip = 0;
    } else {
        // position head + k*chunk: jump by k*chunk, then step head times
        s.pos = seg0 + (uint64_t)(k - 1) * a.chunk;
        const uint64_t left = r.len - s.pos;
        len = left < a.chunk ? left : a.chunk;
        s.head = 0;
        s.poly = a.polys + 5ull * k;
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
    uint32_t qi = 0, base = 0, end = 0;
    while (grab_segments(a, lane, qi, base, end)) {
        const uint32_t idx = base + lane;
        if (idx < end) {
            const Seg d = decode_segment(a, idx);
            const uint32_t *p = a.state + d.stream;
            X128 g{p[0], p[ns], p[2 * ns], p[3 * ns]};
            uint32_t x = p[4 * ns];
            if (d.poly) {
                jump_v0(g, x, d.poly);
                for (uint32_t i = 0; i < d.skip; ++i) x ^= x128_next(g);
            }
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
__global__ __launch_bounds__(64) void k_segments_tile(SegArgs a)
{
    HIP_DYNAMIC_SHARED(uint32_t, lds);
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
            if (d.poly) {
                jump_v0(g, x, d.poly);
                for (uint32_t i = 0; i < d.skip; ++i) x ^= x128_next(g);
            }
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

__global__ void k_commit(uint32_t *state, const uint32_t *state_next, const uint32_t *ids,
                         uint32_t count, uint32_t ns)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t id = ids[i];
#pragma unroll
    for (int k = 0; k < 5; ++k) state[k * (uint64_t)ns + id] = state_next[k * (uint64_t)ns + id];
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

// ------------------------------------------------------------------------
// Dispatch.
// ------------------------------------------------------------------------
template <int VAR, typename T, int K, int MODE>
hipError_t gen_launch(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    const uint32_t grid = (a.ns + c.block - 1) / c.block;
    hipLaunchKernelGGL((k_generate<VAR, T, K, MODE>), dim3(grid), dim3(c.block), 0, st, a);
    return hipGetLastError();
}

template <int VAR, typename T, int K, int S, bool NT>
hipError_t tile_launch(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    const uint64_t waves = ((uint64_t)a.ns + 64u * S - 1) / (64u * S);
    const uint32_t wpb = c.block / 64;
    const uint32_t grid = (uint32_t)((waves + wpb - 1) / wpb);
    size_t lds = (size_t)wpb * 64 * S * K * sizeof(uint32_t);
    const int xm = (VAR == 2) ? (int)c.exchange : XCH_BPERM;
    if (xm == XCH_LDS) lds += (size_t)wpb * 64 * S * sizeof(uint32_t);
    if (lds > kMaxLdsBytes) return hipErrorInvalidValue;   // the host keeps tiles within a workgroup's LDS
    if (c.lds_bytes > lds) lds = c.lds_bytes;
    if constexpr (VAR == 2) {
        if (xm == XCH_LDS)
            hipLaunchKernelGGL((k_generate_tile<VAR, T, K, S, NT, XCH_LDS>), dim3(grid), dim3(c.block), lds, st, a);
        else if (xm == XCH_BPERM2)
            hipLaunchKernelGGL((k_generate_tile<VAR, T, K, S, NT, XCH_BPERM2>), dim3(grid), dim3(c.block), lds, st, a);
        else
            hipLaunchKernelGGL((k_generate_tile<VAR, T, K, S, NT, XCH_BPERM>), dim3(grid), dim3(c.block), lds, st, a);
    } else {
        hipLaunchKernelGGL((k_generate_tile<VAR, T, K, S, NT, XCH_BPERM>), dim3(grid), dim3(c.block), lds, st, a);
    }
    return hipGetLastError();
}

template <int VAR, typename T, int K, bool NT>
hipError_t tile_by_slots(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    switch (c.slots) {
    case 1: return tile_launch<VAR, T, K, 1, NT>(a, c, st);
    case 2: return tile_launch<VAR, T, K, 2, NT>(a, c, st);
    case 4: if constexpr (K <= 128) return tile_launch<VAR, T, K, 4, NT>(a, c, st); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <int VAR, typename T, int K, bool NT>
hipError_t pipe_launch(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    const uint32_t nblk = (a.ns + 63u) / 64u;
    uint32_t grid = c.grid ? c.grid : nblk;
    if (grid > nblk) grid = nblk;
    if (a.n >= (1ull << 26)) return hipErrorInvalidValue;   // in-block offsets are 32-bit
    const int xm = (VAR == 2) ? (int)c.exchange : XCH_BPERM;
    const size_t lds = (size_t)2 * 64 * K * sizeof(uint32_t) + (xm == XCH_LDS ? 64 * sizeof(uint32_t) : 0);
    if (lds > kMaxLdsBytes) return hipErrorInvalidValue;   // the host keeps both tiles within a workgroup's LDS
    if constexpr (VAR == 2) {
        if (xm == XCH_LDS)
            hipLaunchKernelGGL((k_generate_pipe<VAR, T, K, NT, XCH_LDS>), dim3(grid), dim3(64), lds, st, a);
        else if (xm == XCH_BPERM2)
            hipLaunchKernelGGL((k_generate_pipe<VAR, T, K, NT, XCH_BPERM2>), dim3(grid), dim3(64), lds, st, a);
        else
            hipLaunchKernelGGL((k_generate_pipe<VAR, T, K, NT, XCH_BPERM>), dim3(grid), dim3(64), lds, st, a);
    } else {
        hipLaunchKernelGGL((k_generate_pipe<VAR, T, K, NT, XCH_BPERM>), dim3(grid), dim3(64), lds, st, a);
    }
    return hipGetLastError();
}

template <int VAR, typename T, int K, bool NT>
hipError_t ilv_launch(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    const int xm = (VAR == 2) ? (int)c.exchange : XCH_BPERM;
    const bool db = c.slots == 2;            // interleaved tiles: slots = number of tile buffers
    const size_t lds = (size_t)(db ? 2 : 1) * K * c.block * sizeof(uint32_t) +
                       (xm == XCH_LDS ? (size_t)c.block * sizeof(uint32_t) : 0);
    if (lds > kMaxLdsBytes || a.ns % 4u) return hipErrorInvalidValue;
    const uint32_t grid = (a.ns + c.block - 1) / c.block;
#define ILV(B, X, D) hipLaunchKernelGGL((k_generate_ilv<VAR, T, K, B, NT, X, D>), dim3(grid), dim3(B), lds, st, a)
#define ILVB(X, D)                                                   \
    switch (c.block) {                                               \
    case 256: ILV(256, X, D); break;                                 \
    case 512: ILV(512, X, D); break;                                 \
    case 1024: if constexpr (K <= 32) { ILV(1024, X, D); break; } return hipErrorInvalidValue; \
    default: return hipErrorInvalidValue;                            \
    }
#define ILVX(X) if (db) { ILVB(X, true) } else { ILVB(X, false) }
    if constexpr (VAR == 2) {
        if (xm == XCH_LDS) { ILVX(XCH_LDS) }
        else if (xm == XCH_BPERM2) { ILVX(XCH_BPERM2) }
        else { ILVX(XCH_BPERM) }
    } else {
        ILVX(XCH_BPERM)
    }
#undef ILVX
#undef ILVB
#undef ILV
    return hipGetLastError();
}

template <int VAR, typename T, int K>
hipError_t gen_by_mode(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    constexpr bool small = K <= 32;          // per-lane register tiles
    switch (c.store) {
    case ST_DIRECT: if constexpr (small) return gen_launch<VAR, T, K, ST_DIRECT>(a, c, st); break;
    case ST_DIRECT_NT: if constexpr (small) return gen_launch<VAR, T, K, ST_DIRECT_NT>(a, c, st); break;
    case ST_LDS: if constexpr (K >= 16) return tile_by_slots<VAR, T, K, false>(a, c, st); break;
    case ST_LDS_NT: if constexpr (K >= 16) return tile_by_slots<VAR, T, K, true>(a, c, st); break;
    case ST_INTERLEAVED: if constexpr (small) return gen_launch<VAR, T, K, ST_INTERLEAVED>(a, c, st); break;
    case ST_GENERIC: if constexpr (small) return gen_launch<VAR, T, K, ST_GENERIC>(a, c, st); break;
    case ST_ILV_TILE: if constexpr (K >= 8 && K <= 64) return ilv_launch<VAR, T, K, false>(a, c, st); break;
    case ST_ILV_TILE_NT: if constexpr (K >= 8 && K <= 64) return ilv_launch<VAR, T, K, true>(a, c, st); break;
    case ST_PIPE: if constexpr (K >= 16) return pipe_launch<VAR, T, K, false>(a, c, st); break;
    case ST_PIPE_NT: if constexpr (K >= 16) return pipe_launch<VAR, T, K, true>(a, c, st); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <int VAR, typename T>
hipError_t gen_by_unroll(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    // Modes that need K <= 32 fall back to K = 32 when a larger K is asked.
    const bool lds_mode = c.store == ST_LDS || c.store == ST_LDS_NT || c.store == ST_PIPE || c.store == ST_PIPE_NT ||
                          c.store == ST_ILV_TILE || c.store == ST_ILV_TILE_NT;
    const uint32_t k = (!lds_mode && c.unroll > 32) ? 32 : c.unroll;
    switch (k) {
    case 8: return gen_by_mode<VAR, T, 8>(a, c, st);
    case 16: return gen_by_mode<VAR, T, 16>(a, c, st);
    case 32: return gen_by_mode<VAR, T, 32>(a, c, st);
    case 64: return gen_by_mode<VAR, T, 64>(a, c, st);
    case 128: return gen_by_mode<VAR, T, 128>(a, c, st);
    case 256: return gen_by_mode<VAR, T, 256>(a, c, st);
    default: return hipErrorInvalidValue;
    }
}

template <int VAR, typename T>
hipError_t consume_by_unroll(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    const uint32_t grid = (a.ns + c.block - 1) / c.block;
    switch (c.unroll) {
    case 8: hipLaunchKernelGGL((k_consume<VAR, T, 8>), dim3(grid), dim3(c.block), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_consume<VAR, T, 16>), dim3(grid), dim3(c.block), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_consume<VAR, T, 32>), dim3(grid), dim3(c.block), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_generate(const GenArgs &a, int variant, int w32, const LaunchCfg &c, hipStream_t st)
{
    const uint32_t max_block = (c.store == ST_ILV_TILE || c.store == ST_ILV_TILE_NT) ? 1024u : 256u;
    if (c.block == 0 || c.block % 64 != 0 || c.block > max_block) return hipErrorInvalidValue;
    switch (variant) {
    case 0: return gen_by_unroll<0, uint32_t>(a, c, st);
    case 1: return w32 ? gen_by_unroll<1, uint32_t>(a, c, st) : gen_by_unroll<1, uint64_t>(a, c, st);
    case 2: return gen_by_unroll<2, uint32_t>(a, c, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_consume(const GenArgs &a, int variant, int w32, const LaunchCfg &c, hipStream_t st)
{
    if (c.block == 0 || c.block % 64 != 0 || c.block > 256) return hipErrorInvalidValue;
    switch (variant) {
    case 0: return consume_by_unroll<0, uint32_t>(a, c, st);
    case 1: return w32 ? consume_by_unroll<1, uint32_t>(a, c, st) : consume_by_unroll<1, uint64_t>(a, c, st);
    case 2: return consume_by_unroll<2, uint32_t>(a, c, st);
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

hipError_t launch_commit(uint32_t *state, const uint32_t *state_next, const uint32_t *ids,
                         uint32_t count, uint32_t ns, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_commit, dim3((count + 255) / 256), dim3(256), 0, st, state, state_next, ids, count, ns);
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
