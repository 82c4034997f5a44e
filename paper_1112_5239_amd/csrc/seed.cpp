// seed.cpp -- stream initialisation on the host.
//
// The paper fills each GPU thread's generator parameters on the CPU with the
// ISAAC generator (Section 6.1).  This library uses SplitMix64 (Steele, Lea,
// Flood 2014): a 64-bit counter advanced by the odd integer nearest
// 2^64/phi, each value passed through a two-multiply mixing function.  The
// counter of stream s under base seed sigma starts at sigma * 2^32 + s.
#include <cstring>

#include "host.h"

namespace cprng_impl {

namespace {

struct SplitMix64 {
    uint64_t ctr;
    uint64_t next()
    {
        ctr += 0x9E3779B97F4A7C15ull;
        uint64_t z = ctr;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint32_t next32() { return (uint32_t)next(); }
};

}  // namespace

int words_per_stream(int variant)
{
    switch (variant) {
    case CPRNG_V0_PLAIN: return 5;
    case CPRNG_V1_NAIVE3: return 23;
    case CPRNG_V2_SHMEM: return 6;
    case CPRNG_V3_BBS: return 10;
    case CPRNG_V4_XOR64: return 4;
    default: return -1;
    }
}

// Draw order per stream:
//   V0/V2: xor128 words x,y,z,w (all four redrawn while all are zero), the
//          chaotic state x, then for V2 the initial mixed word.
//   V1   : xorshift word (redrawn while zero), xor128 x,y,z,w (redrawn while
//          all zero), xorwow x,y,z,w,v (redrawn while all zero), xorwow d,
//          then x.  With 32-bit words each draw keeps its low half.
//   V3   : for BBS slots 1..8, r = draw mod M (redrawn while r < 2 or r shares
//          a factor with M), state r^2 mod M; then x, then the initial mixed
//          word.
//   V4   : xor64 word (redrawn while zero), x, then the initial mixed word.
void seed_streams(int variant, bool w32, uint64_t sigma, uint64_t first, uint64_t count,
                  uint32_t *aos)
{
    std::vector<uint64_t> ctr(count);
    for (uint64_t k = 0; k < count; ++k) ctr[k] = (sigma << 32) + first + k;
    seed_streams_at(variant, w32, ctr.data(), count, aos);
}

void seed_streams_at(int variant, bool w32, const uint64_t *counters, uint64_t count, uint32_t *aos)
{
    const int nw = words_per_stream(variant);
    const uint64_t mask = w32 ? 0xFFFFFFFFull : ~0ull;
    for (uint64_t k = 0; k < count; ++k) {
        SplitMix64 r{counters[k]};
        uint32_t *st = aos + k * (uint64_t)nw;
        std::memset(st, 0, sizeof(uint32_t) * nw);
        if (variant == CPRNG_V3_BBS) {
            for (int k = 0; k < 8; ++k) {
                const uint64_t M = kBbsModuli[k];
                uint64_t v;
                for (;;) {
                    v = r.next() % M;
                    uint64_t a = v, b = M;        // gcd(v, M)
                    while (b) { const uint64_t t = a % b; a = b; b = t; }
                    if (v >= 2 && a == 1) break;
                }
                st[k] = (uint32_t)(v * v % M);
            }
            st[8] = r.next32();
            st[9] = r.next32();
        } else if (variant == CPRNG_V4_XOR64) {
            uint64_t y;
            do { y = r.next(); } while (y == 0);
            st[0] = (uint32_t)y;
            st[1] = (uint32_t)(y >> 32);
            st[2] = r.next32();
            st[3] = r.next32();
        } else if (variant == CPRNG_V0_PLAIN || variant == CPRNG_V2_SHMEM) {
            uint32_t w[4];
            do {
                for (int j = 0; j < 4; ++j) w[j] = r.next32();
            } while ((w[0] | w[1] | w[2] | w[3]) == 0u);
            std::memcpy(st, w, sizeof w);
            st[4] = r.next32();
            if (variant == CPRNG_V2_SHMEM) st[5] = r.next32();
        } else {
            uint64_t words64[11];
            do { words64[0] = r.next() & mask; } while (words64[0] == 0);
            do {
                for (int j = 1; j <= 4; ++j) words64[j] = r.next() & mask;
            } while ((words64[1] | words64[2] | words64[3] | words64[4]) == 0);
            do {
                for (int j = 5; j <= 9; ++j) words64[j] = r.next() & mask;
            } while ((words64[5] | words64[6] | words64[7] | words64[8] | words64[9]) == 0);
            words64[10] = r.next() & mask;
            for (int j = 0; j < 11; ++j) {
                st[2 * j] = (uint32_t)words64[j];
                st[2 * j + 1] = (uint32_t)(words64[j] >> 32);
            }
            st[22] = r.next32();
        }
    }
}

// The paper leaves the combination arrays of Algorithm 4 unspecified.  The
// library's default: Fisher-Yates shuffles of [0,C) (j from C-1 down to 1,
// swap j with draw mod (j+1)), comb1 then comb2, from one SplitMix64
// counter starting at 2^64-1; the pair is redrawn (continuing the same
// counter) until every thread mixes two distinct other threads.
bool default_combs(uint32_t C, uint32_t *comb1, uint32_t *comb2)
{
    if (C < 3) return false;
    SplitMix64 r{~0ull};
    for (int attempt = 0; attempt < 1000000; ++attempt) {
        uint32_t *arr[2] = {comb1, comb2};
        for (uint32_t *a : arr) {
            for (uint32_t j = 0; j < C; ++j) a[j] = j;
            for (uint32_t j = C - 1; j >= 1; --j) {
                const uint32_t k = (uint32_t)(r.next() % (uint64_t)(j + 1));
                const uint32_t t = a[j];
                a[j] = a[k];
                a[k] = t;
            }
        }
        bool ok = true;
        for (uint32_t j = 0; j < C && ok; ++j)
            ok = comb1[j] != j && comb2[j] != j && comb1[j] != comb2[j];
        if (ok) return true;
    }
    return false;
}

// The paper leaves Algorithm 5's 16 arrangement arrays unspecified.  The
// library's default: arrays 0..15 in turn, each a Fisher-Yates shuffle of
// [0,C) from one SplitMix64 counter starting at 2^64-2, reshuffled
// (continuing the counter) until no entry maps to itself.
bool default_bbs_combs(uint32_t C, uint32_t *out)
{
    if (C < 3) return false;
    SplitMix64 r{~0ull - 1ull};
    for (int a = 0; a < 16; ++a) {
        uint32_t *arr = out + (size_t)a * C;
        bool ok = false;
        for (int attempt = 0; attempt < 1000000 && !ok; ++attempt) {
            for (uint32_t j = 0; j < C; ++j) arr[j] = j;
            for (uint32_t j = C - 1; j >= 1; --j) {
                const uint32_t k = (uint32_t)(r.next() % (uint64_t)(j + 1));
                const uint32_t t = arr[j];
                arr[j] = arr[k];
                arr[k] = t;
            }
            ok = true;
            for (uint32_t j = 0; j < C && ok; ++j) ok = arr[j] != j;
        }
        if (!ok) return false;
    }
    return true;
}

}  // namespace cprng_impl
