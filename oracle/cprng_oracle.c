/*
 * cprng_oracle.c -- CPU oracle for the chaotic-iteration PRNG hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links, loads or calls it, and it shares no code,
 * header, table or constant generator with the product library.
 *
 * Paper: Bahi, Couturier, Guyeux, Heam, "Efficient and Cryptographically
 * Secure Generation of Chaotic Pseudorandom Numbers on GPU" (arXiv 1112.5239).
 *
 * What is computed (each function below cites the passage it follows):
 *   - the chaotic-iteration step with vectorial negation, x^n = x^{n-1} xor S^n
 *     (Section 4.2, Eq. "Oplus" and the general chaotic iterations that follow);
 *   - strategy words S^n from Marsaglia xor-like generators (Algorithm 2 of
 *     Section 4.1; the xorshift / xor128 / xorwow trio of Listing 1, Section 5);
 *   - three variants:
 *       V0 PLAIN  : one xor128 with 32-bit words as the strategy (Section 5,
 *                   first idea; the object X of Section 8; Algorithm 4 with the
 *                   neighbour exchange removed),
 *       V1 NAIVE3 : Listing 1 per stream (Algorithm 3 of Section 6.1),
 *       V2 SHMEM  : Algorithm 4 of Section 6.2 (xor128 per thread, mixed with
 *                   two neighbours' previous words through a combination array);
 *       V3 BBS    : Algorithm 5 of Section 9.1 (the strategy word assembled from
 *                   eight small Blum-Blum-Shub generators, mixed with two
 *                   neighbours' previous words as in Algorithm 4);
 *       V4 XOR64  : Algorithm 4 with Marsaglia's xor64 as the per-thread
 *                   generator, the generator Section 7 names for the
 *                   optimized versions measured in its first figure;
 *     and, for V1, the xor64 alternative for Listing 1's "xorshift" (flag
 *     ORC_F_XOR64);
 *   - the in-kernel consumption mode (quarter-circle hit counts), a use of the
 *     numbers in the spirit of the "versions without storage" of Section 7.
 *
 * Readings where the paper is silent or ambiguous (kept identical to the
 * library's documented contract):
 *   - seeding: SplitMix64 (Steele, Lea, Flood 2014) stands in for the ISAAC
 *     initialiser of Section 6.1; stream s of base seed sigma starts its draw
 *     counter at sigma*2^32 + s;
 *   - Listing 1 uses 64-bit words (its text calls the three generators 64-bit);
 *     a 32-bit-word variant (W=32) is kept as an option;
 *   - the Listing 1 "xorshift" is the shift triple (13,17,5) of Algorithm 2;
 *   - Algorithm 4 reads the neighbours' words of the previous step (all threads
 *     of a group read, then all write), group size C = 32, combination arrays
 *     drawn by Fisher-Yates from SplitMix64 as in orc_comb_tables();
 *   - outputs are stream-major: out[s*n + i] (the printed index collides);
 *   - Algorithm 5: the eight moduli of orc_bbs_moduli() (products of two
 *     primes = 3 mod 4 near 256, each below 2^16 so squares fit 32 bits), one
 *     per BBS slot; the second array index "8+bbs2&7" read as 8 + (bbs2 & 7);
 *     the sixteen arrangement arrays drawn as in orc_bbs_comb_tables(); the
 *     arrays are chosen once per call from the slot-1 and slot-2 states at
 *     the start of the call, and the slot states rotate (slot k -> k+1, 8 ->
 *     1) at the end of every call that produces outputs;
 *   - xor64 is the 64-bit xorshift with triple (13,7,17) (left, right, left),
 *     one of Marsaglia's full-period 64-bit triples; V4's 32-bit word is the
 *     xor of the two 32-bit halves of each 64-bit output, the convention
 *     Listing 1 applies to its 64-bit generators.
 *
 * Parity unpinned: the order in which the seeding draws fill the state
 * words; everything else is pinned by the test suite (SplitMix64 and xor64 by
 * their published outputs: from state 0, and from Marsaglia's example seed).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>


#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

enum { ORC_V0 = 0, ORC_V1 = 1, ORC_V2 = 2, ORC_V3 = 3, ORC_V4 = 4 };
/* V1 modifier: xor64 (13,7,17) in place of the (13,17,5) triple as the first
 * generator of Listing 1 (64-bit words only). */
#define ORC_F_XOR64 0x100

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): a counter that advances by  */
/* the odd integer nearest 2^64/phi, followed by a mixing finaliser.         */
/* ------------------------------------------------------------------------ */
#define ORC_SM64_GAMMA 0x9E3779B97F4A7C15ull

uint64_t orc_sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t sm64_draw(uint64_t *ctr)
{
    *ctr += ORC_SM64_GAMMA;
    return orc_sm64_mix(*ctr);
}

/* n consecutive draws starting from counter value z (test helper). */
void orc_sm64_draws(uint64_t z, uint64_t n, uint64_t *out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = sm64_draw(&z);
}

static uint64_t wmask(int W) { return W == 64 ? ~0ull : ((1ull << W) - 1ull); }

/* ------------------------------------------------------------------------ */
/* Strategy generators on W-bit words (W = 32 or 64).  Shifts discard the    */
/* bits pushed out of the word; every operation is taken modulo 2^W.         */
/* ------------------------------------------------------------------------ */

/* One xorshift round with shift triple (a,b,c): Algorithm 2 (Section 4.1)
 * is the case (13,17,5) on a 32-bit word.  Returns the new word. */
uint64_t orc_xs_step(uint64_t *y, int a, int b, int c, int W)
{
    uint64_t m = wmask(W);
    uint64_t z = *y & m;
    z = z ^ ((z << a) & m);
    z = z ^ (z >> b);
    z = z ^ ((z << c) & m);
    *y = z;
    return z;
}

/* Marsaglia's xor128 (the generator named for Algorithm 4 in Section 6.2 and
 * as the second generator of Listing 1).  s = {x,y,z,w}; returns new w. */
uint64_t orc_x128_step(uint64_t s[4], int W)
{
    uint64_t m = wmask(W);
    uint64_t t = s[0] ^ ((s[0] << 11) & m);
    s[0] = s[1];
    s[1] = s[2];
    s[2] = s[3];
    s[3] = (s[3] ^ (s[3] >> 19)) ^ (t ^ (t >> 8));
    return s[3];
}

/* Marsaglia's xor64: the 64-bit xorshift with triple (13,7,17), named by
 * Section 7 as the generator of the optimized versions.  Returns the new
 * word. */
uint64_t orc_xor64_step(uint64_t *y) { return orc_xs_step(y, 13, 7, 17, 64); }

/* Marsaglia's xorwow (third generator of Listing 1).  s = {x,y,z,w,v,d};
 * returns d + v after the Weyl increment of d. */
uint64_t orc_xwow_step(uint64_t s[6], int W)
{
    uint64_t m = wmask(W);
    uint64_t t = s[0] ^ (s[0] >> 2);
    s[0] = s[1];
    s[1] = s[2];
    s[2] = s[3];
    s[3] = s[4];
    s[4] = (s[4] ^ ((s[4] << 4) & m)) ^ (t ^ ((t << 1) & m));
    s[5] = (s[5] + 362437ull) & m;
    return (s[5] + s[4]) & m;
}

/* n consecutive outputs of one generator from a given state (test helper).
 * kind: 0 = xorshift(13,17,5), 1 = xor128, 2 = xorwow, 3 = xor64 (W = 64
 * only).  State is updated. */
int orc_gen_outputs(int kind, int W, uint64_t *state, uint64_t n, uint64_t *out)
{
    if (W != 32 && W != 64) return ORC_EINVAL;
    for (uint64_t i = 0; i < n; ++i) {
        if (kind == 0)      out[i] = orc_xs_step(state, 13, 17, 5, W);
        else if (kind == 1) out[i] = orc_x128_step(state, W);
        else if (kind == 2) out[i] = orc_xwow_step(state, W);
        else if (kind == 3 && W == 64) out[i] = orc_xor64_step(state);
        else return ORC_EINVAL;
    }
    return ORC_OK;
}

/* Orbit length of Algorithm 2 from seed y0 on 32-bit words: steps until the
 * word returns to y0, capped at limit.  *hit_zero is set if 0 is visited. */
uint64_t orc_xs32_orbit(uint32_t y0, uint64_t limit, int *hit_zero)
{
    uint64_t y = y0, n = 0;
    *hit_zero = 0;
    do {
        orc_xs_step(&y, 13, 17, 5, 32);
        ++n;
        if (y == 0) *hit_zero = 1;
    } while (y != y0 && n < limit);
    return n;
}

/* ------------------------------------------------------------------------ */
/* The chaotic-iteration step (Section 4.2).  With f the vectorial negation,  */
/* component k of x changes iff bit k of the strategy word S is 1, which is   */
/* the bitwise exclusive or of Eq. (Oplus).                                   */
/* ------------------------------------------------------------------------ */
uint32_t orc_ci_step(uint32_t x, uint32_t S) { return x ^ S; }

void orc_ci_step_batch(const uint32_t *x, const uint32_t *S, uint32_t *out, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = orc_ci_step(x[i], S[i]);
}

/* ------------------------------------------------------------------------ */
/* Per-stream state, as 32-bit words (array of structures, stream by stream). */
/*   V0: x128{x,y,z,w}, ci_x                                    (5 words)    */
/*   V2: x128{x,y,z,w}, ci_x, t_prev                            (6 words)    */
/*   V1: xs{lo,hi}, x128{x,y,z,w}{lo,hi}, xwow{x,y,z,w,v,d}{lo,hi}, ci_x     */
/*                                                              (23 words)   */
/*   V3: bbs[8] (slot 1..8), ci_x, t_prev                       (10 words)   */
/*   V4: xor64{lo,hi}, ci_x, t_prev                             (4 words)    */
/* ------------------------------------------------------------------------ */
int orc_state_words(int variant)
{
    if ((variant & ~0xFF) && variant != (ORC_V1 | ORC_F_XOR64)) return ORC_EINVAL;
    switch (variant & 0xFF) {
    case ORC_V0: return 5;
    case ORC_V1: return 23;
    case ORC_V2: return 6;
    case ORC_V3: return 10;
    case ORC_V4: return 4;
    default: return ORC_EINVAL;
    }
}

/* Moduli of the eight BBS of Algorithm 5 (Section 9.1): the paper asks for
 * M = p*q with p, q prime and = 3 mod 4, M < 2^16 so that x^2 fits 32 bits,
 * "primes around 256", and allows a different M per BBS.  Reading: the
 * primes 211, 223, 227, 239, 251 (all = 3 mod 4), eight distinct products. */
static const uint32_t orc_bbs_mod[8] = {251u * 239u, 251u * 227u, 251u * 223u, 251u * 211u,
                                        239u * 227u, 239u * 223u, 239u * 211u, 227u * 223u};

void orc_bbs_moduli(uint32_t out[8])
{
    for (int k = 0; k < 8; ++k) out[k] = orc_bbs_mod[k];
}

/* One BBS step x <- x^2 mod M of slot k (0-based); returns the new state. */
uint32_t orc_bbs_step(uint32_t *x, int k)
{
    *x = (uint32_t)(((uint64_t)*x * (uint64_t)*x) % orc_bbs_mod[k]);
    return *x;
}

static uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

static uint64_t get64(const uint32_t *w, int k) { return (uint64_t)w[2 * k] | ((uint64_t)w[2 * k + 1] << 32); }
static void put64(uint32_t *w, int k, uint64_t v) { w[2 * k] = (uint32_t)v; w[2 * k + 1] = (uint32_t)(v >> 32); }

/* Seed streams first_stream .. first_stream+n_streams-1 of base seed sigma.
 * Draw order: V0/V2 draw the four xor128 words (redrawn together until not
 * all zero), then x, then (V2) the initial neighbour word.  V1 draws the
 * xorshift word (until nonzero), the four xor128 words (until not all zero),
 * the five xorwow words (until not all zero), the Weyl counter d, then x.
 * W = 32 keeps the low 32 bits of each draw (rejection on the kept bits).
 * V3 draws, for slots 1..8 in turn, r = D64 mod M (redrawn until r >= 2 and
 * gcd(r, M) = 1) and keeps r^2 mod M (a quadratic residue coprime to M, the
 * usual BBS start); then x, then the initial neighbour word.  V4 draws the
 * xor64 word (until nonzero), then x, then the initial neighbour word. */
int orc_seed(int variant, int W, uint64_t sigma, uint64_t first_stream,
             uint64_t n_streams, uint32_t *state)
{
    int nw = orc_state_words(variant);
    if (nw < 0 || (W != 32 && W != 64)) return ORC_EINVAL;
    if ((variant & ORC_F_XOR64) && W != 64) return ORC_EINVAL;
    variant &= 0xFF;
    uint64_t m = wmask(W);
    for (uint64_t k = 0; k < n_streams; ++k) {
        uint64_t ctr = (sigma << 32) + (first_stream + k);
        uint32_t *st = state + k * (uint64_t)nw;
        memset(st, 0, sizeof(uint32_t) * (size_t)nw);
        if (variant == ORC_V3) {
            for (int k = 0; k < 8; ++k) {
                uint64_t M = orc_bbs_mod[k], r;
                do { r = sm64_draw(&ctr) % M; } while (r < 2 || gcd64(r, M) != 1);
                st[k] = (uint32_t)((r * r) % M);
            }
            st[8] = (uint32_t)sm64_draw(&ctr);
            st[9] = (uint32_t)sm64_draw(&ctr);
        } else if (variant == ORC_V4) {
            uint64_t y;
            do { y = sm64_draw(&ctr); } while (y == 0);
            put64(st, 0, y);
            st[2] = (uint32_t)sm64_draw(&ctr);
            st[3] = (uint32_t)sm64_draw(&ctr);
        } else if (variant == ORC_V0 || variant == ORC_V2) {
            uint32_t a[4];
            do {
                for (int j = 0; j < 4; ++j) a[j] = (uint32_t)sm64_draw(&ctr);
            } while ((a[0] | a[1] | a[2] | a[3]) == 0);
            for (int j = 0; j < 4; ++j) st[j] = a[j];
            st[4] = (uint32_t)sm64_draw(&ctr);
            if (variant == ORC_V2) st[5] = (uint32_t)sm64_draw(&ctr);
        } else {
            uint64_t g1, g2[4], g3[6];
            do { g1 = sm64_draw(&ctr) & m; } while (g1 == 0);
            do {
                for (int j = 0; j < 4; ++j) g2[j] = sm64_draw(&ctr) & m;
            } while ((g2[0] | g2[1] | g2[2] | g2[3]) == 0);
            do {
                for (int j = 0; j < 5; ++j) g3[j] = sm64_draw(&ctr) & m;
            } while ((g3[0] | g3[1] | g3[2] | g3[3] | g3[4]) == 0);
            g3[5] = sm64_draw(&ctr) & m;
            put64(st, 0, g1);
            for (int j = 0; j < 4; ++j) put64(st, 1 + j, g2[j]);
            for (int j = 0; j < 6; ++j) put64(st, 5 + j, g3[j]);
            st[22] = (uint32_t)sm64_draw(&ctr);
        }
    }
    return ORC_OK;
}

/* Combination arrays of Algorithm 4 (Section 6.2).  The paper gives neither C
 * nor the arrays; the reading used here: two permutations of [0,C) drawn by
 * Fisher-Yates (j = C-1 down to 1, swap with index draw mod (j+1)) from a
 * SplitMix64 counter starting at 2^64-1, comb1 then comb2, redrawn (the same
 * draw sequence continuing) until for every j: comb1[j] != j, comb2[j] != j
 * and comb1[j] != comb2[j], so each thread mixes two distinct other threads. */
int orc_comb_tables(uint32_t C, uint32_t *comb1, uint32_t *comb2)
{
    if (C < 3 || C > 4096) return ORC_EINVAL;
    uint64_t ctr = ~0ull;
    for (int attempt = 0; attempt < 1000000; ++attempt) {
        uint32_t *arr[2] = {comb1, comb2};
        for (int a = 0; a < 2; ++a) {
            for (uint32_t j = 0; j < C; ++j) arr[a][j] = j;
            for (uint32_t j = C - 1; j >= 1; --j) {
                uint32_t k = (uint32_t)(sm64_draw(&ctr) % (uint64_t)(j + 1));
                uint32_t tmp = arr[a][j];
                arr[a][j] = arr[a][k];
                arr[a][k] = tmp;
            }
        }
        int ok = 1;
        for (uint32_t j = 0; j < C; ++j)
            if (comb1[j] == j || comb2[j] == j || comb1[j] == comb2[j]) ok = 0;
        if (ok) return ORC_OK;
    }
    return ORC_EINVAL;
}

/* The sixteen arrangement arrays of Algorithm 5 (not given in the paper).
 * Reading: sixteen permutations of [0,C), arrays 0..15 in turn, each drawn by
 * Fisher-Yates as in orc_comb_tables() from one SplitMix64 counter starting
 * at 2^64-2 and redrawn (the sequence continuing) until it has no fixed
 * point, so no thread reads its own word.  out: 16*C entries, array a at
 * out[a*C .. a*C+C-1]. */
int orc_bbs_comb_tables(uint32_t C, uint32_t *out)
{
    if (C < 3 || C > 4096) return ORC_EINVAL;
    uint64_t ctr = ~0ull - 1ull;
    for (int a = 0; a < 16; ++a) {
        uint32_t *arr = out + (size_t)a * C;
        int ok = 0;
        for (int attempt = 0; attempt < 1000000 && !ok; ++attempt) {
            for (uint32_t j = 0; j < C; ++j) arr[j] = j;
            for (uint32_t j = C - 1; j >= 1; --j) {
                uint32_t k = (uint32_t)(sm64_draw(&ctr) % (uint64_t)(j + 1));
                uint32_t tmp = arr[j];
                arr[j] = arr[k];
                arr[k] = tmp;
            }
            ok = 1;
            for (uint32_t j = 0; j < C; ++j)
                if (arr[j] == j) ok = 0;
        }
        if (!ok) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Generation.                                                               */
/* ------------------------------------------------------------------------ */

/* V0: S = xor128 step on 32-bit words; x = x xor S; emit x (Eq. Oplus). */
static void gen_v0_stream(uint32_t *st, uint64_t n, uint32_t *out, uint32_t *strat)
{
    uint64_t g[4] = {st[0], st[1], st[2], st[3]};
    uint32_t x = st[4];
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t S = (uint32_t)orc_x128_step(g, 32);
        x = orc_ci_step(x, S);
        if (out) out[i] = x;
        if (strat) strat[i] = S;
    }
    for (int j = 0; j < 4; ++j) st[j] = (uint32_t)g[j];
    st[4] = x;
}

/* The 32-bit fold of a generator output: its low half xor its high half (the
 * high half is 0 for 32-bit words). */
static uint32_t fold32(uint64_t v) { return (uint32_t)v ^ (uint32_t)(v >> 32); }

/* V1: Listing 1 per stream (Algorithm 3).  Each of the three generators
 * steps once per output, and the strategy word takes every 32-bit half of
 * the three new outputs once under xor: S is the fold of t1 xor t2 xor t3
 * (xor is associative and commutative, so the order in which the listing
 * takes the six halves does not matter).  alt: the first generator is xor64
 * (13,7,17) instead of the (13,17,5) triple. */
static void gen_v1_stream(uint32_t *st, int W, int alt, uint64_t n, uint32_t *out, uint32_t *strat)
{
    uint64_t g1 = get64(st, 0), g2[4], g3[6];
    for (int j = 0; j < 4; ++j) g2[j] = get64(st, 1 + j);
    for (int j = 0; j < 6; ++j) g3[j] = get64(st, 5 + j);
    uint32_t x = st[22];
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t t1 = alt ? orc_xor64_step(&g1) : orc_xs_step(&g1, 13, 17, 5, W);
        const uint64_t t2 = orc_x128_step(g2, W);
        const uint64_t t3 = orc_xwow_step(g3, W);
        const uint32_t S = fold32(t1 ^ t2 ^ t3);
        x = orc_ci_step(x, S);
        if (out) out[i] = x;
        if (strat) strat[i] = S;
    }
    put64(st, 0, g1);
    for (int j = 0; j < 4; ++j) put64(st, 1 + j, g2[j]);
    for (int j = 0; j < 6; ++j) put64(st, 5 + j, g3[j]);
    st[22] = x;
}

/* V2: Algorithm 4 on one group of C consecutive streams.  Thread j of the
 * group reads the words that threads comb1[j] and comb2[j] of the same group
 * produced at the previous step; every thread reads before any writes.
 * out/strat are indexed [j*stride + i]. */
static int gen_v2_group(uint32_t *st, uint32_t C, const uint32_t *comb1, const uint32_t *comb2,
                        uint64_t n, uint32_t *out, uint32_t *strat, uint64_t stride)
{
    uint64_t (*g)[4] = malloc(sizeof(*g) * C);
    uint32_t *tprev = malloc(sizeof(uint32_t) * C);
    uint32_t *tnext = malloc(sizeof(uint32_t) * C);
    uint32_t *u = malloc(sizeof(uint32_t) * C);
    if (!g || !tprev || !tnext || !u) {
        free(g); free(tprev); free(tnext); free(u);
        return ORC_ENOMEM;
    }
    for (uint32_t j = 0; j < C; ++j) {
        for (int k = 0; k < 4; ++k) g[j][k] = st[j * 6 + k];
        tprev[j] = st[j * 6 + 5];
    }
    for (uint64_t i = 0; i < n; ++i) {
        for (uint32_t j = 0; j < C; ++j) u[j] = (uint32_t)orc_x128_step(g[j], 32);
        for (uint32_t j = 0; j < C; ++j) tnext[j] = u[j] ^ tprev[comb1[j]] ^ tprev[comb2[j]];
        for (uint32_t j = 0; j < C; ++j) {
            tprev[j] = tnext[j];
            uint32_t x = orc_ci_step(st[j * 6 + 4], tnext[j]);
            st[j * 6 + 4] = x;
            if (out) out[j * stride + i] = x;
            if (strat) strat[j * stride + i] = tnext[j];
        }
    }
    for (uint32_t j = 0; j < C; ++j) {
        for (int k = 0; k < 4; ++k) st[j * 6 + k] = (uint32_t)g[j][k];
        st[j * 6 + 5] = tprev[j];
    }
    free(g); free(tprev); free(tnext); free(u);
    return ORC_OK;
}

/* V4: Algorithm 4 with xor64 as each thread's generator (Section 7).  The
 * thread's word is the xor of the two 32-bit halves of its xor64 output; the
 * exchange is V2's: thread j mixes the previous-step words of threads
 * comb1[j] and comb2[j] of its group, all reads before any write. */
static int gen_v4_group(uint32_t *st, uint32_t C, const uint32_t *comb1, const uint32_t *comb2,
                        uint64_t n, uint32_t *out, uint32_t *strat, uint64_t stride)
{
    uint64_t *y = malloc(sizeof(uint64_t) * C);
    uint32_t *tprev = malloc(sizeof(uint32_t) * C);
    uint32_t *tnext = malloc(sizeof(uint32_t) * C);
    if (!y || !tprev || !tnext) {
        free(y); free(tprev); free(tnext);
        return ORC_ENOMEM;
    }
    for (uint32_t j = 0; j < C; ++j) {
        y[j] = get64(st + (size_t)j * 4, 0);
        tprev[j] = st[j * 4 + 3];
    }
    for (uint64_t i = 0; i < n; ++i) {
        for (uint32_t j = 0; j < C; ++j) {
            uint64_t v = orc_xor64_step(&y[j]);
            tnext[j] = (uint32_t)v ^ (uint32_t)(v >> 32);
        }
        for (uint32_t j = 0; j < C; ++j) tnext[j] ^= tprev[comb1[j]] ^ tprev[comb2[j]];
        for (uint32_t j = 0; j < C; ++j) {
            tprev[j] = tnext[j];
            uint32_t x = orc_ci_step(st[j * 4 + 2], tnext[j]);
            st[j * 4 + 2] = x;
            if (out) out[j * stride + i] = x;
            if (strat) strat[j * stride + i] = tnext[j];
        }
    }
    for (uint32_t j = 0; j < C; ++j) {
        put64(st + (size_t)j * 4, 0, y[j]);
        st[j * 4 + 3] = tprev[j];
    }
    free(y); free(tprev); free(tnext);
    return ORC_OK;
}

/* Strategy bits of one step of Algorithm 5 for one thread, before the
 * neighbour mixing, as bit fields of the 32-bit word.  Each of the eight BBS
 * gives one output whose low nibble fills a 4-bit field, BBS1's the top one
 * (bits 28..31) down to BBS8's (bits 0..3).  Then BBS3 and BBS7 each give a
 * second output whose low two bits are shift counts s1 and s2 (0..3), and
 * BBS1 and BBS2 a second output whose low s1 and s2 bits fill the vacated
 * places: the word is the nibble word moved up by s1 + s2 bits (its top bits
 * dropped), BBS1's s1 bits at bits s2 .. s2+s1-1 and BBS2's s2 bits at bits
 * 0 .. s2-1.  Slots are stepped in the order the paper's kernel steps them
 * (each slot's own outputs are what matter; slots are independent). */
uint32_t orc_bbs_word(uint32_t b[8])
{
    uint32_t nibbles = 0;
    for (int k = 0; k < 8; ++k) nibbles |= (orc_bbs_step(&b[k], k) & 15u) << (28 - 4 * k);
    const uint32_t s1 = orc_bbs_step(&b[2], 2) & 3u;
    const uint32_t f1 = orc_bbs_step(&b[0], 0) & ((1u << s1) - 1u);
    const uint32_t s2 = orc_bbs_step(&b[6], 6) & 3u;
    const uint32_t f2 = orc_bbs_step(&b[1], 1) & ((1u << s2) - 1u);
    return (nibbles << (s1 + s2)) | (f1 << s2) | f2;
}

/* V3: Algorithm 5 on one group of C consecutive streams (10-word states).
 * At the start of the call thread j takes o1 from array (bbs1 & 7) and o2
 * from array 8 + (bbs2 & 7); each step it mixes its strategy bits with the
 * previous words of threads o1, o2 of the group (all read before any write),
 * x = x xor t; at the end of a call with outputs the slot states rotate. */
static int gen_v3_group(uint32_t *st, uint32_t C, const uint32_t *combs, uint64_t n, uint32_t *out,
                        uint32_t *strat, uint64_t stride)
{
    uint32_t *o1 = malloc(sizeof(uint32_t) * C), *o2 = malloc(sizeof(uint32_t) * C);
    uint32_t *tprev = malloc(sizeof(uint32_t) * C), *tnext = malloc(sizeof(uint32_t) * C);
    if (!o1 || !o2 || !tprev || !tnext) {
        free(o1); free(o2); free(tprev); free(tnext);
        return ORC_ENOMEM;
    }
    for (uint32_t j = 0; j < C; ++j) {
        const uint32_t *s = st + (size_t)j * 10;
        o1[j] = combs[(size_t)(s[0] & 7u) * C + j];
        o2[j] = combs[(size_t)(8u + (s[1] & 7u)) * C + j];
        tprev[j] = s[9];
    }
    for (uint64_t i = 0; i < n; ++i) {
        for (uint32_t j = 0; j < C; ++j) tnext[j] = orc_bbs_word(st + (size_t)j * 10);
        for (uint32_t j = 0; j < C; ++j) tnext[j] ^= tprev[o1[j]] ^ tprev[o2[j]];
        for (uint32_t j = 0; j < C; ++j) {
            tprev[j] = tnext[j];
            uint32_t x = orc_ci_step(st[(size_t)j * 10 + 8], tnext[j]);
            st[(size_t)j * 10 + 8] = x;
            if (out) out[j * stride + i] = x;
            if (strat) strat[j * stride + i] = tnext[j];
        }
    }
    for (uint32_t j = 0; j < C; ++j) {
        uint32_t *s = st + (size_t)j * 10;
        if (n > 0) {
            uint32_t last = s[7];
            for (int k = 7; k > 0; --k) s[k] = s[k - 1];
            s[0] = last;
        }
        s[9] = tprev[j];
    }
    free(o1); free(o2); free(tprev); free(tnext);
    return ORC_OK;
}

/* Generate n outputs per stream for n_streams streams whose states are in
 * `state` (updated in place, so a second call continues the streams).
 * out (optional) and strat (optional, the strategy words S^n) are
 * stream-major: [s*n + i].  V2 and V4 need n_streams % C == 0 and the two
 * combination arrays; V3 needs n_streams % C == 0 and the sixteen arrays of
 * orc_bbs_comb_tables() in comb1 (16*C entries; comb2 unused); W only
 * matters for V1.  One call is one call of the paper's kernel (V3 chooses its
 * arrays at the start and rotates its slots at the end). */
int orc_generate(int variant, int W, uint64_t n_streams, uint32_t *state, uint64_t n,
                 uint32_t *out, uint32_t *strat, uint32_t C,
                 const uint32_t *comb1, const uint32_t *comb2)
{
    int nw = orc_state_words(variant);
    if (nw < 0 || (W != 32 && W != 64)) return ORC_EINVAL;
    const int alt = (variant & ORC_F_XOR64) != 0;
    if (alt && W != 64) return ORC_EINVAL;
    variant &= 0xFF;
    if (variant == ORC_V0) {
        for (uint64_t s = 0; s < n_streams; ++s)
            gen_v0_stream(state + s * 5, n, out ? out + s * n : NULL, strat ? strat + s * n : NULL);
    } else if (variant == ORC_V1) {
        for (uint64_t s = 0; s < n_streams; ++s)
            gen_v1_stream(state + s * 23, W, alt, n, out ? out + s * n : NULL, strat ? strat + s * n : NULL);
    } else if (variant == ORC_V3) {
        if (C == 0 || !comb1 || n_streams % C != 0) return ORC_EINVAL;
        for (uint32_t j = 0; j < 16 * C; ++j)
            if (comb1[j] >= C) return ORC_EINVAL;
        for (uint64_t g0 = 0; g0 < n_streams; g0 += C) {
            int rc = gen_v3_group(state + g0 * 10, C, comb1, n, out ? out + g0 * n : NULL,
                                  strat ? strat + g0 * n : NULL, n);
            if (rc) return rc;
        }
    } else {
        if (C == 0 || !comb1 || !comb2 || n_streams % C != 0) return ORC_EINVAL;
        for (uint32_t j = 0; j < C; ++j)
            if (comb1[j] >= C || comb2[j] >= C) return ORC_EINVAL;
        for (uint64_t g0 = 0; g0 < n_streams; g0 += C) {
            int rc = variant == ORC_V4
                ? gen_v4_group(state + g0 * 4, C, comb1, comb2, n,
                               out ? out + g0 * n : NULL, strat ? strat + g0 * n : NULL, n)
                : gen_v2_group(state + g0 * 6, C, comb1, comb2, n,
                               out ? out + g0 * n : NULL, strat ? strat + g0 * n : NULL, n);
            if (rc) return rc;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* In-kernel consumption: quarter-circle hit counts.                          */
/* Outputs 2k and 2k+1 of a stream form a pair (r1, r2); each is turned into  */
/* a float in [0,1) from its top 24 bits, u = (r >> 8) * 2^-24 (exact), and   */
/* the pair is a hit iff fl(fl(u*u) + fl(v*v)) < 1 in IEEE binary32 with      */
/* round-to-nearest-even and no fused multiply-add.                           */
/* ------------------------------------------------------------------------ */
static uint64_t count_hits(const uint32_t *r, uint64_t n)
{
    uint64_t hits = 0;
    for (uint64_t k = 0; k + 1 < n; k += 2) {
        float u = (float)(r[k] >> 8) * 0x1p-24f;
        float v = (float)(r[k + 1] >> 8) * 0x1p-24f;
        float uu = u * u;
        float vv = v * v;
        float s = uu + vv;
        if (s < 1.0f) ++hits;
    }
    return hits;
}

/* counts[s] = hits among the n/2 pairs of stream s's next n outputs; the
 * states advance by n exactly as orc_generate would.  n must be even. */
int orc_consume_qc(int variant, int W, uint64_t n_streams, uint32_t *state, uint64_t n,
                   uint64_t *counts, uint32_t C, const uint32_t *comb1, const uint32_t *comb2)
{
    int nw = orc_state_words(variant);
    if (nw < 0 || (n & 1)) return ORC_EINVAL;
    const int base = variant & 0xFF;
    uint64_t group = (base == ORC_V2 || base == ORC_V3 || base == ORC_V4) ? C : 1;
    if (group == 0 || n_streams % group != 0) return ORC_EINVAL;
    uint64_t words = group * n;
    uint32_t *buf = malloc(sizeof(uint32_t) * (size_t)(words > 0 ? words : 1));
    if (!buf) return ORC_ENOMEM;
    for (uint64_t g0 = 0; g0 < n_streams; g0 += group) {
        int rc = orc_generate(variant, W, group, state + g0 * (uint64_t)nw, n, buf, NULL, C, comb1, comb2);
        if (rc) { free(buf); return rc; }
        for (uint64_t j = 0; j < group; ++j) counts[g0 + j] = count_hits(buf + j * n, n);
    }
    free(buf);
    return ORC_OK;
}

/* Float predicate of one pair, exposed for tests. */
int orc_qc_hit(uint32_t r1, uint32_t r2)
{
    uint32_t r[2] = {r1, r2};
    return (int)count_hits(r, 2);
}
