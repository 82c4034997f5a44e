// groupjump.cpp -- batched uneven runs of the exchange variants (V2, V4)
// and of V1: jump-ahead polynomials and the chunked launches.
//
// A group of C streams of Algorithm 4 advances in lockstep, and every
// operation of one step -- the xor-shift generator (xor128 on 32-bit words
// for V2, xor64 for V4), the mixing with two neighbours' previous words, the
// chaotic update x ^= t -- is a xor or a shift.  So the group's one-step map
// A is linear over GF(2) on the concatenated states (generator words, x, t
// of every stream), and A^J = r(A) with r = X^J mod q for any q with
// q(A) = 0.  A chunk of a group that starts J steps in therefore starts from
// sum_k r_k A^k s0: deg(q) steps of the group with a masked accumulate.
//
// q is the minimal polynomial of A, found per handle (it depends on C and the
// combination arrays): Berlekamp-Massey on random parities of the simulated
// group state gives the minimal polynomials of those sequences; their least
// common multiple is q with high probability, and q(A) v = 0 is then checked
// on random states before use.
#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <random>

#include "host.h"
#include "tune.h"

#define HIP_TRY(call, what)                                    \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return hip_error(_e, what);      \
    } while (0)

namespace cprng_impl {

namespace {

using Poly = std::vector<uint64_t>;   // bit i = coefficient of X^i

int pdeg(const Poly &p)
{
    for (int i = (int)p.size() - 1; i >= 0; --i)
        if (p[i]) return i * 64 + 63 - __builtin_clzll(p[i]);
    return -1;
}
bool pbit(const Poly &p, int i) { return (size_t)(i >> 6) < p.size() && ((p[i >> 6] >> (i & 63)) & 1u); }
void pflip(Poly &p, int i)
{
    if ((size_t)(i >> 6) >= p.size()) p.resize((i >> 6) + 1, 0);
    p[i >> 6] ^= 1ull << (i & 63);
}
void ptrim(Poly &p)
{
    while (!p.empty() && !p.back()) p.pop_back();
}
// a ^= b << s
void pxor_shift(Poly &a, const Poly &b, int s)
{
    const int db = pdeg(b);
    if (db < 0) return;
    const size_t need = (size_t)((db + s) >> 6) + 1;
    if (a.size() < need) a.resize(need, 0);
    const int ws = s >> 6, bs = s & 63;
    for (size_t i = 0; i < b.size(); ++i) {
        if (!b[i]) continue;
        a[i + ws] ^= b[i] << bs;
        if (bs && i + ws + 1 < a.size()) a[i + ws + 1] ^= b[i] >> (64 - bs);
    }
}
// a mod m (m != 0), in place.
void pmod(Poly &a, const Poly &m)
{
    const int dm = pdeg(m);
    for (int d = pdeg(a); d >= dm; d = pdeg(a)) pxor_shift(a, m, d - dm);
    ptrim(a);
}
Poly pmul(const Poly &a, const Poly &b)
{
    Poly r;
    const int da = pdeg(a);
    for (int i = 0; i <= da; ++i)
        if (pbit(a, i)) pxor_shift(r, b, i);
    ptrim(r);
    return r;
}
Poly pmulmod(const Poly &a, const Poly &b, const Poly &m)
{
    Poly r = pmul(a, b);
    pmod(r, m);
    return r;
}
// quotient and remainder of a / b
void pdivmod(Poly a, const Poly &b, Poly &q, Poly &r)
{
    q.clear();
    const int db = pdeg(b);
    for (int d = pdeg(a); d >= db; d = pdeg(a)) {
        pflip(q, d - db);
        pxor_shift(a, b, d - db);
    }
    ptrim(a);
    ptrim(q);
    r = a;
}
Poly pgcd(Poly a, Poly b)
{
    ptrim(a);
    ptrim(b);
    while (pdeg(b) >= 0) {
        Poly q, r;
        pdivmod(a, b, q, r);
        a = b;
        b = r;
    }
    return a;
}
Poly plcm(const Poly &a, const Poly &b)
{
    Poly q, r;
    pdivmod(pmul(a, b), pgcd(a, b), q, r);
    return q;
}
// sum_{i=1..n} X^i mod m, by doubling: S(2k) = S(k) + X^k S(k),
// S(k+1) = S(k) + X^(k+1).
Poly pgeomsum(uint64_t n, const Poly &m)
{
    Poly S, P{1}, X;
    pflip(X, 1);
    pmod(P, m);
    pmod(X, m);
    bool started = false;                           // past the leading zero bits of n
    for (int b = 63; b >= 0; --b) {
        if (started) {
            Poly PS = pmulmod(P, S, m);
            for (size_t i = 0; i < PS.size(); ++i) {
                if (i >= S.size()) S.resize(i + 1, 0);
                S[i] ^= PS[i];
            }
            ptrim(S);
            P = pmulmod(P, P, m);
        }
        if ((n >> b) & 1u) {
            started = true;
            P = pmulmod(P, X, m);
            for (size_t i = 0; i < P.size(); ++i) {
                if (i >= S.size()) S.resize(i + 1, 0);
                S[i] ^= P[i];
            }
            ptrim(S);
        }
    }
    return S;
}

// X^e mod m
Poly pxpow(uint64_t e, const Poly &m)
{
    Poly r{1}, base;
    pflip(base, 1);
    pmod(r, m);
    pmod(base, m);
    while (e) {
        if (e & 1) r = pmulmod(r, base, m);
        base = pmulmod(base, base, m);
        e >>= 1;
    }
    return r;
}

// Berlekamp-Massey over GF(2): minimal polynomial (reciprocal of the
// connection polynomial, as a polynomial in X) of the sequence s, and its
// linear complexity.
Poly berlekamp_massey(const std::vector<uint8_t> &s, int *L_out)
{
    const size_t n = s.size();
    std::vector<uint8_t> C(n + 1, 0), B(n + 1, 0), T;
    C[0] = B[0] = 1;
    int L = 0, m = 1;
    for (size_t i = 0; i < n; ++i) {
        uint8_t d = s[i];
        for (int j = 1; j <= L; ++j) d ^= C[j] & s[i - j];
        if (!d) {
            ++m;
        } else if (2 * L <= (int)i) {
            T = C;
            for (size_t j = 0; j + m <= n; ++j) C[j + m] ^= B[j];
            L = (int)i + 1 - L;
            B = T;
            m = 1;
        } else {
            for (size_t j = 0; j + m <= n; ++j) C[j + m] ^= B[j];
            ++m;
        }
    }
    // connection C(X) = 1 + c1 X + ... + cL X^L; minimal polynomial X^L C(1/X)
    Poly p;
    for (int j = 0; j <= L; ++j)
        if (C[j]) pflip(p, L - j);
    *L_out = L;
    return p;
}

// The group of C streams, simulated on the host: words per stream in the
// library's state order (V2: xor128 x,y,z,w, x, t; V4: y lo, y hi, x, t).
struct GroupSim {
    uint32_t variant, C;
    const uint8_t *c1, *c2;
    std::vector<uint32_t> w;   // C * words
    uint32_t words() const { return variant == CPRNG_V2_SHMEM ? 6u : 4u; }
    void step()
    {
        const uint32_t nw = words();
        std::vector<uint32_t> u(C), tprev(C);
        for (uint32_t j = 0; j < C; ++j) {
            uint32_t *s = &w[j * nw];
            if (variant == CPRNG_V2_SHMEM) {
                const uint32_t t = s[0] ^ (s[0] << 11);
                s[0] = s[1];
                s[1] = s[2];
                s[2] = s[3];
                s[3] = (s[3] ^ (s[3] >> 19)) ^ (t ^ (t >> 8));
                u[j] = s[3];
            } else {
                uint64_t y = (uint64_t)s[0] | ((uint64_t)s[1] << 32);
                y ^= y << 13;
                y ^= y >> 7;
                y ^= y << 17;
                s[0] = (uint32_t)y;
                s[1] = (uint32_t)(y >> 32);
                u[j] = s[0] ^ s[1];
            }
            tprev[j] = s[nw - 1];
        }
        for (uint32_t j = 0; j < C; ++j) {
            uint32_t *s = &w[j * nw];
            const uint32_t t = u[j] ^ tprev[c1[j]] ^ tprev[c2[j]];
            s[nw - 1] = t;
            s[nw - 2] ^= t;
        }
    }
};

// q(A) v == 0 for 24 random states v (if q(A) != 0, its kernel is a proper
// subspace, which holds a random v with probability at most 1/2 per trial).
bool check_annihilates(GroupSim g, const Poly &q, std::mt19937_64 &rng)
{
    const int d = pdeg(q);
    for (int trial = 0; trial < 24; ++trial) {
        for (auto &x : g.w) x = (uint32_t)rng();
        std::vector<uint32_t> acc(g.w.size(), 0);
        for (int k = 0; k <= d; ++k) {
            if (pbit(q, k))
                for (size_t i = 0; i < acc.size(); ++i) acc[i] ^= g.w[i];
            g.step();
        }
        for (uint32_t x : acc)
            if (x) return false;
    }
    return true;
}

// Minimal polynomial of a linear map on `nwords` words of W bits (mask) given
// its one-step function, found and checked (24 random states) as for the
// group map.
bool linear_minpoly(size_t nwords, uint64_t mask, const std::function<void(std::vector<uint64_t> &)> &step,
                    std::mt19937_64 &rng, Poly &q)
{
    const int n_obs = 12;
    for (int len = 1024; len <= 8192; len *= 2) {
        std::vector<uint64_t> s(nwords);
        for (auto &x : s) x = rng() & mask;
        std::vector<std::vector<uint64_t>> masks(n_obs, std::vector<uint64_t>(nwords));
        for (auto &m : masks)
            for (auto &x : m) x = rng() & mask;
        std::vector<std::vector<uint8_t>> seq(n_obs, std::vector<uint8_t>(len));
        for (int i = 0; i < len; ++i) {
            for (int o = 0; o < n_obs; ++o) {
                uint64_t acc = 0;
                for (size_t k = 0; k < nwords; ++k) acc ^= s[k] & masks[o][k];
                seq[o][i] = (uint8_t)(__builtin_popcountll(acc) & 1);
            }
            step(s);
        }
        Poly p{1};
        bool long_enough = true;
        for (int o = 0; o < n_obs; ++o) {
            int L = 0;
            Poly b = berlekamp_massey(seq[o], &L);
            if (2 * L + 64 > len) long_enough = false;
            p = plcm(p, b);
        }
        if (!long_enough) continue;
        bool annihilates = true;
        const int d = pdeg(p);
        for (int trial = 0; trial < 24 && annihilates; ++trial) {
            std::vector<uint64_t> v(nwords), acc(nwords, 0);
            for (auto &x : v) x = rng() & mask;
            for (int k = 0; k <= d; ++k) {
                if (pbit(p, k))
                    for (size_t i = 0; i < nwords; ++i) acc[i] ^= v[i];
                step(v);
            }
            for (uint64_t x : acc)
                if (x) annihilates = false;
        }
        if (!annihilates) continue;
        q = p;
        return true;
    }
    return false;
}

// The minimal polynomials of V1's three generators for one word width and
// first-generator triple, computed once per process.
struct V1Polys {
    Poly q[3];
    int deg[3] = {0, 0, 0};
    bool ok = false;
};

const V1Polys &v1_polys(int W, uint32_t sb, uint32_t sc)
{
    static std::mutex mu;
    static std::map<uint64_t, V1Polys> cache;
    std::lock_guard<std::mutex> lock(mu);
    const uint64_t key = ((uint64_t)W << 16) | (sb << 8) | sc;
    auto f = cache.find(key);
    if (f != cache.end()) return f->second;
    V1Polys &r = cache[key];
    const uint64_t m = W == 64 ? ~0ull : 0xFFFFFFFFull;
    std::mt19937_64 rng(0x1e5eed11ull);
    auto g1 = [&](std::vector<uint64_t> &s) {
        uint64_t a = s[0];
        a ^= (a << 13) & m;
        a ^= a >> sb;
        a ^= (a << sc) & m;
        s[0] = a;
    };
    auto g2 = [&](std::vector<uint64_t> &s) {
        const uint64_t t = s[0] ^ ((s[0] << 11) & m);
        s[0] = s[1];
        s[1] = s[2];
        s[2] = s[3];
        s[3] = (s[3] ^ (s[3] >> 19)) ^ (t ^ (t >> 8));
    };
    auto g3 = [&](std::vector<uint64_t> &s) {
        const uint64_t u = s[0] ^ (s[0] >> 2);
        s[0] = s[1];
        s[1] = s[2];
        s[2] = s[3];
        s[3] = s[4];
        s[4] = (s[4] ^ ((s[4] << 4) & m)) ^ (u ^ ((u << 1) & m));
    };
    r.ok = linear_minpoly(1, m, g1, rng, r.q[0]) && linear_minpoly(4, m, g2, rng, r.q[1]) &&
           linear_minpoly(5, m, g3, rng, r.q[2]);
    for (int k = 0; k < 3; ++k) r.deg[k] = pdeg(r.q[k]);
    return r;
}

}  // namespace

int group_minpoly(cprng_t *h)
{
    if (h->gj_deg > 0) return CPRNG_OK;
    GroupSim g{h->variant, h->group, h->comb1, h->comb2, {}};
    const uint32_t nw = g.words();
    g.w.assign((size_t)h->group * nw, 0);
    std::mt19937_64 rng(0x5eed5eedull);
    // Observations: parities of random masks of the state, one per step.
    const int n_obs = 24;
    for (int len = 2048; len <= 32768; len *= 2) {
        for (auto &x : g.w) x = (uint32_t)rng();
        std::vector<std::vector<uint32_t>> masks(n_obs, std::vector<uint32_t>(g.w.size()));
        for (auto &m : masks)
            for (auto &x : m) x = (uint32_t)rng();
        std::vector<std::vector<uint8_t>> seq(n_obs, std::vector<uint8_t>(len));
        GroupSim s = g;
        for (int i = 0; i < len; ++i) {
            for (int o = 0; o < n_obs; ++o) {
                uint32_t acc = 0;
                for (size_t k = 0; k < s.w.size(); ++k) acc ^= s.w[k] & masks[o][k];
                seq[o][i] = (uint8_t)(__builtin_popcount(acc) & 1);
            }
            s.step();
        }
        Poly q{1};
        bool long_enough = true;
        for (int o = 0; o < n_obs; ++o) {
            int L = 0;
            Poly p = berlekamp_massey(seq[o], &L);
            if (2 * L + 64 > len) long_enough = false;
            q = plcm(q, p);
        }
        if (!long_enough) continue;
        if (!check_annihilates(g, q, rng)) continue;
        h->gj_q = q;
        h->gj_deg = pdeg(q);
        return CPRNG_OK;
    }
    return set_error(CPRNG_E_HIP, "group jump-ahead: no annihilating polynomial found");
}

void group_jump_rows(const cprng_t *h, uint64_t chunk, uint32_t rows, std::vector<uint32_t> &out)
{
    const uint32_t W = (uint32_t)((h->gj_deg + 31) / 32);
    out.assign((size_t)rows * W, 0);
    const Poly base = pxpow(chunk, h->gj_q);
    Poly r{1};
    pmod(r, h->gj_q);
    for (uint32_t c = 0; c < rows; ++c) {
        for (int k = 0; k < h->gj_deg; ++k)
            if (pbit(r, k)) out[(size_t)c * W + (k >> 5)] |= 1u << (k & 31);
        r = pmulmod(r, base, h->gj_q);
    }
}

namespace {

// Store round of the chunk kernels: 32, 64 or 128 words.
uint32_t norm_round(uint32_t u) { return (u == 32 || u == 64 || u == 128) ? u : 64u; }

// Waves of a chunk kernel that stay resident per CU, from its tiles' LDS
// (the kernels' other limits are looser): per wave, V1 64 rows of K + 1
// words, the group kernel 64 rings of 2K + 1 words, each with a 512-byte
// table of line addresses.
uint64_t chunk_resident_waves(const ChunkCfg &c, bool v1)
{
    const uint64_t K = c.round, W = c.wg_waves;
    const uint64_t wave_lds = (v1 ? 64u * (K + 1u) * 4u : 64u * (2u * K + 1u) * 4u) + 512u;
    return std::min<uint64_t>(32u, (kMaxLdsBytes / (W * wave_lds)) * W);
}

// Shortest chunk, a multiple of 64 in [lo, 2^20], with n_items(chunk) <= cap
// (n_items does not grow with the chunk); 2^20 if none.
template <typename F>
uint64_t fit_chunk(uint64_t lo, uint64_t cap, F &&n_items)
{
    lo = std::max<uint64_t>(64u, (lo + 63u) / 64u * 64u);
    uint64_t hi = 1ull << 20;
    if (lo >= hi || n_items(hi) > cap) return hi;
    if (n_items(lo) <= cap) return lo;
    while (hi - lo > 64u) {                 // n_items(lo) > cap >= n_items(hi)
        const uint64_t mid = lo + ((hi - lo) / 128u) * 64u;
        if (n_items(mid) <= cap) hi = mid; else lo = mid;
    }
    return hi;
}

// Device buffer that grows on demand.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

int ensure(DevBuf &b, size_t bytes)
{
    if (b.p && b.cap >= bytes) return CPRNG_OK;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    if (hipMalloc(&b.p, std::max<size_t>(bytes, 16)) != hipSuccess)
        return set_error(CPRNG_E_NOMEM, "hipMalloc of batched-run buffers failed");
    b.cap = bytes;
    return CPRNG_OK;
}

void release(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

template <typename T>
int put(DevBuf &b, const std::vector<T> &v)
{
    int rc = ensure(b, v.size() * sizeof(T));
    if (rc || v.empty()) return rc;
    if (hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return set_error(CPRNG_E_HIP, "hipMemcpy of batched-run tables");
    return CPRNG_OK;
}

}  // namespace

// Device tables of one batched call of V1 or V2/V4.
struct ChunkBufs {
    DevBuf items, rows, sub_rows, offs, order, agg, sfirst;
    void release_all()
    {
        for (DevBuf *b : {&items, &rows, &sub_rows, &offs, &order, &agg, &sfirst}) release(*b);
    }
};

// A cached batched call: its inputs, tables and captured graph.
struct ChunkPlan {
    std::vector<uint64_t> lengths, offsets;
    uint32_t *out = nullptr;
    ChunkCfg cfg;
    ChunkBufs bufs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

namespace {

uint64_t g_chunk_clock = 0;

void free_chunk_plan(ChunkPlan *p)
{
    if (!p) return;
    // A replay of this plan may still be queued or running: let the device
    // finish before the graph and its tables go.
    if (p->exec) (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->bufs.release_all();
    delete p;
}

// Host side of one batched call: the chunk list, jump rows and offsets.
struct ChunkHost {
    ChunkCfg cfg;                      // resolved: chunk > 0
    std::vector<GroupItem> gitems;     // V2/V4
    std::vector<V1Item> vitems;        // V1
    std::vector<uint32_t> order;       // V1: chunks with a successor
    std::vector<uint32_t> sfirst;      // V1: first chunk per stream (+ end)
    std::vector<uint32_t> rows, sub_rows;
    std::vector<uint64_t> offs;
    uint32_t row_words = 0, off[3] = {0, 0, 0}, deg[3] = {0, 0, 0}, w3 = 0, n_rows = 0;
};

bool is_v1(const cprng_t *h) { return h->variant == CPRNG_V1_NAIVE3; }

const V1Polys &v1_polys_of(const cprng_t *h)
{
    const bool w32 = (h->flags & CPRNG_F_V1_W32) != 0;
    const bool xor64 = (h->flags & CPRNG_F_V1_XOR64) != 0;
    return v1_polys(w32 ? 32 : 64, xor64 ? 7u : 17u, xor64 ? 17u : 5u);
}

// Automatic chunk: the shortest multiple of 64 (at least 16 x the jump's
// length, at most 2^20) whose chunks fill at most 31/32 of `passes` passes
// of the chunk kernel's resident waves.  Its time follows whole passes (a
// last pass that is mostly empty costs a whole chunk's time); the exchange
// variants want their chunks in one pass (the exchange reads' latency needs
// many waves; fewer, longer runs in flight store better), V1 in six (its
// aggregate pass wants the waves, and shorter chunks even out the lanes'
// work by more than their extra jumps cost: 4,096 runs log-uniform in
// 1e3..1e7 took 8.1 ms at six passes against 8.6 at two).  The 3% slack
// keeps a workgroup the dispatcher places late from opening another pass.
uint64_t auto_chunk(const cprng_t *h, const uint64_t *lengths, const ChunkCfg &c, uint64_t jump_len)
{
    if (is_v1(h)) {
        const uint64_t cap = 6u * (uint64_t)h->n_cu * chunk_resident_waves(c, true) * 64u * 31u / 32u;
        return fit_chunk(16ull * jump_len, cap, [&](uint64_t ch) {
            uint64_t n = 0;
            for (uint32_t s = 0; s < h->ns; ++s) n += (lengths[s] + ch - 1) / ch;
            return n;
        });
    }
    const uint32_t C = h->group;
    const uint64_t cap = (uint64_t)h->n_cu * chunk_resident_waves(c, false) * (64u / C) * 31u / 32u;
    return fit_chunk(16ull * jump_len, cap, [&](uint64_t ch) {
        uint64_t n = 0;
        for (uint32_t g = 0; g < h->ns / C; ++g) n += (lengths[(size_t)g * C] + ch - 1) / ch;
        return n;
    });
}

uint64_t jump_length(const cprng_t *h)
{
    if (is_v1(h)) {
        const V1Polys &P = v1_polys_of(h);
        return (uint64_t)(P.deg[0] + P.deg[1] + P.deg[2]);
    }
    return (uint64_t)h->gj_deg;
}

// Minimal polynomials of the handle's variant (V1: per process; V2/V4: per
// handle).
int prepare_polys(cprng_t *h)
{
    if (is_v1(h)) return v1_polys_of(h).ok ? CPRNG_OK : set_error(CPRNG_E_HIP, "V1 jump-ahead: no annihilating polynomial found");
    return group_minpoly(h);
}

void fill_offsets(const cprng_t *h, const uint64_t *lengths, const uint64_t *offsets, std::vector<uint64_t> &offs)
{
    offs.resize(h->ns);
    uint64_t acc = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        offs[s] = offsets ? offsets[s] : acc;
        acc += lengths[s];
    }
}

int plan_groups(const cprng_t *h, const uint64_t *lengths, const uint64_t *offsets, ChunkHost &p)
{
    const uint32_t C = h->group;
    const uint32_t n_groups = h->ns / C;
    uint64_t max_len = 0;
    for (uint32_t g = 0; g < n_groups; ++g) max_len = std::max(max_len, lengths[(size_t)g * C]);
    const uint64_t chunk = p.cfg.chunk;
    uint64_t n_items = 0;
    for (uint32_t g = 0; g < n_groups; ++g) n_items += (lengths[(size_t)g * C] + chunk - 1) / chunk;
    if (n_items > (1ull << 26)) return set_error(CPRNG_E_INVAL, "more than 2^26 chunks (raise the chunk length)");
    p.gitems.reserve(n_items);
    for (uint32_t g = 0; g < n_groups; ++g) {
        const uint64_t L = lengths[(size_t)g * C];
        for (uint64_t a = 0, c = 0; a < L; a += chunk, ++c) {
            GroupItem it{};
            it.group = g;
            it.row = (uint32_t)c;
            it.start = a;
            it.len = std::min(chunk, L - a);
            it.last = (a + chunk >= L) ? 1u : 0u;
            p.gitems.push_back(it);
        }
    }
    p.n_rows = (uint32_t)((max_len + chunk - 1) / chunk);
    group_jump_rows(h, chunk, p.n_rows, p.rows);
    p.row_words = (uint32_t)((h->gj_deg + 31) / 32);
    fill_offsets(h, lengths, offsets, p.offs);
    return CPRNG_OK;
}

void put_poly(std::vector<uint32_t> &dst, size_t word0, const Poly &r, int deg)
{
    for (int b = 0; b < deg; ++b)
        if (pbit(r, b)) dst[word0 + (b >> 5)] |= 1u << (b & 31);
}

int plan_v1(const cprng_t *h, const uint64_t *lengths, const uint64_t *offsets, ChunkHost &p)
{
    const V1Polys &P = v1_polys_of(h);
    uint64_t max_len = 0;
    for (uint32_t s = 0; s < h->ns; ++s) max_len = std::max(max_len, lengths[s]);
    const uint64_t chunk = p.cfg.chunk;
    const uint32_t parts = p.cfg.parts;
    uint64_t n_items = 0;
    for (uint32_t s = 0; s < h->ns; ++s) n_items += (lengths[s] + chunk - 1) / chunk;
    if (n_items > (1ull << 26)) return set_error(CPRNG_E_INVAL, "more than 2^26 chunks (raise the chunk length)");
    p.vitems.reserve(n_items);
    p.sfirst.resize((size_t)h->ns + 1);
    for (uint32_t s = 0; s < h->ns; ++s) {
        const uint32_t first = (uint32_t)p.vitems.size();
        p.sfirst[s] = first;
        for (uint64_t a = 0, c = 0; a < lengths[s]; a += chunk, ++c) {
            V1Item it{};
            it.stream = s;
            it.row = (uint32_t)c;
            it.start = a;
            it.len = std::min(chunk, lengths[s] - a);
            it.last = (a + chunk >= lengths[s]) ? 1u : 0u;
            it.first = first;
            if (!it.last) p.order.push_back((uint32_t)p.vitems.size());
            p.vitems.push_back(it);
        }
        if (p.vitems.size() > 0xFFFFFFF0ull) return set_error(CPRNG_E_INVAL, "too many chunks");
    }
    p.sfirst[h->ns] = (uint32_t)p.vitems.size();
    if (p.order.size() * (uint64_t)parts > 0xFFFFFFF0ull) return set_error(CPRNG_E_INVAL, "too many chunks");
    p.n_rows = (uint32_t)((max_len + chunk - 1) / chunk);
    uint32_t wk[3];
    p.row_words = 0;
    for (int k = 0; k < 3; ++k) {
        p.deg[k] = (uint32_t)P.deg[k];
        wk[k] = (uint32_t)((P.deg[k] + 31) / 32);
        p.off[k] = p.row_words;
        p.row_words += wk[k];
    }
    p.w3 = wk[2];
    // rows 0..n_rows-1: X^(c * chunk) per generator; row n_rows: the sums
    // sum_{i=1..chunk} X^i of the xorshift and xor128 maps (full chunks'
    // aggregates)
    p.rows.assign((size_t)(p.n_rows + 1) * p.row_words, 0);
    for (int k = 0; k < 2; ++k)
        put_poly(p.rows, (size_t)p.n_rows * p.row_words + p.off[k], pgeomsum(chunk, P.q[k]), P.deg[k]);
    for (int k = 0; k < 3; ++k) {
        const Poly base = pxpow(chunk, P.q[k]);
        Poly r{1};
        pmod(r, P.q[k]);
        for (uint32_t c = 0; c < p.n_rows; ++c) {
            put_poly(p.rows, (size_t)c * p.row_words + p.off[k], r, P.deg[k]);
            r = pmulmod(r, base, P.q[k]);
        }
    }
    // xorwow sub-starts of the aggregate pass: X^(c * chunk + j * chunk / parts)
    const Poly step = pxpow(chunk / parts, P.q[2]);
    p.sub_rows.assign((size_t)p.n_rows * parts * p.w3, 0);
    Poly r{1};
    pmod(r, P.q[2]);
    for (uint32_t c = 0; c < p.n_rows; ++c)
        for (uint32_t j = 0; j < parts; ++j) {
            put_poly(p.sub_rows, ((size_t)c * parts + j) * p.w3, r, P.deg[2]);
            r = pmulmod(r, step, P.q[2]);       // after `parts` steps: X^((c + 1) * chunk)
        }
    fill_offsets(h, lengths, offsets, p.offs);
    return CPRNG_OK;
}

int upload(const ChunkHost &p, ChunkBufs &b)
{
    int rc = put(b.rows, p.rows);
    if (!rc) rc = put(b.offs, p.offs);
    if (p.vitems.empty()) {
        if (!rc) rc = put(b.items, p.gitems);
        return rc;
    }
    if (!rc) rc = put(b.items, p.vitems);
    if (!rc) rc = put(b.order, p.order);
    if (!rc) rc = put(b.sfirst, p.sfirst);
    if (!rc) rc = put(b.sub_rows, p.sub_rows);
    if (!rc) rc = ensure(b.agg, p.vitems.size() * sizeof(uint32_t));
    return rc;
}

// Kernels of one call, in stream order: copy of the start states, the chunk
// kernels, commit of the end states.
hipError_t enqueue(const cprng_t *h, const ChunkHost &p, const ChunkBufs &b, uint32_t *out, hipStream_t st)
{
    const size_t nwords = (size_t)h->ns * h->words;
    hipError_t e = launch_copy(h->d_gj_next, h->d_state, nwords, st);
    if (e != hipSuccess) return e;
    if (!p.vitems.empty()) {
        V1ChunkArgs a;
        std::memset(&a, 0, sizeof a);
        fill_gen_args(h, a.g);
        a.state_next = h->d_gj_next;
        a.items = (const V1Item *)b.items.p;
        a.n_items = (uint32_t)p.vitems.size();
        a.row_words = p.row_words;
        a.deg1 = p.deg[0];
        a.deg2 = p.deg[1];
        a.deg3 = p.deg[2];
        a.off2 = p.off[1];
        a.off3 = p.off[2];
        a.rows = (const uint32_t *)b.rows.p;
        a.agg = (uint32_t *)b.agg.p;
        a.out = out;
        a.offsets = (const uint64_t *)b.offs.p;
        a.chunk = p.cfg.chunk;
        a.sum_row = p.n_rows;
        a.round = p.cfg.round;
        a.wg_waves = p.cfg.wg_waves;
        a.order = (const uint32_t *)b.order.p;
        a.n_agg = (uint32_t)p.order.size();
        a.parts = p.cfg.parts;
        a.sub_rows = (const uint32_t *)b.sub_rows.p;
        a.w3 = p.w3;
        a.sfirst = (const uint32_t *)b.sfirst.p;
        e = launch_v1_chunks(a, (h->flags & CPRNG_F_V1_W32) != 0, st);
    } else if (!p.gitems.empty()) {
        GroupJumpArgs a;
        std::memset(&a, 0, sizeof a);
        fill_gen_args(h, a.g);
        a.state_next = h->d_gj_next;
        a.items = (const GroupItem *)b.items.p;
        a.n_items = (uint32_t)p.gitems.size();
        a.rows = (const uint32_t *)b.rows.p;
        a.row_words = p.row_words;
        a.deg = (uint32_t)h->gj_deg;
        a.round = p.cfg.round;
        a.wg_waves = p.cfg.wg_waves;
        a.out = out;
        a.offsets = (const uint64_t *)b.offs.p;
        e = launch_group_chunks(a, (int)h->variant, st);
    }
    if (e != hipSuccess) return e;
    return launch_copy(h->d_state, h->d_gj_next, nwords, st);
}

int plan_host(cprng_t *h, const uint64_t *lengths, const uint64_t *offsets, const ChunkCfg &cfg, ChunkHost &p)
{
    p.cfg = cfg;
    p.cfg.round = norm_round(cfg.round);
    p.cfg.wg_waves = cfg.wg_waves == 1 ? 1u : 4u;
    if (!is_v1(h) && p.cfg.round == 128) p.cfg.wg_waves = 1;   // the group kernel's K = 128 rings: one wave per workgroup
    p.cfg.parts = (cfg.parts == 1 || cfg.parts == 2 || cfg.parts == 4) ? cfg.parts : 2u;
    if (!p.cfg.chunk) p.cfg.chunk = auto_chunk(h, lengths, p.cfg, jump_length(h));
    if (p.cfg.chunk % 64u || p.cfg.chunk > (1ull << 40))
        return set_error(CPRNG_E_INVAL, "chunk must be a multiple of 64");
    return is_v1(h) ? plan_v1(h, lengths, offsets, p) : plan_groups(h, lengths, offsets, p);
}

int ensure_next(cprng_t *h)
{
    const size_t need = (size_t)h->ns * h->words;
    if (h->d_gj_next && h->gj_next_cap >= need) return CPRNG_OK;
    if (h->d_gj_next) (void)hipFree(h->d_gj_next);       // waits for the device
    h->d_gj_next = nullptr;
    h->gj_next_cap = 0;
    if (hipMalloc((void **)&h->d_gj_next, need * sizeof(uint32_t)) != hipSuccess)
        return set_error(CPRNG_E_NOMEM, "hipMalloc of the end-state buffer failed");
    h->gj_next_cap = need;
    return CPRNG_OK;
}

bool same_cfg(const ChunkCfg &a, const ChunkCfg &b)
{
    return a.chunk == b.chunk && a.round == b.round && a.wg_waves == b.wg_waves && a.parts == b.parts;
}

ChunkPlan *find_chunk_plan(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets,
                           const ChunkCfg &cfg)
{
    for (ChunkPlan *p : h->chunk_plans) {
        if (p->out != out || !same_cfg(p->cfg, cfg)) continue;
        if (std::memcmp(p->lengths.data(), lengths, sizeof(uint64_t) * h->ns) != 0) continue;
        bool same = true;
        uint64_t acc = 0;
        for (uint32_t s = 0; s < h->ns && same; ++s) {
            same = p->offsets[s] == (offsets ? offsets[s] : acc);
            acc += lengths[s];
        }
        if (same) return p;
    }
    return nullptr;
}

int build_chunk_plan(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets,
                     const ChunkCfg &cfg, ChunkPlan **res)
{
    ChunkHost hp;
    int rc = plan_host(h, lengths, offsets, cfg, hp);
    if (rc) return rc;
    std::unique_ptr<ChunkPlan, void (*)(ChunkPlan *)> p(new ChunkPlan(), free_chunk_plan);
    p->lengths.assign(lengths, lengths + h->ns);
    fill_offsets(h, lengths, offsets, p->offsets);
    p->out = out;
    p->cfg = cfg;
    if ((rc = upload(hp, p->bufs))) return rc;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return set_error(CPRNG_E_HIP, "hipStreamCreate (capture)");
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = enqueue(h, hp, p->bufs, out, cs);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_error(e, "capture of the batched kernels");
    }
    if (e2 != hipSuccess) return hip_error(e2, "hipStreamEndCapture");
    p->graph = graph;
    e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_error(e, "hipGraphInstantiate");
    *res = p.release();
    return CPRNG_OK;
}

void drop_chunk_plan(cprng_t *h, ChunkPlan *p)
{
    auto it = std::find(h->chunk_plans.begin(), h->chunk_plans.end(), p);
    if (it != h->chunk_plans.end()) h->chunk_plans.erase(it);
    free_chunk_plan(p);
}

int check_group_lengths(const cprng_t *h, const uint64_t *lengths)
{
    if (is_v1(h)) return CPRNG_OK;
    const uint32_t C = h->group;
    for (uint32_t g0 = 0; g0 < h->ns; g0 += C)
        for (uint32_t j = 1; j < C; ++j)
            if (lengths[g0 + j] != lengths[g0])
                return set_error(CPRNG_E_INVAL, "V2/V4: lengths must be equal within each group of C streams");
    return CPRNG_OK;
}

}  // namespace

// Defaults measured on MI355X (4,096 V1 streams / 128 V2 groups of 32,
// lengths log-uniform in [1e3, 1e7]), four-wave workgroups and the
// automatic chunk: V1 rounds of 64 words, aggregates split over two lanes;
// the group kernel rounds of 32 words (128-byte lines; its two-line rings
// then leave 8 waves per CU).
ChunkCfg default_chunk_cfg(const cprng_t *h)
{
    ChunkCfg c;
    c.chunk = 0;
    c.round = is_v1(h) ? 64u : 32u;
    c.wg_waves = 4;
    c.parts = 2;
    return c;
}

ChunkCfg resolve_chunk_cfg(const cprng_t *h, uint64_t total, uint64_t max_len)
{
    ChunkCfg c = default_chunk_cfg(h);
    TuneEntry e;
    if (tune_cache_lookup_key(tune_key_ragged(h, total, max_len), &e)) {
        c.chunk = e.chunk;
        if (e.unroll) c.round = e.unroll;
        if (e.block) c.wg_waves = e.block == 64 ? 1u : 4u;
        if (e.slots) c.parts = e.slots;
    }
    if (h->tuning.chunk) c.chunk = h->tuning.chunk;
    if (h->tuning.unroll) c.round = h->tuning.unroll;
    if (h->tuning.block == 64 || h->tuning.block == 256) c.wg_waves = h->tuning.block == 64 ? 1u : 4u;
    if (h->tuning.streams_per_lane) c.parts = h->tuning.streams_per_lane;
    c.round = norm_round(c.round);
    if (c.parts != 1 && c.parts != 2 && c.parts != 4) c.parts = 2;
    return c;
}

int ragged_chunked(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st,
                   const ChunkCfg &cfg, bool cached)
{
    int rc = check_group_lengths(h, lengths);
    if (rc) return rc;
    uint64_t total = 0;
    for (uint32_t s = 0; s < h->ns; ++s) total += lengths[s];
    if (total == 0) return CPRNG_OK;
    if ((rc = prepare_polys(h))) return rc;
    if ((rc = ensure_next(h))) return rc;
    if (!cached) {
        // One-off call (request rounds): plan, wait until the previous call
        // has released the shared tables, upload, launch.
        ChunkHost hp;
        if ((rc = plan_host(h, lengths, offsets, cfg, hp))) return rc;
        if (!h->chunk_direct) h->chunk_direct = new ChunkBufs();
        HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        if ((rc = upload(hp, *h->chunk_direct))) return rc;
        if ((rc = timing_begin(h, st))) return rc;
        HIP_TRY(enqueue(h, hp, *h->chunk_direct, out, st), "batched kernels");
        return timing_end(h, st);
    }
    ChunkPlan *p = find_chunk_plan(h, out, lengths, offsets, cfg);
    if (!p) {
        if ((rc = build_chunk_plan(h, out, lengths, offsets, cfg, &p))) return rc;
        if (h->chunk_plans.size() >= 8) {
            auto it = std::min_element(h->chunk_plans.begin(), h->chunk_plans.end(),
                                       [](ChunkPlan *a, ChunkPlan *b) { return a->last_use < b->last_use; });
            free_chunk_plan(*it);
            h->chunk_plans.erase(it);
        }
        h->chunk_plans.push_back(p);
    }
    p->last_use = ++g_chunk_clock;
    if (h->timing && hipEventRecord(h->ev0, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
    HIP_TRY(hipGraphLaunch(p->exec, st), "hipGraphLaunch");
    if (h->timing) {
        if (hipEventRecord(h->ev1, st) != hipSuccess) return set_error(CPRNG_E_HIP, "hipEventRecord");
        h->ev_pending = true;
    }
    return CPRNG_OK;
}

int chunk_for(cprng_t *h, const uint64_t *lengths, const ChunkCfg &cfg, uint64_t *chunk)
{
    if (cfg.chunk) {
        *chunk = cfg.chunk;
        return CPRNG_OK;
    }
    const int rc = prepare_polys(h);
    if (rc) return rc;
    ChunkCfg c = cfg;
    c.round = norm_round(c.round);
    c.wg_waves = c.wg_waves == 1 ? 1u : 4u;
    if (!is_v1(h) && c.round == 128) c.wg_waves = 1;
    *chunk = auto_chunk(h, lengths, c, jump_length(h));
    return CPRNG_OK;
}

int ragged_groups(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st)
{
    uint64_t total = 0, max_len = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        total += lengths[s];
        max_len = std::max(max_len, lengths[s]);
    }
    return ragged_chunked(h, out, lengths, offsets, st, resolve_chunk_cfg(h, total, max_len), true);
}

int ragged_v1(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st,
              bool cached)
{
    uint64_t total = 0, max_len = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        total += lengths[s];
        max_len = std::max(max_len, lengths[s]);
    }
    return ragged_chunked(h, out, lengths, offsets, st, resolve_chunk_cfg(h, total, max_len), cached);
}

// Autotuner of the chunk kernels (V1, V2, V4): store round, workgroup
// shape, chunk length around the automatic one and (V1) the aggregate
// pass's lanes per chunk.  Each candidate runs as its own cached graph;
// only the winner's graph is kept.
int autotune_chunked(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st,
                     uint64_t total, uint64_t max_len)
{
    (void)max_len;
    int rc = check_group_lengths(h, lengths);
    if (rc) return rc;
    if (total == 0) return CPRNG_OK;
    if ((rc = prepare_polys(h))) return rc;
    if ((rc = ensure_next(h))) return rc;
    std::vector<ChunkCfg> cands;
    cands.push_back(default_chunk_cfg(h));                    // candidate 0: the defaults
    const uint32_t parts_v1[] = {1, 2, 4};
    const uint32_t parts_grp[] = {2};
    const uint32_t *parts = is_v1(h) ? parts_v1 : parts_grp;
    const int n_parts = is_v1(h) ? 3 : 1;
    for (uint32_t K : {32u, 64u, 128u})
        for (uint32_t W : {1u, 4u})
            for (int pi = 0; pi < n_parts; ++pi)
                for (int scale = 0; scale < 3; ++scale) {
                    if (!is_v1(h) && K == 128 && W == 4) continue; // group rings of K = 128: one wave per workgroup
                    ChunkCfg c;
                    c.round = K;
                    c.wg_waves = W;
                    c.parts = parts[pi];
                    c.chunk = 0;
                    if (scale) {
                        const uint64_t a = auto_chunk(h, lengths, c, jump_length(h));
                        c.chunk = scale == 1 ? std::max<uint64_t>(64u, a / 2u / 64u * 64u) : std::min<uint64_t>(a * 2u, 1ull << 20);
                    }
                    cands.push_back(c);
                }
    const bool saved_timing = h->timing;
    h->timing = false;
    auto drop = [&](const ChunkCfg &c) {
        if (ChunkPlan *p = find_chunk_plan(h, out, lengths, offsets, c)) drop_chunk_plan(h, p);
    };
    size_t best = 0;
    rc = tune_select(
        cands.size(), 0, st, [&](size_t i) { return ragged_chunked(h, out, lengths, offsets, st, cands[i], true); },
        [&](size_t i, bool kept) {
            if (!kept) drop(cands[i]);
        },
        &best);
    for (size_t i = 0; i < cands.size(); ++i)
        if (i != best) drop(cands[i]);
    h->timing = saved_timing;
    if (rc) return rc;
    const ChunkCfg &b = cands[best];
    TuneEntry e;
    e.chunk = (uint32_t)b.chunk;
    e.unroll = b.round;
    e.block = b.wg_waves == 1 ? 64u : 256u;
    e.slots = b.parts;
    tune_cache_store(tune_key_ragged(h, total, max_len), e);
    return CPRNG_OK;
}

void destroy_group_buffers(cprng_t *h)
{
    for (ChunkPlan *p : h->chunk_plans) free_chunk_plan(p);
    h->chunk_plans.clear();
    if (h->chunk_direct) {
        h->chunk_direct->release_all();
        delete h->chunk_direct;
        h->chunk_direct = nullptr;
    }
    if (h->d_gj_next) (void)hipFree(h->d_gj_next);
    h->d_gj_next = nullptr;
    h->gj_next_cap = 0;
}

}  // namespace cprng_impl

using namespace cprng_impl;

// Host-only self-test of the jump-ahead machinery (no device work).
extern "C" int cprng_jump_selftest(uint32_t variant, uint32_t C, const uint32_t *comb1, const uint32_t *comb2,
                                   uint64_t J)
{
    const uint32_t var = variant & 0xffu, flags = variant & ~0xffu;
    std::mt19937_64 rng(0xabcdef12ull + J);
    if (var == CPRNG_V2_SHMEM || var == CPRNG_V4_XOR64) {
        if (flags) return set_error(CPRNG_E_INVAL, "no flags for the group self-test");
        if (C < 3 || C > 64 || (64 % C)) return set_error(CPRNG_E_INVAL, "C must divide 64");
        uint32_t c1[64], c2[64];
        if (comb1 && comb2) {
            for (uint32_t j = 0; j < C; ++j) {
                if (comb1[j] >= C || comb2[j] >= C) return set_error(CPRNG_E_INVAL, "combination entry out of range");
                c1[j] = comb1[j];
                c2[j] = comb2[j];
            }
        } else if (!default_combs(C, c1, c2)) {
            return set_error(CPRNG_E_INVAL, "no default combination arrays");
        }
        cprng h;
        h.variant = var;
        h.group = C;
        for (uint32_t j = 0; j < 64; ++j) {
            h.comb1[j] = (uint8_t)c1[j % C];
            h.comb2[j] = (uint8_t)c2[j % C];
        }
        int rc = group_minpoly(&h);
        if (rc) return rc;
        GroupSim g{var, C, h.comb1, h.comb2, {}};
        g.w.assign((size_t)C * g.words(), 0);
        for (auto &x : g.w) x = (uint32_t)rng();
        const Poly r = pxpow(J, h.gj_q);
        GroupSim walk = g, direct = g;
        std::vector<uint32_t> acc(g.w.size(), 0);
        for (int k = 0; k < h.gj_deg; ++k) {
            if (pbit(r, k))
                for (size_t i = 0; i < acc.size(); ++i) acc[i] ^= walk.w[i];
            walk.step();
        }
        for (uint64_t k = 0; k < J; ++k) direct.step();
        return acc == direct.w ? CPRNG_OK : set_error(CPRNG_E_HIP, "group jump differs from stepping");
    }
    if (var == CPRNG_V1_NAIVE3) {
        if (flags & ~(uint32_t)(CPRNG_F_V1_W32 | CPRNG_F_V1_XOR64)) return set_error(CPRNG_E_INVAL, "unknown flag bits");
        const bool w32 = (flags & CPRNG_F_V1_W32) != 0, x64 = (flags & CPRNG_F_V1_XOR64) != 0;
        if (w32 && x64) return set_error(CPRNG_E_INVAL, "xor64 needs 64-bit words");
        const uint32_t sb = x64 ? 7u : 17u, sc = x64 ? 17u : 5u;
        const V1Polys &P = v1_polys(w32 ? 32 : 64, sb, sc);
        if (!P.ok) return set_error(CPRNG_E_HIP, "V1 jump-ahead: no annihilating polynomial found");
        const uint64_t m = w32 ? 0xFFFFFFFFull : ~0ull;
        auto step = [&](int k, std::vector<uint64_t> &s) {
            if (k == 0) {
                uint64_t a = s[0];
                a ^= (a << 13) & m;
                a ^= a >> sb;
                a ^= (a << sc) & m;
                s[0] = a;
            } else if (k == 1) {
                const uint64_t t = s[0] ^ ((s[0] << 11) & m);
                s[0] = s[1]; s[1] = s[2]; s[2] = s[3];
                s[3] = (s[3] ^ (s[3] >> 19)) ^ (t ^ (t >> 8));
            } else {
                const uint64_t u = s[0] ^ (s[0] >> 2);
                s[0] = s[1]; s[1] = s[2]; s[2] = s[3]; s[3] = s[4];
                s[4] = (s[4] ^ ((s[4] << 4) & m)) ^ (u ^ ((u << 1) & m));
            }
        };
        const size_t nw[3] = {1, 4, 5};
        for (int k = 0; k < 3; ++k) {
            std::vector<uint64_t> s0(nw[k]);
            for (auto &x : s0) x = rng() & m;
            // jump: X^J mod q_k
            const Poly r = pxpow(J, P.q[k]);
            std::vector<uint64_t> walk = s0, direct = s0, acc(nw[k], 0), sum(nw[k], 0), sumd(nw[k], 0);
            for (int b = 0; b < P.deg[k]; ++b) {
                if (pbit(r, b))
                    for (size_t i = 0; i < nw[k]; ++i) acc[i] ^= walk[i];
                step(k, walk);
            }
            for (uint64_t i = 0; i < J; ++i) {
                step(k, direct);
                for (size_t w = 0; w < nw[k]; ++w) sumd[w] ^= direct[w];
            }
            if (acc != direct) return set_error(CPRNG_E_HIP, "V1 generator jump differs from stepping");
            // geometric sum: sum_{i=1..J} A^i s0
            const Poly g = pgeomsum(J, P.q[k]);
            walk = s0;
            for (int b = 0; b < P.deg[k]; ++b) {
                if (pbit(g, b))
                    for (size_t i = 0; i < nw[k]; ++i) sum[i] ^= walk[i];
                step(k, walk);
            }
            if (sum != sumd) return set_error(CPRNG_E_HIP, "V1 aggregate sum differs from stepping");
        }
        return CPRNG_OK;
    }
    return set_error(CPRNG_E_INVAL, "the jump self-test covers V1, V2 and V4");
}
