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

template <typename T>
int ensure_buf(T **p, size_t *cap, size_t n)
{
    if (*cap >= n && *p) return CPRNG_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
        return set_error(CPRNG_E_NOMEM, "hipMalloc of group-jump buffers failed");
    *cap = n;
    return CPRNG_OK;
}

// Store round of the chunk kernels: the tuning's unroll when it is 32, 64 or
// 128 words, else the default.
uint32_t chunk_round(const cprng_t *h)
{
    const uint32_t u = h->tuning.unroll;
    return (u == 32 || u == 64 || u == 128) ? u : 64u;
}

// Waves per workgroup of the chunk kernels: 4 for a tuning block of 256, 1
// for 64, else the default.
uint32_t chunk_wg_waves(const cprng_t *h)
{
    const uint32_t b = h->tuning.block;
    return b == 256 ? 4u : b == 64 ? 1u : 4u;
}

// Waves of a chunk kernel that stay resident per CU, from its tile's LDS
// (the kernels' other limits are looser).
uint64_t chunk_resident_waves(const cprng_t *h)
{
    const uint64_t K = chunk_round(h), W = chunk_wg_waves(h);
    const uint64_t wg_lds = W * 64u * (K + 1u) * 4u;
    return std::min<uint64_t>(32u, (kMaxLdsBytes / wg_lds) * W);
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

}  // namespace

int ragged_groups(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets,
                  hipStream_t st)
{
    const uint32_t C = h->group;
    for (uint32_t g0 = 0; g0 < h->ns; g0 += C)
        for (uint32_t j = 1; j < C; ++j)
            if (lengths[g0 + j] != lengths[g0])
                return set_error(CPRNG_E_INVAL, "V2/V4: lengths must be equal within each group of C streams");
    int rc = group_minpoly(h);
    if (rc) return rc;
    const uint32_t n_groups = h->ns / C;
    uint64_t group_steps = 0, max_len = 0;
    for (uint32_t g = 0; g < n_groups; ++g) {
        group_steps += lengths[(size_t)g * C];
        max_len = std::max(max_len, lengths[(size_t)g * C]);
    }
    if (group_steps == 0) return CPRNG_OK;
    // Chunk: the shortest (a multiple of 64, at least 16 x the jump's length,
    // at most 2^20) whose items all fit one pass of the chip's resident waves.
    // The exchange reads' latency wants many waves, fewer and longer runs in
    // flight store better, and a second pass that is only partly full costs
    // nearly a whole chunk's time.  Resident waves per CU follow from the
    // tile's LDS (the kernel's other limits are looser); the pass is filled
    // to 31/32, so a workgroup the dispatcher places late does not start a
    // second one.
    uint64_t chunk = h->tuning.chunk ? h->tuning.chunk : 0;
    if (!chunk) {
        const uint64_t cap = (uint64_t)h->n_cu * chunk_resident_waves(h) * (64u / C) * 31u / 32u;   // 3% slack
        chunk = fit_chunk(16ull * (uint64_t)h->gj_deg, cap, [&](uint64_t c) {
            uint64_t n = 0;
            for (uint32_t g = 0; g < n_groups; ++g) n += (lengths[(size_t)g * C] + c - 1) / c;
            return n;
        });
    }
    std::vector<GroupItem> items;
    for (uint32_t g = 0; g < n_groups; ++g) {
        const uint64_t L = lengths[(size_t)g * C];
        for (uint64_t a = 0, c = 0; a < L; a += chunk, ++c) {
            GroupItem it{};
            it.group = g;
            it.row = (uint32_t)c;
            it.start = a;
            it.len = std::min(chunk, L - a);
            it.last = (a + chunk >= L) ? 1u : 0u;
            items.push_back(it);
        }
    }
    const uint32_t n_rows = (uint32_t)((max_len + chunk - 1) / chunk);
    std::vector<uint32_t> rows;
    group_jump_rows(h, chunk, n_rows, rows);
    std::vector<uint64_t> offs(h->ns);
    uint64_t acc = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        offs[s] = offsets ? offsets[s] : acc;
        acc += lengths[s];
    }
    // The buffers are reused by the next call: wait for the previous one.
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    const size_t nwords = (size_t)h->ns * h->words;
    if ((rc = ensure_buf(&h->d_gj_next, &h->gj_next_cap, nwords))) return rc;
    if ((rc = ensure_buf(&h->d_gj_items, &h->gj_items_cap, items.size()))) return rc;
    if ((rc = ensure_buf(&h->d_gj_rows, &h->gj_rows_cap, rows.size()))) return rc;
    if ((rc = ensure_buf(&h->d_gj_offsets, &h->gj_offsets_cap, offs.size()))) return rc;
    HIP_TRY(hipMemcpy(h->d_gj_items, items.data(), items.size() * sizeof(GroupItem), hipMemcpyHostToDevice),
            "hipMemcpy items");
    HIP_TRY(hipMemcpy(h->d_gj_rows, rows.data(), rows.size() * sizeof(uint32_t), hipMemcpyHostToDevice),
            "hipMemcpy jump rows");
    HIP_TRY(hipMemcpy(h->d_gj_offsets, offs.data(), offs.size() * sizeof(uint64_t), hipMemcpyHostToDevice),
            "hipMemcpy offsets");
    GroupJumpArgs a;
    fill_gen_args(h, a.g);
    a.state_next = h->d_gj_next;
    a.items = h->d_gj_items;
    a.n_items = (uint32_t)items.size();
    a.rows = h->d_gj_rows;
    a.row_words = (uint32_t)((h->gj_deg + 31) / 32);
    a.deg = (uint32_t)h->gj_deg;
    a.round = chunk_round(h);
    a.wg_waves = chunk_wg_waves(h);
    a.out = out;
    a.offsets = h->d_gj_offsets;
    int trc = timing_begin(h, st);
    if (trc) return trc;
    HIP_TRY(launch_copy(h->d_gj_next, h->d_state, nwords, st), "state copy");
    HIP_TRY(launch_group_chunks(a, (int)h->variant, st), "group chunk kernel launch");
    HIP_TRY(launch_copy(h->d_state, h->d_gj_next, nwords, st), "state commit");
    return timing_end(h, st);
}

int ragged_v1(cprng_t *h, uint32_t *out, const uint64_t *lengths, const uint64_t *offsets, hipStream_t st)
{
    const bool w32 = (h->flags & CPRNG_F_V1_W32) != 0;
    const bool xor64 = (h->flags & CPRNG_F_V1_XOR64) != 0;
    const V1Polys &P = v1_polys(w32 ? 32 : 64, xor64 ? 7u : 17u, xor64 ? 17u : 5u);
    if (!P.ok) return set_error(CPRNG_E_HIP, "V1 jump-ahead: no annihilating polynomial found");
    uint64_t total = 0, max_len = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        total += lengths[s];
        max_len = std::max(max_len, lengths[s]);
    }
    if (total == 0) return CPRNG_OK;
    const uint64_t jump_steps = (uint64_t)(P.deg[0] + P.deg[1] + P.deg[2]);
    // Chunk: one lane per chunk.  The shortest (a multiple of 64, at least
    // 16 x the jump's steps, at most 2^20) whose chunks fill at most 31/32 of
    // two passes of the generating kernel's resident waves: its time follows
    // whole passes (a last pass that is mostly empty costs a whole chunk's
    // time), and the aggregate pass's serial xorwow chains want the twice as
    // many waves that two passes' worth of chunks give it.
    uint64_t chunk = h->tuning.chunk ? h->tuning.chunk : 0;
    if (!chunk) {
        const uint64_t cap = 2u * (uint64_t)h->n_cu * chunk_resident_waves(h) * 64u * 31u / 32u;
        chunk = fit_chunk(16ull * jump_steps, cap, [&](uint64_t c) {
            uint64_t n = 0;
            for (uint32_t s = 0; s < h->ns; ++s) n += (lengths[s] + c - 1) / c;
            return n;
        });
    }
    std::vector<V1Item> items;
    for (uint32_t s = 0; s < h->ns; ++s) {
        const uint32_t first = (uint32_t)items.size();
        for (uint64_t a = 0, c = 0; a < lengths[s]; a += chunk, ++c) {
            V1Item it{};
            it.stream = s;
            it.row = (uint32_t)c;
            it.start = a;
            it.len = std::min(chunk, lengths[s] - a);
            it.last = (a + chunk >= lengths[s]) ? 1u : 0u;
            it.first = first;
            items.push_back(it);
        }
    }
    if (items.size() > 0xFFFFFFFFull) return set_error(CPRNG_E_INVAL, "too many chunks");
    const uint32_t n_rows = (uint32_t)((max_len + chunk - 1) / chunk);
    uint32_t wk[3], off[3];
    uint32_t row_words = 0;
    for (int k = 0; k < 3; ++k) {
        wk[k] = (uint32_t)((P.deg[k] + 31) / 32);
        off[k] = row_words;
        row_words += wk[k];
    }
    // rows 0..n_rows-1: X^(c * chunk) per generator; row n_rows: the sums
    // sum_{i=1..chunk} X^i of the xorshift and xor128 maps (full chunks'
    // aggregates)
    std::vector<uint32_t> rows((size_t)(n_rows + 1) * row_words, 0);
    for (int k = 0; k < 2; ++k) {
        const Poly g = pgeomsum(chunk, P.q[k]);
        for (int b = 0; b < P.deg[k]; ++b)
            if (pbit(g, b)) rows[(size_t)n_rows * row_words + off[k] + (b >> 5)] |= 1u << (b & 31);
    }
    for (int k = 0; k < 3; ++k) {
        const Poly base = pxpow(chunk, P.q[k]);
        Poly r{1};
        pmod(r, P.q[k]);
        for (uint32_t c = 0; c < n_rows; ++c) {
            for (int b = 0; b < P.deg[k]; ++b)
                if (pbit(r, b)) rows[(size_t)c * row_words + off[k] + (b >> 5)] |= 1u << (b & 31);
            r = pmulmod(r, base, P.q[k]);
        }
    }
    std::vector<uint64_t> offs(h->ns);
    uint64_t acc = 0;
    for (uint32_t s = 0; s < h->ns; ++s) {
        offs[s] = offsets ? offsets[s] : acc;
        acc += lengths[s];
    }
    // aggregate pass order: full chunks, then the shorter last ones
    std::vector<uint32_t> order;
    order.reserve(items.size());
    for (int pass = 0; pass < 2; ++pass)
        for (uint32_t i = 0; i < (uint32_t)items.size(); ++i)
            if ((items[i].len == chunk) == (pass == 0)) order.push_back(i);
    // The buffers are reused by the next call: wait for the previous one.
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    const size_t nwords = (size_t)h->ns * h->words;
    int rc;
    if ((rc = ensure_buf(&h->d_gj_next, &h->gj_next_cap, nwords))) return rc;
    if ((rc = ensure_buf(&h->d_v1_items, &h->v1_items_cap, items.size()))) return rc;
    if ((rc = ensure_buf(&h->d_v1_order, &h->v1_order_cap, order.size()))) return rc;
    HIP_TRY(hipMemcpy(h->d_v1_order, order.data(), order.size() * sizeof(uint32_t), hipMemcpyHostToDevice),
            "hipMemcpy order");
    if ((rc = ensure_buf(&h->d_v1_agg, &h->v1_agg_cap, items.size()))) return rc;
    if ((rc = ensure_buf(&h->d_gj_rows, &h->gj_rows_cap, rows.size()))) return rc;
    if ((rc = ensure_buf(&h->d_gj_offsets, &h->gj_offsets_cap, offs.size()))) return rc;
    HIP_TRY(hipMemcpy(h->d_v1_items, items.data(), items.size() * sizeof(V1Item), hipMemcpyHostToDevice),
            "hipMemcpy items");
    HIP_TRY(hipMemcpy(h->d_gj_rows, rows.data(), rows.size() * sizeof(uint32_t), hipMemcpyHostToDevice),
            "hipMemcpy jump rows");
    HIP_TRY(hipMemcpy(h->d_gj_offsets, offs.data(), offs.size() * sizeof(uint64_t), hipMemcpyHostToDevice),
            "hipMemcpy offsets");
    V1ChunkArgs a;
    fill_gen_args(h, a.g);
    a.state_next = h->d_gj_next;
    a.items = h->d_v1_items;
    a.n_items = (uint32_t)items.size();
    a.row_words = row_words;
    a.deg1 = (uint32_t)P.deg[0];
    a.deg2 = (uint32_t)P.deg[1];
    a.deg3 = (uint32_t)P.deg[2];
    a.off2 = off[1];
    a.off3 = off[2];
    a.rows = h->d_gj_rows;
    a.agg = h->d_v1_agg;
    a.out = out;
    a.offsets = h->d_gj_offsets;
    a.chunk = chunk;
    a.sum_row = n_rows;
    a.round = chunk_round(h);
    a.wg_waves = chunk_wg_waves(h);
    a.order = h->d_v1_order;
    int trc = timing_begin(h, st);
    if (trc) return trc;
    HIP_TRY(launch_copy(h->d_gj_next, h->d_state, nwords, st), "state copy");
    HIP_TRY(launch_v1_chunks(a, w32, st), "V1 chunk kernels launch");
    HIP_TRY(launch_copy(h->d_state, h->d_gj_next, nwords, st), "state commit");
    return timing_end(h, st);
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

namespace cprng_impl {
void destroy_group_buffers(cprng_t *h)
{
    if (h->d_v1_items) (void)hipFree(h->d_v1_items);
    if (h->d_v1_agg) (void)hipFree(h->d_v1_agg);
    if (h->d_v1_order) (void)hipFree(h->d_v1_order);
    h->d_v1_items = nullptr;
    h->d_v1_agg = nullptr;
    h->d_v1_order = nullptr;
    if (h->d_gj_next) (void)hipFree(h->d_gj_next);
    if (h->d_gj_items) (void)hipFree(h->d_gj_items);
    if (h->d_gj_rows) (void)hipFree(h->d_gj_rows);
    if (h->d_gj_offsets) (void)hipFree(h->d_gj_offsets);
    h->d_gj_next = nullptr;
    h->d_gj_items = nullptr;
    h->d_gj_rows = nullptr;
    h->d_gj_offsets = nullptr;
}

}  // namespace cprng_impl
