// gf2.cpp -- jump-ahead polynomials for the plain variant.
//
// One step of the plain variant maps v = (xor128 words x,y,z,w ; chaotic
// state x) to A'v = (xor128 step ; x xor new w).  Every operation is a xor
// or a shift, so A' is a 160x160 matrix over GF(2) and the state after J
// steps is A'^J v.  If q(A') = 0 then A'^J = r(A') with r = X^J mod q, so a
// chunk of a stream can start J steps ahead after deg(q)+1 steps of
// accumulate-and-step (the output sequence is the prefix-xor of the strategy
// words, construction X of Section 8, and rides along in the same map).
//
// q is found here, once, as follows: p = the minimal polynomial of the
// xor128 output bits (Berlekamp-Massey on 512 bits; degree 128).  Writing
// A' in block form [[A,0],[eA,I]] gives q(A') = 0 for q = p(X)(X+1), since
// sum_k q_k A'^k has blocks q(A) = 0 and (A+I)^{-1}A(q(A) + q(1)I) = 0.  The
// result is checked by simulation before use.
#include <array>
#include <map>
#include <mutex>

#include "host.h"

namespace cprng_impl {

namespace {

struct Gen {
    uint32_t x, y, z, w, c;
    void step()
    {
        uint32_t t = x ^ (x << 11);
        x = y;
        y = z;
        z = w;
        w = (w ^ (w >> 19)) ^ (t ^ (t >> 8));
        c ^= w;
    }
};

// Polynomials of degree <= 191 as 3 words.
struct P3 {
    uint64_t w[3] = {0, 0, 0};
    bool bit(int i) const { return (w[i >> 6] >> (i & 63)) & 1u; }
    void flip(int i) { w[i >> 6] ^= 1ull << (i & 63); }
    int deg() const
    {
        for (int i = 191; i >= 0; --i)
            if (bit(i)) return i;
        return -1;
    }
};

std::once_flag g_once;
bool g_ok = false;
std::string g_why;
P3 g_q;          // modulus
int g_deg = 0;   // degree of q

// Berlekamp-Massey over GF(2); returns connection polynomial C with
// s_n = sum_{i=1..L} c_i s_{n-i}, and L.
int berlekamp_massey(const std::vector<uint8_t> &s, std::vector<uint8_t> &C)
{
    const size_t N = s.size();
    C.assign(N + 1, 0);
    std::vector<uint8_t> B(N + 1, 0), T;
    C[0] = B[0] = 1;
    int L = 0;
    size_t m = 1;
    for (size_t n = 0; n < N; ++n) {
        uint8_t d = s[n];
        for (int i = 1; i <= L; ++i) d ^= C[i] & s[n - i];
        if (d == 0) {
            ++m;
        } else if (2 * L <= (int)n) {
            T = C;
            for (size_t i = 0; i + m <= N; ++i) C[i + m] ^= B[i];
            L = (int)n + 1 - L;
            B = T;
            m = 1;
        } else {
            for (size_t i = 0; i + m <= N; ++i) C[i + m] ^= B[i];
            ++m;
        }
    }
    C.resize(L + 1);
    return L;
}

void init_once()
{
    // Minimal polynomial of the xor128 output bit 0 from a fixed state.
    Gen g{123456789u, 362436069u, 521288629u, 88675123u, 0u};
    std::vector<uint8_t> bits(512);
    for (auto &b : bits) {
        g.step();
        b = g.w & 1u;
    }
    std::vector<uint8_t> C;
    const int L = berlekamp_massey(bits, C);
    if (L != 128) {
        g_why = "xor128 linear complexity is not 128";
        return;
    }
    // characteristic polynomial p(X) = X^L C(1/X): coefficient of X^(L-i) is c_i
    P3 p;
    for (int i = 0; i <= L; ++i)
        if (C[i]) p.flip(L - i);
    // q = p * (X + 1)
    P3 q;
    for (int i = 0; i <= 128; ++i)
        if (p.bit(i)) {
            q.flip(i);
            q.flip(i + 1);
        }
    g_q = q;
    g_deg = q.deg();
    // Check sum_k q_k A'^{n+k} v = 0 on every one of the 160 bits for a few n.
    Gen v{0x9E3779B9u, 0x7F4A7C15u, 0x85EBCA6Bu, 0xC2B2AE35u, 0x27D4EB2Fu};
    std::vector<Gen> seq(g_deg + 8);
    for (auto &e : seq) {
        e = v;
        v.step();
    }
    for (int n = 0; n < 7; ++n) {
        Gen acc{0, 0, 0, 0, 0};
        for (int k = 0; k <= g_deg; ++k)
            if (q.bit(k)) {
                acc.x ^= seq[n + k].x; acc.y ^= seq[n + k].y; acc.z ^= seq[n + k].z;
                acc.w ^= seq[n + k].w; acc.c ^= seq[n + k].c;
            }
        if (acc.x | acc.y | acc.z | acc.w | acc.c) {
            g_why = "jump modulus does not annihilate the one-step map";
            return;
        }
    }
    g_ok = true;
}

// r = r * X mod q
inline void mulx(P3 &r)
{
    const bool top = r.bit(g_deg - 1);
    r.w[2] = (r.w[2] << 1) | (r.w[1] >> 63);
    r.w[1] = (r.w[1] << 1) | (r.w[0] >> 63);
    r.w[0] <<= 1;
    if (top) {
        // X^deg = q - X^deg (lower terms); clear the X^deg bit we just set.
        for (int j = 0; j < 3; ++j) r.w[j] ^= g_q.w[j];
    }
}

}  // namespace

bool jump_init(std::string *why)
{
    std::call_once(g_once, init_once);
    if (!g_ok && why) *why = g_why;
    return g_ok;
}

JPoly jump_one()
{
    JPoly r{{1, 0, 0}};
    return r;
}

JPoly jump_mul(const JPoly &a, const JPoly &b)
{
    P3 r;
    P3 A;
    for (int j = 0; j < 3; ++j) A.w[j] = a.w[j];
    // Horner over the bits of b from the top.
    for (int i = g_deg - 1; i >= 0; --i) {
        mulx(r);
        if ((b.w[i >> 6] >> (i & 63)) & 1u)
            for (int j = 0; j < 3; ++j) r.w[j] ^= A.w[j];
    }
    JPoly out;
    for (int j = 0; j < 3; ++j) out.w[j] = r.w[j];
    return out;
}

JPoly jump_xpow(uint64_t J)
{
    JPoly result = jump_one();
    P3 xb;
    xb.flip(1);                       // X (deg q > 1)
    JPoly base{{xb.w[0], xb.w[1], xb.w[2]}};
    while (J) {
        if (J & 1u) result = jump_mul(result, base);
        base = jump_mul(base, base);
        J >>= 1;
    }
    return result;
}

void jump_pack(const JPoly &p, uint32_t out[5])
{
    out[0] = (uint32_t)p.w[0];
    out[1] = (uint32_t)(p.w[0] >> 32);
    out[2] = (uint32_t)p.w[1];
    out[3] = (uint32_t)(p.w[1] >> 32);
    out[4] = (uint32_t)(p.w[2] & 1u);   // coefficient of X^128
}

}  // namespace cprng_impl

namespace cprng_impl {

namespace {
std::mutex g_tab_mu;
// Per chunk length: X^(k*chunk) mod q for k = 0, 1, 2, ...
std::map<uint32_t, std::vector<JPoly>> g_tables;
}  // namespace

void jump_table(uint32_t chunk, uint32_t kcap, std::vector<uint32_t> &out)
{
    std::lock_guard<std::mutex> lk(g_tab_mu);
    std::vector<JPoly> &r = g_tables[chunk];
    if (r.size() < kcap) {
        const JPoly step = jump_xpow(chunk);
        if (r.empty()) r.push_back(jump_xpow(0));
        r.reserve(kcap);
        while (r.size() < kcap) r.push_back(jump_mul(r.back(), step));
    }
    out.assign((size_t)kcap * 5, 0u);
    for (uint32_t k = 0; k < kcap; ++k) jump_pack(r[k], &out[(size_t)k * 5]);
}

}  // namespace cprng_impl
