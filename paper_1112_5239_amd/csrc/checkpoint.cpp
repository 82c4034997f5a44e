// checkpoint.cpp -- versioned, self-describing checkpoints of a handle's
// stream states.
//
// The GPU kernels write every stream's state back at the end of a call
// (Algorithms 3 and 4 store their internal variables after the loop), so the
// device state between calls is a complete checkpoint of the generator.  A
// checkpoint image is a 256-byte header followed by the states, stream after
// stream in the order of cprng_get_state:
//
//   offset  size  field
//   0       8     magic "CPRNGCKP"
//   8       4     format version (1)
//   12      4     header bytes (256)
//   16      4     variant | flags of the handle
//   20      4     n_streams
//   24      4     state words per stream
//   28      4     group size C (0 for the variants without exchange)
//   32      64    comb1[0..63] (V2/V4: entry j mod C; else 0)
//   96      64    comb2[0..63]
//   160     8     payload bytes (n_streams * words * 4)
//   168     8     FNV-1a 64 of the payload
//   176     8     FNV-1a 64 of header bytes 0..175
//   184     72    zero
//
// All integers little-endian.  Loading checks every field against the
// handle, both hashes, and the state rules of cprng_set_state.
#include <cstring>
#include <vector>

#include "host.h"

namespace {

constexpr char kMagic[8] = {'C', 'P', 'R', 'N', 'G', 'C', 'K', 'P'};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeader = 256;

// FNV-1a, 64-bit (Fowler, Noll, Vo): offset basis and prime as published.
uint64_t fnv1a64(const unsigned char *p, size_t n)
{
    uint64_t h = 14695981039346656037ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

void put32(unsigned char *p, uint32_t v)
{
    for (int i = 0; i < 4; ++i) p[i] = (unsigned char)(v >> (8 * i));
}
void put64(unsigned char *p, uint64_t v)
{
    for (int i = 0; i < 8; ++i) p[i] = (unsigned char)(v >> (8 * i));
}
uint32_t get32(const unsigned char *p)
{
    uint32_t v = 0;
    for (int i = 0; i < 4; ++i) v |= (uint32_t)p[i] << (8 * i);
    return v;
}
uint64_t get64(const unsigned char *p)
{
    uint64_t v = 0;
    for (int i = 0; i < 8; ++i) v |= (uint64_t)p[i] << (8 * i);
    return v;
}

// Header of handle h (hashes filled by the caller).
void make_header(const cprng_t *h, unsigned char *hd)
{
    std::memset(hd, 0, kHeader);
    std::memcpy(hd, kMagic, 8);
    put32(hd + 8, kVersion);
    put32(hd + 12, (uint32_t)kHeader);
    put32(hd + 16, h->variant | h->flags);
    put32(hd + 20, h->ns);
    put32(hd + 24, h->words);
    put32(hd + 28, h->group);
    if (h->variant == CPRNG_V2_SHMEM || h->variant == CPRNG_V4_XOR64) {
        std::memcpy(hd + 32, h->comb1, 64);
        std::memcpy(hd + 96, h->comb2, 64);
    }
    put64(hd + 160, (uint64_t)h->ns * h->words * 4u);
}

}  // namespace

using namespace cprng_impl;

extern "C" size_t cprng_checkpoint_bytes(const cprng_t *h)
{
    if (!h) return 0;
    return kHeader + (size_t)h->ns * h->words * sizeof(uint32_t);
}

extern "C" int cprng_checkpoint_save(cprng_t *h, void *host_buf, size_t bytes)
{
    if (!h || !host_buf) return set_error(CPRNG_E_INVAL, "NULL argument");
    if (bytes != cprng_checkpoint_bytes(h)) return set_error(CPRNG_E_INVAL, "bytes must be cprng_checkpoint_bytes(h)");
    unsigned char *hd = static_cast<unsigned char *>(host_buf);
    std::vector<uint32_t> words((size_t)h->ns * h->words);
    const int rc = cprng_get_state(h, words.data(), words.size());
    if (rc) return rc;
    std::memcpy(hd + kHeader, words.data(), words.size() * sizeof(uint32_t));
    make_header(h, hd);
    put64(hd + 168, fnv1a64(hd + kHeader, words.size() * sizeof(uint32_t)));
    put64(hd + 176, fnv1a64(hd, 176));
    return CPRNG_OK;
}

extern "C" int cprng_checkpoint_load(cprng_t *h, const void *host_buf, size_t bytes)
{
    if (!h || !host_buf) return set_error(CPRNG_E_INVAL, "NULL argument");
    const unsigned char *hd = static_cast<const unsigned char *>(host_buf);
    if (bytes < kHeader) return set_error(CPRNG_E_INVAL, "checkpoint shorter than its header");
    if (std::memcmp(hd, kMagic, 8) != 0) return set_error(CPRNG_E_INVAL, "not a checkpoint (magic)");
    if (get32(hd + 8) != kVersion) return set_error(CPRNG_E_INVAL, "unsupported checkpoint version");
    if (get32(hd + 12) != kHeader) return set_error(CPRNG_E_INVAL, "unexpected checkpoint header size");
    if (get64(hd + 176) != fnv1a64(hd, 176)) return set_error(CPRNG_E_INVAL, "checkpoint header hash mismatch");
    unsigned char want[kHeader];
    make_header(h, want);
    if (std::memcmp(hd + 16, want + 16, 4) != 0) return set_error(CPRNG_E_INVAL, "checkpoint of another variant or flags");
    if (std::memcmp(hd + 20, want + 20, 8) != 0)
        return set_error(CPRNG_E_INVAL, "checkpoint of another stream count or state size");
    if (std::memcmp(hd + 28, want + 28, 4 + 128) != 0)
        return set_error(CPRNG_E_INVAL, "checkpoint of another group size or combination arrays");
    const uint64_t payload = get64(hd + 160);
    if (payload != get64(want + 160) || bytes != kHeader + payload)
        return set_error(CPRNG_E_INVAL, "checkpoint payload size mismatch");
    if (get64(hd + 168) != fnv1a64(hd + kHeader, (size_t)payload))
        return set_error(CPRNG_E_INVAL, "checkpoint payload hash mismatch");
    std::vector<uint32_t> words((size_t)h->ns * h->words);
    std::memcpy(words.data(), hd + kHeader, (size_t)payload);
    return cprng_set_state(h, words.data(), words.size());
}
