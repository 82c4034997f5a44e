// noalloc.hip -- batched uneven streams of the plain variant with no device
// allocation: the work buffers of the chunk kernels (queue counters, run
// descriptors, commit list, jump table, end-state staging) live in one
// file-scope device array instead of buffers the handle allocates.  The
// kernels are those of cprng_generate_ragged; only where their buffers live
// differs, and the launches are enqueued directly (no graph, whose
// instantiation allocates).
#include <cstring>
#include <mutex>
#include <vector>

#include "host.h"
#include "tune.h"

// Each device the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, not the device array:
// every host use goes through the per-device address from scratch_base().
static __device__ __align__(256) unsigned char scratch[CPRNG_NOALLOC_SCRATCH_BYTES];

namespace cprng_impl {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (which must be current),
// looked up once per device.
int scratch_base(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return set_error(CPRNG_E_UNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(CPRNG_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return CPRNG_OK;
}

constexpr size_t round256(size_t v) { return (v + 255u) & ~(size_t)255u; }

}  // namespace
}  // namespace cprng_impl

using namespace cprng_impl;

extern "C" int cprng_generate_ragged_noalloc(cprng_t *h, uint32_t *out, const uint64_t *lengths,
                                             const uint64_t *offsets, cprng_stream_t stream)
{
    if (!h) return set_error(CPRNG_E_INVAL, "NULL handle");
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != h->device && hipSetDevice(h->device) != hipSuccess) return set_error(CPRNG_E_HIP, "hipSetDevice failed");
    struct Restore {
        int dev, prev;
        ~Restore()
        {
            if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
        }
    } restore{h->device, prev};

    V0Launch p;
    int rc = plan_ragged_v0(h, out, lengths, offsets, p);
    if (rc) return rc;
    if (p.runs.empty()) return CPRNG_OK;

    // Layout of the array: counters | runs | commit ids | jump table | end states.
    const size_t off_runs = 256;
    const size_t off_ids = off_runs + round256(p.runs.size() * sizeof(RunDesc));
    const size_t off_polys = off_ids + round256(p.ids.size() * sizeof(uint32_t));
    const size_t off_next = off_polys + round256((size_t)p.kcap * 5u * sizeof(uint32_t));
    const size_t end = off_next + round256((size_t)5u * h->ns * sizeof(uint32_t));
    if (end > CPRNG_NOALLOC_SCRATCH_BYTES)
        return set_error(CPRNG_E_INVAL,
                         "allocation-free path: " + std::to_string(p.runs.size()) + " runs, " +
                             std::to_string(p.kcap) + " jump rows and " + std::to_string(h->ns) +
                             " streams need " + std::to_string(end) + " bytes of scratch, above its " +
                             std::to_string((size_t)CPRNG_NOALLOC_SCRATCH_BYTES) + " bytes");
    unsigned char *base = nullptr;
    rc = scratch_base(h->device, &base);
    if (rc) return rc;

    // Descriptors staged in host memory and copied into the array in stream
    // order (after any earlier work on `stream` that still reads it).
    std::vector<uint32_t> polys;
    jump_table(p.chunk, p.kcap, polys);
    std::vector<unsigned char> stage(off_next - off_runs, 0);
    std::memcpy(stage.data(), p.runs.data(), p.runs.size() * sizeof(RunDesc));
    std::memcpy(stage.data() + (off_ids - off_runs), p.ids.data(), p.ids.size() * sizeof(uint32_t));
    std::memcpy(stage.data() + (off_polys - off_runs), polys.data(), polys.size() * sizeof(uint32_t));
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(base + off_runs, stage.data(), stage.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_error(e, "copy of the run descriptors into scratch");
    rc = timing_begin(h, st);
    if (rc) return rc;
    e = launch_ragged_v0(h, p, reinterpret_cast<const RunDesc *>(base + off_runs),
                         reinterpret_cast<const uint32_t *>(base + off_ids),
                         reinterpret_cast<const uint32_t *>(base + off_polys), reinterpret_cast<uint32_t *>(base),
                         reinterpret_cast<uint32_t *>(base + off_next), st);
    if (e != hipSuccess) return hip_error(e, "allocation-free chunk kernels");
    return timing_end(h, st);
}
