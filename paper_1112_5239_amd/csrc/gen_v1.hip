// gen_v1.hip -- generate and consume kernels of the Listing-1 variant (V1; 32- and 64-bit words), instantiated from
// gen_kernels.inc in a source file of their own so the variants compile in
// parallel.
#include "internal.h"

#pragma clang fp contract(off)

namespace cprng_impl {
namespace {

#include "device_common.inc"
#include "gen_kernels.inc"
#include "consume_kernels.inc"
#include "chunk_kernels.inc"

}  // namespace

hipError_t launch_generate_v1(const GenArgs &a, bool w32, const LaunchCfg &c, hipStream_t st)
{
    return w32 ? gen_by_unroll<1, uint32_t>(a, c, st) : gen_by_unroll<1, uint64_t>(a, c, st);
}

hipError_t launch_consume_v1(const GenArgs &a, bool w32, const LaunchCfg &c, hipStream_t st)
{
    return w32 ? consume_by_unroll<1, uint32_t>(a, c, st) : consume_by_unroll<1, uint64_t>(a, c, st);
}

hipError_t launch_v1_chunks(const V1ChunkArgs &a, bool w32, hipStream_t st)
{
    return w32 ? v1_chunks_launch<uint32_t>(a, st) : v1_chunks_launch<uint64_t>(a, st);
}

}  // namespace cprng_impl
