// gen_v4.hip -- generate and consume kernels of the xor64 exchange variant
// (V4: Algorithm 4 with xor64 as each stream's generator), instantiated from
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

hipError_t launch_generate_v4(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    return gen_by_unroll<4, uint32_t>(a, c, st);
}

hipError_t launch_consume_v4(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    return consume_by_unroll<4, uint32_t>(a, c, st);
}

hipError_t launch_group_chunks_v4(const GroupJumpArgs &a, hipStream_t st)
{
    return group_chunks_launch<4>(a, st);
}

}  // namespace cprng_impl
