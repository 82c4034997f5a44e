// gen_v2.hip -- generate and consume kernels of the neighbour-exchange variant (V2, Algorithm 4), instantiated from
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

hipError_t launch_generate_v2(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    return gen_by_unroll<2, uint32_t>(a, c, st);
}

hipError_t launch_consume_v2(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    return consume_by_unroll<2, uint32_t>(a, c, st);
}

hipError_t launch_group_chunks_v2(const GroupJumpArgs &a, hipStream_t st)
{
    return group_chunks_launch<2>(a, st);
}

}  // namespace cprng_impl
