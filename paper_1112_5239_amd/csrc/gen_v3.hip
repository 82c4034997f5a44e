// gen_v3.hip -- generate and consume kernels of the BBS-based variant (V3, Algorithm 5), instantiated from
// gen_kernels.inc in a source file of their own so the variants compile in
// parallel.
#include "internal.h"

#pragma clang fp contract(off)

namespace cprng_impl {
namespace {

#include "device_common.inc"
#include "gen_kernels.inc"
#include "consume_kernels.inc"

}  // namespace

hipError_t launch_generate_v3(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    return gen_by_unroll<3, uint32_t>(a, c, st);
}

hipError_t launch_consume_v3(const GenArgs &a, const LaunchCfg &c, hipStream_t st)
{
    return consume_by_unroll<3, uint32_t>(a, c, st);
}

}  // namespace cprng_impl
