// fdm_stage_f32.hip -- FP32-arithmetic instances of the stage kernels
// (float32 state).
//
// Implicit multiply-add contraction is off: the fused operations are the
// explicit madd() calls of the stage code, the same in every unrolled copy of
// the row loop and in every kernel instance, so results do not depend on the
// tile height or on the batched / plain schedule.
#pragma clang fp contract(off)
#include "fdm_stage.h"

namespace fdm {

hipError_t launch_stage_f32(const InstDev &I, int mode, hipStream_t s)
{
    return launch_stage_r<float, float>(I, mode, s);
}

namespace {
template <bool MID>
hipError_t launch_fused_r(const InstDev &I, int dir, hipStream_t s)
{
    if (I.vkind != VK_LAW && I.vkind != VK_PRESCRIBED) return hipErrorInvalidValue;   // semi-discrete scheme only
    return with_limiter<true>(I.limiter, [&](auto t) -> hipError_t {
        constexpr int L = decltype(t)::value;
        if (I.vkind == VK_PRESCRIBED) return launch_fused_t<L, VK_PRESCRIBED, false, MID>(I, dir, s);
        if (I.v0f != nullptr) return launch_fused_t<L, VK_LAW, true, MID>(I, dir, s);
        return launch_fused_t<L, VK_LAW, false, MID>(I, dir, s);
    });
}
}  // namespace

hipError_t launch_fused(const InstDev &I, int dir, bool mid, hipStream_t s)
{
    return mid ? launch_fused_r<true>(I, dir, s) : launch_fused_r<false>(I, dir, s);
}

hipError_t launch_fused_batched(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles, int dir,
                                bool mid, hipStream_t s)
{
    const int64_t blocks = (total_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_xcd = (int)((blocks + 7) / 8);
    const dim3 grid(8 * per_xcd), block(kBlock);
    if (mid) {
        if (dir)
            hipLaunchKernelGGL((fused_kernel_batched<1, true>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles,
                               per_xcd);
        else
            hipLaunchKernelGGL((fused_kernel_batched<0, true>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles,
                               per_xcd);
    } else {
        if (dir)
            hipLaunchKernelGGL((fused_kernel_batched<1, false>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles,
                               per_xcd);
        else
            hipLaunchKernelGGL((fused_kernel_batched<0, false>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles,
                               per_xcd);
    }
    return hipGetLastError();
}

hipError_t launch_stage_batched_f32(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles,
                                    int mode, bool fd, hipStream_t s)
{
    return launch_batched_r<float, float>(d_inst, d_tile_inst, total_tiles, mode, fd, s);
}

}  // namespace fdm
