// fdm_stage_f64.hip -- FP64-arithmetic instances of the stage kernels
// (float32 or float64 state).
//
// Multiply-add contraction is off in this file: a fused a*b + c*d rounds one
// product and not the other, which breaks exact ties between mirrored corner
// values (e.g. |p|^2 of (px-, py+) and (px+, py-) on x<->y symmetric data).
// The speed v0 p/|p| is discontinuous at p = 0, so such 1e-17 asymmetries
// grow over hundreds of steps; with float64 state nothing rounds them away.
#pragma clang fp contract(off)
#include "fdm_stage.h"

namespace fdm {

hipError_t launch_stage_f64(const InstDev &I, int mode, bool f64_state, hipStream_t s)
{
    return f64_state ? launch_stage_r<double, double>(I, mode, s) : launch_stage_r<double, float>(I, mode, s);
}

hipError_t launch_stage_batched_f64(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles,
                                    int mode, bool fd, bool f64_state, hipStream_t s)
{
    return f64_state ? launch_batched_r<double, double>(d_inst, d_tile_inst, total_tiles, mode, fd, s)
                     : launch_batched_r<double, float>(d_inst, d_tile_inst, total_tiles, mode, fd, s);
}

}  // namespace fdm
