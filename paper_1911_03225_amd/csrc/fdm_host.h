// fdm_host.h -- host-side validation and set-up shared by the C-ABI entry
// points: descriptor checks, the step and its stability bound, the tiling
// and the stage sequence of an instance.
#pragma once

#include <stdint.h>

#include <string>

#include "../../include/fdm.h"
#include "fdm_internal.h"

namespace fdm {
namespace host {

bool finite_pos(double v);

// "" if the descriptor is valid, else the reason (no HIP call).
std::string check_desc(const fdm_transport_desc &d);

// Largest float not above x (x > 0).
float round_down_float(double x);

// "" if the step the descriptor implies is within the stability bound
// (nu2 = dt (S1/dx + S2/dy) <= 1, or <= 1/2 for one limited forward-Euler
// stage, order 1), else the reason.  smax_law: max |v0| (LAW with a fixed
// dt; unused otherwise).
std::string check_courant(const fdm_transport_desc &d, int32_t order, double smax_law);

// max speed of a descriptor without a celerity field: |v0| (LAW, float32) or
// max(|V1|/dx, |V2|/dy) min(dx, dy) (PRESCRIBED).
double smax_uniform(const fdm_transport_desc &d);

// The float32 step: the given dt, or cfl min(dx,dy) / smax rounded down
// (the unit-speed step when smax = 0).
float step_dt(const fdm_transport_desc &d, double smax);

// The device view of one instance with step dt and stage buffer (w11, w12);
// the state pointers and the tiling are left unset.
void fill_inst(InstDev &I, const fdm_transport_desc &d, float dt, void *w11, void *w12);

// Rows per wave tile of the stage kernels: `requested`, or the default rule
// for `strip_rows` (strip, row) pairs in the launch.
int pick_rows(int64_t strip_rows, int ny, int requested);

// (strip, row) pairs of one instance in the stage kernels' tiling.
int64_t strip_rows_of(const fdm_transport_desc &d);

// Stage launches of step number `step` for an integrator order (1 Euler,
// 2 Heun, 3 explicit midpoint): the modes in order, their count returned.
int stage_modes(int32_t order, int32_t step, int modes[2]);

// Message of the last failed call without a context (fdm_last_error(NULL)).
void set_init_error(const std::string &msg);

}  // namespace host
}  // namespace fdm
