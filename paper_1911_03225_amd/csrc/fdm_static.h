// fdm_static.h -- internal interface of the static (stress) solve of the
// layer case and of the coupled velocity law; see fdm_static.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace fdm {

enum class StaticStatus { Ok, Device, OutOfMemory };

struct StaticParams {
    int nx, ny;
    double dx, dy;       // dx == dy: cubic voxels, x3 spacing dx
    double mu, lambda;
    int h, n3;           // layer and cell height in voxels, 1 <= h <= n3
    bool f64;            // double arrays and FFT, else float
};

struct StaticPlan;

// Builds the multiplier table and the FFT plans (synchronizes s).
StaticStatus static_plan_create(const StaticParams &q, hipStream_t s, StaticPlan **out, std::string &err);
void static_plan_destroy(StaticPlan *p);

// Enqueues tau13 = layer average of sigma13 for densities (a11, a12) and
// mean stress sigma_bar on s.  a11/a12 are read only; tau13 is written.
StaticStatus static_plan_run(StaticPlan *p, const void *a11, const void *a12, void *tau13, double sigma_bar,
                             hipStream_t s, std::string &err);

// v0 = -S_tau0(tau13) * mobility (soft threshold), written as float32.
StaticStatus velocity_law(const void *tau13, bool f64, float *v0, int64_t n, double tau0, double mobility,
                          hipStream_t s, std::string &err);

}  // namespace fdm
