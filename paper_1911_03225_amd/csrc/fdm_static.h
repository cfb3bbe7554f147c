// fdm_static.h -- internal interface of the static (stress) solve of the
// layer case and of the coupled velocity law; see fdm_static.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "fdm_internal.h"

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
// the mean stress *sigma_bar (a device double, read when the kernel runs)
// on s.  a11/a12 are read only; tau13 is written.  slip (may be null): a
// coupled step's pending slip update, run by the first kernel (before
// anything reads the mean stress or slip).
StaticStatus static_plan_run(StaticPlan *p, const void *a11, const void *a12, void *tau13, const double *sigma_bar,
                             const SlipArgs *slip, hipStream_t s, std::string &err);

// As static_plan_run, and also phi (= U^p_13) at the nodes with the mean
// *phi_mean (a device double), from the same forward transforms.
StaticStatus static_plan_run_phi(StaticPlan *p, const void *a11, const void *a12, void *tau13, void *phi,
                                 const double *sigma_bar, const double *phi_mean, const SlipArgs *slip,
                                 hipStream_t s, std::string &err);

// Two device doubles owned by the plan, for callers that hold the mean
// stress and slip on the host (upload them before a run).
double *static_plan_scalars(StaticPlan *p);

// Celerity at the nodes, written as float32, m = mobility * mfield[i] (mfield
// may be null):
//   wiggly = false: v0 = -m S_tau0(tau13), S the soft threshold;
//   wiggly = true:  v0 = m (tau_y cos(phi / beta) - tau13).
struct LawParams {
    bool wiggly;
    double tau0, mobility, tau_y, beta;
    const float *mfield;
};
// Also writes one max |v0| partial per block (NaN marks a non-finite value)
// into partial[0 .. velocity_law_blocks(n)), for the step size.
constexpr int kLawBlocks = 1024;
int velocity_law_blocks(int64_t n);
StaticStatus velocity_law(const void *tau13, const void *phi, bool f64, float *v0, int64_t n, const LawParams &law,
                          float *partial, hipStream_t s, std::string &err);

}  // namespace fdm
