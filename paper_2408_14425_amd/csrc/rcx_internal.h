// rcx_internal.h -- shared declarations of librcx's host code and kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/rcx.h"

namespace rcx {

// Geometry of one cascade as the march/merge kernel sees it.
struct LevelDesc {
    int32_t px, pz;     // probes per axis
    int32_t nd;         // directions
    int32_t qx, qz;     // probes per axis of the cascade above (for bilinear taps)
    int32_t nd_up;      // directions of the cascade above
    int32_t has_up;     // 1 if the merged cascade above is read
    int32_t max_steps;  // bound on cells a ray can cross
    double s;           // probe spacing, cells
    double ta, tb;      // interval [ta, tb) in cells; tb = +inf on the top cascade
};

// Error plumbing: set the thread-local message and return the code.
int32_t fail(int32_t code, const std::string& msg);
int32_t hip_fail(hipError_t e, const char* what);

#define RCX_HIP_TRY(expr)                                   \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return ::rcx::hip_fail(e_, #expr); \
    } while (0)

// Kernel launchers (fs_kernels.hip). All enqueue on `st` and return the
// launch status.
hipError_t launch_prep(const float* chi, const float* eta, float2* F, int32_t n_wave, int64_t ncell,
                       float voxel, hipStream_t st);
// Wavelengths per batch of the field and cascade layouts.
int32_t batch_width();
// Fb: the batch's slice of F ([ncell][batch_width] float2); up/out: cascade
// buffers [rays][batch_width].
hipError_t launch_march_merge(const LevelDesc& L, int32_t nx, int32_t nz, const float2* Fb,
                              const double4* dirs, const float* up, float* out, hipStream_t st);
hipError_t launch_j(const float* I0, float* J, int32_t n_wave, int32_t batch, int64_t ncell, int32_t n0,
                    hipStream_t st);

}  // namespace rcx
