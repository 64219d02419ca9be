/*
 * rcx.h -- C ABI of librcx, an MI355X (gfx950) radiance-cascades formal
 * solver (Osborne & Sannikov, arXiv:2408.14425).
 *
 * Conventions for every entry point:
 *   - Returns int32_t: RCX_OK (0) on success, a negative RCX_E_* code on
 *     error, or a positive RCX_W_* warning. The library never aborts and
 *     never prints; rcx_last_error() gives a thread-local message.
 *   - Array arguments are caller-owned DEVICE pointers unless the name ends
 *     in _host. The library never frees them and keeps none after the call
 *     returns.
 *   - Handles (rcx_plan) are library-owned and released by their _destroy.
 *   - Work is enqueued on the caller's hipStream_t and the call returns
 *     without synchronising, except for calls with _host outputs, which
 *     synchronise that stream. One plan must not be used on two streams at
 *     the same time.
 *   - Layouts are row-major with x fastest: fields [n_wave][nz][nx] float32;
 *     cell (x, z) covers [x, x+1) x [z, z+1) in cell units.
 */
#ifndef RCX_H
#define RCX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define RCX_OK 0
#define RCX_W_NOT_CONVERGED 1
#define RCX_E_INVALID (-1)     /* null pointer, non-positive size, bad enum     */
#define RCX_E_UNSUPPORTED (-2) /* valid request this build does not implement   */
#define RCX_E_NOMEM (-3)       /* device or host allocation failed              */
#define RCX_E_HIP (-4)         /* a HIP runtime call failed (see last error)    */
#define RCX_E_WORKSPACE (-5)   /* caller workspace too small                    */

/* Cascade interval rule (Eq. RcScalingLaw, alpha = 2). */
#define RCX_T_GEOMETRIC 0  /* t_0 = 0, t_i = c0_t1 * 4^(i-1)                    */
#define RCX_T_LENGTH_X4 1  /* t_i = c0_t1 * (4^i - 1) / 3 (lengths x4)          */

/* Storage of merged cascade radiance between levels. */
#define RCX_STORE_F32 0

/* Uniform 2D grid. chi is per unit of voxel_scale length: the optical depth
 * of a path of dt cells is chi * dt * voxel_scale (Sec. 3.2). */
typedef struct {
    int32_t nx, nz;
    double voxel_scale;
} rcx_grid;

/* Cascade parameters (Sec. 2.3; Sec. 4.6 gives the defaults).
 *   n_cascades: 0 = automatic, ceil(log4(max(nx, nz))) + 2.
 *   c0_dirs:    directions on cascade 0 (4); cascade i has c0_dirs * 4^i,
 *               the cone centres theta = 2 pi (k + 1/2) / N_i.
 *   c0_t1:      end of the cascade-0 interval = start of cascade 1, in cells.
 *   t_rule:     RCX_T_GEOMETRIC or RCX_T_LENGTH_X4.
 *   storage:    RCX_STORE_F32.
 *   n_incl:     inclination rays per flatland ray; must be 1 (flatland J).
 *   flags:      reserved, 0. */
typedef struct {
    int32_t n_cascades;
    int32_t c0_dirs;
    double c0_t1;
    int32_t t_rule;
    int32_t storage;
    int32_t n_incl;
    uint32_t flags;
} rcx_params;

/* Work counts of one formal solve per wavelength (Sec. 2.4 ray counts):
 * ray intervals over all cascades (all, and those that intersect the
 * domain), and cell steps (segments marched) summed over all intervals. */
typedef struct {
    int32_t n_cascades;
    int32_t top_skipped;      /* 1 if the top cascade lies wholly outside the domain */
    int64_t rays_all;
    int64_t rays_nonempty;
    int64_t cell_steps;
    int64_t level_rays[16];
    int64_t level_steps[16];
} rcx_work;

typedef struct rcx_plan rcx_plan;

/* Fill *p with the paper's defaults: auto cascades, 4 directions, t1 = 1.5,
 * geometric intervals, FP32 storage, flatland. */
int32_t rcx_params_default(rcx_params* p);

/* Create a plan for grid g and at most max_wave wavelengths per call
 * (Sec. 2.3 geometry; Sec. 3.2 probes at cell centres). Builds the
 * direction tables on the device and allocates the plan-owned workspace
 * used when a call passes workspace == NULL.
 * Errors: RCX_E_INVALID (null, nx/nz/max_wave <= 0, c0_dirs <= 0,
 * c0_t1 <= 0, n_cascades outside [1, 16]); RCX_E_UNSUPPORTED (n_incl != 1,
 * unknown storage); RCX_E_NOMEM; RCX_E_HIP. On error *out is NULL. */
int32_t rcx_plan_create(const rcx_grid* g, const rcx_params* p, int32_t max_wave, rcx_plan** out);

/* Bytes of device workspace a solve of n_wave wavelengths needs. */
int32_t rcx_plan_workspace_bytes(const rcx_plan* plan, int32_t n_wave, size_t* bytes_host);

/* Work counts of the plan's geometry (computed on the host, cached). */
int32_t rcx_plan_work(rcx_plan* plan, rcx_work* out_host);

/* GivenFs formal solution (Sec. 3.7 mode GivenFs; method Secs. 2.2-2.3, 3.2):
 * isotropic chi, eta [n_wave][nz][nx] (device, float32) -> J [n_wave][nz][nx]
 * (device, float32), the flatland mean intensity (1/N_0) sum_k I_0(k) of the
 * merged cascade 0. Free-space boundary (Sec. 3.4). chi must be >= 0;
 * cells with chi * voxel_scale < 1e-20 are treated as having that opacity.
 * Grids are limited to nx * nz <= 2^24 cells (RCX_E_UNSUPPORTED beyond).
 * workspace: device buffer of at least rcx_plan_workspace_bytes(n_wave)
 * bytes, or NULL to use the plan's own.
 * Errors: RCX_E_INVALID (null arrays, n_wave <= 0 or > max_wave);
 * RCX_E_WORKSPACE; RCX_E_HIP. */
int32_t rcx_formal_solve(rcx_plan* plan, int32_t n_wave, const float* chi, const float* eta,
                         float* J, void* workspace, size_t ws_bytes, hipStream_t stream);

/* Kernel timing for measurement: when enabled, every solve records HIP
 * events on its stream around each cascade's march+merge launch and around
 * the other launches (prep, J). rcx_plan_get_timing() synchronises on the
 * recorded events and returns the accumulated milliseconds per cascade
 * (ms_level_host[n_cascades]), the accumulated prep + J time, the number of
 * march+merge launches and of solves since the last get, then resets. */
int32_t rcx_plan_set_timing(rcx_plan* plan, int32_t enable);
int32_t rcx_plan_get_timing(rcx_plan* plan, double* ms_level_host, double* ms_other_host,
                            int64_t* n_march_launches_host, int64_t* n_solves_host);

/* Release a plan and its device memory. NULL is accepted. */
int32_t rcx_plan_destroy(rcx_plan* plan);

/* Static description of a status code. */
const char* rcx_error_string(int32_t code);

/* Copy the calling thread's last error message into buf (always
 * NUL-terminated when n > 0). Returns the last status code. */
int32_t rcx_last_error(char* buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* RCX_H */
