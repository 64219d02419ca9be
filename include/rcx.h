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
#define RCX_E_NONFINITE (-6)   /* an input value is not finite or out of range
                                  (only with RCX_FLAG_CHECK_INPUT)              */

/* Cascade interval rule (Eq. RcScalingLaw, alpha = 2). */
#define RCX_T_GEOMETRIC 0  /* t_0 = 0, t_i = c0_t1 * 4^(i-1)                    */
#define RCX_T_LENGTH_X4 1  /* t_i = c0_t1 * (4^i - 1) / 3 (lengths x4)          */

/* Storage of merged cascade radiance between levels. F16_SCALED stores
 * cascades >= 1 as 16-bit codes with FP16's precision and a per-wavelength
 * exponent offset: the FP32 radiance rounded to a 10-bit significand (to
 * nearest, ties to even; relative rounding 2^-11) with its exponent rebased
 * into 6 bits below 2 x the wavelength's largest source function (FP16's
 * sign bit spent on range, radiances being non-negative), so 63 binades
 * keep that precision; smaller values flush to 0. Valid because no merged
 * radiance exceeds the largest source function along its path. Cascade 0
 * stays FP32. */
#define RCX_STORE_F32 0
#define RCX_STORE_F16_SCALED 1
/* rcx_params.flags */
#define RCX_FLAG_BILINEAR_FIX 1u
/* Check the inputs of every call before computing (formal solves, batches,
 * emergent intensity: chi and eta finite and >= 0; non-LTE atmospheres: T,
 * n_e and ntot finite and > 0, velocities finite). One extra pass over the
 * inputs and one stream synchronisation per call; a failed check returns
 * RCX_E_NONFINITE (rcx_last_error names the array and the kind of value)
 * before anything else is enqueued. */
#define RCX_FLAG_CHECK_INPUT 2u

/* Uniform 2D grid. chi is per unit of voxel_scale length: the optical depth
 * of a path of dt cells is chi * dt * voxel_scale (Sec. 3.2). */
typedef struct {
    int32_t nx, nz;
    double voxel_scale;
} rcx_grid;

/* Cascade parameters (Sec. 2.3; Sec. 4.5 gives the defaults).
 *   n_cascades: 0 = automatic, ceil(log4(max(nx, nz))) + 2.
 *   c0_dirs:    directions on cascade 0 (4); cascade i has c0_dirs * 4^i,
 *               the cone centres theta = 2 pi (k + 1/2) / N_i.
 *   c0_t1:      end of the cascade-0 interval = start of cascade 1, in cells.
 *   t_rule:     RCX_T_GEOMETRIC or RCX_T_LENGTH_X4.
 *   storage:    RCX_STORE_F32 or RCX_STORE_F16_SCALED.
 *   n_incl:     inclination rays per flatland ray, in [1, 16] (Sec. 3.1, 2D
 *               invariance): rays with the same x-z projection inclined to
 *               the invariant y axis, mu = cos(inclination) on a Gauss-Radau
 *               rule over [0, 1] with the node mu = 0 (the in-plane ray)
 *               fixed; J = sum_m w_m J_m, J_m the flatland J with the path
 *               per projected cell scaled by 1/sqrt(1 - mu_m^2). 1 = flatland
 *               (the default); the paper uses 8 (with FP32 cascades the 8
 *               run as slots of one march: 8 x the cascade workspace).
 *               The formal solve and the non-LTE solver support n_incl > 1
 *               (the non-LTE solver marches one pass per inclination);
 *               batches return RCX_E_UNSUPPORTED for it.
 *   flags:      RCX_FLAG_BILINEAR_FIX, RCX_FLAG_CHECK_INPUT or their OR, or 0
 *               (other bits must be 0).
 *               RCX_FLAG_BILINEAR_FIX (Sec. 2.5, the remedy for ringing and
 *               for light leaking through thin occluders): every cascade
 *               below the top traces each interval once per bilinear probe
 *               q of the cascade above, from its start p + t_i w_k to the
 *               start q + t_{i+1} w_k of the child cone on q, merges it with
 *               q's children and sums the four results with the bilinear
 *               weights (4 x the rays below the top cascade). Formal solve
 *               only (with any n_incl): batches and the non-LTE solver
 *               return RCX_E_UNSUPPORTED for it. */
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
 * c0_t1 <= 0, n_cascades outside [1, 16], n_incl outside [1, 16], unknown
 * flags); RCX_E_UNSUPPORTED (unknown storage, too many top-cascade
 * directions, more than 2^24 cells); RCX_E_NOMEM; RCX_E_HIP. On error *out
 * is NULL. */
int32_t rcx_plan_create(const rcx_grid* g, const rcx_params* p, int32_t max_wave, rcx_plan** out);

/* Sparse solve (Sec. 3.5). active_host [nz][nx] (host, caller-owned, read
 * during the call) flags the cells of interest, non-zero = flagged; they are
 * the flagged probes of cascade 0, and every probe of cascade i+1 that is a
 * bilinear tap (clamped at the grid edge) of a flagged probe of cascade i is
 * flagged in turn, up to the top cascade. Later rcx_formal_solve calls on
 * the plan march only the flagged probes' rays, treat unflagged cells as
 * transparent with no emission, and write J = 0 at unflagged cells; with
 * the bilinear fix the flagged probes trace their four rays each.
 * active_host = NULL makes every probe active again (the dense solve).
 * level_active_host (nullable) receives the number of flagged probes of
 * each cascade [n_cascades]. Builds the flagged-probe lists on the host and
 * copies them to plan-owned device memory (synchronous; memory the size of
 * one int32 per flagged probe plus one byte per cell).
 * Errors: RCX_E_INVALID (null plan); RCX_E_HIP (allocation or copy: the plan
 * is then dense). */
int32_t rcx_plan_set_active_host(rcx_plan* plan, const uint8_t* active_host, int64_t* level_active_host);

/* Bytes of device workspace a solve of n_wave wavelengths needs. */
int32_t rcx_plan_workspace_bytes(const rcx_plan* plan, int32_t n_wave, size_t* bytes_host);

/* Work counts of the plan's geometry (computed on the host, cached). */
int32_t rcx_plan_work(rcx_plan* plan, rcx_work* out_host);

/* GivenFs formal solution (Sec. 3.8 mode GivenFs; method Secs. 2.2-2.3, 3.2):
 * isotropic chi, eta [n_wave][nz][nx] (device, float32) -> J [n_wave][nz][nx]
 * (device, float32), the flatland mean intensity (1/N_0) sum_k I_0(k) of the
 * merged cascade 0. Free-space boundary (Sec. 3.4). chi must be >= 0;
 * cells with chi * voxel_scale < 1e-20 are treated as having that opacity.
 * Grids are limited to nx * nz <= 2^24 cells (RCX_E_UNSUPPORTED beyond).
 * workspace: device buffer of at least rcx_plan_workspace_bytes(n_wave)
 * bytes, or NULL to use the plan's own.
 * Errors: RCX_E_INVALID (null arrays, n_wave <= 0 or > max_wave);
 * RCX_E_WORKSPACE; RCX_E_NONFINITE (with RCX_FLAG_CHECK_INPUT: a chi or eta
 * value not finite or negative; nothing is computed); RCX_E_HIP. */
int32_t rcx_formal_solve(rcx_plan* plan, int32_t n_wave, const float* chi, const float* eta,
                         float* J, void* workspace, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * formal solve of rcx_formal_solve with no allocation at all. Its workspace
 * is the library's scratch, a 64 MiB array held on each GPU the library
 * runs on until the process ends (its address on the device is looked up
 * once, by rcx_plan_create). Every call on a GPU shares that GPU's scratch:
 * calls that overlap on one GPU (two streams, two threads) race and must
 * be ordered by the caller; the scratch keeps the last call's contents and
 * every value a solve reads from it is written first by that solve. Calls
 * no hipMalloc, hipFree or allocating library routine; the plan must not
 * have kernel timing enabled (it records events).
 * Errors: RCX_E_INVALID (null arrays, n_wave outside [1, max_wave], timing
 * enabled); RCX_E_WORKSPACE when rcx_plan_workspace_bytes(n_wave) exceeds
 * the 64 MiB (e.g. more than about 256^2 cells x 16 wavelengths: use
 * rcx_formal_solve); RCX_E_NONFINITE; RCX_E_HIP. */
int32_t rcx_formal_solve_noalloc(rcx_plan* plan, int32_t n_wave, const float* chi, const float* eta, float* J,
                                 hipStream_t stream);

/* Emergent intensity along parallel long characteristics (Sec. 3.9, the
 * post-processing formal solver): a beam of n_rays rays of light direction
 * (wx, wz) (any non-zero vector; normalised), one cell apart across the beam
 * and centred on the domain (ray j at offset j + 1/2 - n_rays/2 cells along
 * (-wz, wx) from the domain centre), each traced front to back from outside
 * the domain on the observer's side through isotropic chi, eta
 * [n_wave][nz][nx] (device, float32, as for rcx_formal_solve) with the same
 * cell walk and piecewise-constant update as the cascade march; nothing
 * enters from behind (free-space boundary). I [n_wave][n_rays] (device,
 * float32, caller-owned). Uses the plan's own workspace (the field batches),
 * so it must not overlap another call on the plan; a sparse plan's
 * unflagged cells are empty. Errors: RCX_E_INVALID (null arrays, n_wave
 * outside [1, max_wave], n_rays <= 0, zero or non-finite direction);
 * RCX_E_NONFINITE (with RCX_FLAG_CHECK_INPUT). */
int32_t rcx_emergent(rcx_plan* plan, int32_t n_wave, const float* chi, const float* eta, double wx, double wz,
                     int32_t n_rays, float* I, hipStream_t stream);

/* Kernel timing for measurement: when enabled, every solve records HIP
 * events on its stream around each cascade's march+merge launch and around
 * the other launches (prep, J). rcx_plan_get_timing() synchronises on the
 * recorded events and returns the accumulated milliseconds per cascade
 * (ms_level_host[n_cascades]), the accumulated prep + J time, the number of
 * march+merge launches and of solves since the last get, then resets. */
int32_t rcx_plan_set_timing(rcx_plan* plan, int32_t enable);
int32_t rcx_plan_get_timing(rcx_plan* plan, double* ms_level_host, double* ms_other_host,
                            int64_t* n_march_launches_host, int64_t* n_solves_host);

/* Launch order of cascade `level`'s march (the rays of a launch run in
 * this order; results do not depend on it, bit for bit): tile_p = 0 for
 * probe-major order (directions of a probe consecutive), else groups of
 * tile_p x tile_p probes x tile_d directions (tile_d a multiple of 4
 * dividing the cascade's directions), and workgroups given to the 8 XCDs in
 * chunks of xcd_chunk consecutive ones. shared_walk = 1 (0 or 1): with an
 * even tile_p, in the basic march of a dense plan with one inclination (not
 * the bilinear-fix kernel, not the cascade-0 J launch; elsewhere the
 * setting is kept but changes nothing), the march takes the rays of a group
 * probe-fastest, so the 4 rays of a
 * wavefront are 4 probes of one direction, and walks their cells once for
 * all 4 (their probe centres lie whole cells apart; every ray still
 * marches exactly its own segments). Defaults: 4 x 4 x 32, chunk 128, row
 * walks, on cascades with at least 256 directions; probe-major, chunk 128,
 * below. A sparse plan's flagged-probe lists are rebuilt to follow the
 * order (synchronous). RCX_E_INVALID for a bad level or order. */
int32_t rcx_plan_set_order(rcx_plan* plan, int32_t level, int32_t tile_p, int32_t tile_d, int32_t xcd_chunk,
                           int32_t shared_walk);
/* order4_host = {tile_p, tile_d, xcd_chunk, shared_walk} of cascade `level`. */
int32_t rcx_plan_get_order(const rcx_plan* plan, int32_t level, int32_t* order4_host);

/* Autotuner of the launch order (growth pattern (2)): for every cascade
 * with at least 256 directions, times the plan's formal solve of up to 32
 * wavelengths on uniform fields (the march's work and memory traffic do not
 * depend on the values) for each candidate order, tile_p in {0, 2, 4, 8} x
 * tile_d in {16, 32, 64} x xcd_chunk in {32, 128, 512} x shared_walk in
 * {0, 1} (for tile_p > 0, where the walk applies), with the plan's
 * kernel timing, and keeps the fastest per cascade. cache_path (nullable): a
 * text file of JSON lines keyed by the device (architecture, compute units)
 * and the plan's geometry, storage, flags and sparsity; a hit applies the
 * stored orders without timing, a miss appends the result. Allocates its
 * temporary fields (and a workspace when the plan has none) and
 * synchronises the stream; pending timing records are consumed. Errors:
 * RCX_E_INVALID; RCX_E_NOMEM; RCX_E_HIP. */
int32_t rcx_autotune(rcx_plan* plan, const char* cache_path, hipStream_t stream);

/* Release a plan and its device memory. NULL is accepted. */
int32_t rcx_plan_destroy(rcx_plan* plan);

/* ================================================================ batches
 * Many formal solutions at once (several atmospheres, each with its
 * wavelength batches; every one an independent formal solution, Secs. 2.3
 * and 3.2). Tasks (atmosphere, 16-wavelength batch, cascade) are grouped
 * into generations by their distance from the atmosphere's top cascade;
 * each generation is one launch that sweeps the rays of all its tasks, and
 * stream order provides every dependency, so no workgroup waits on another.
 * An atmosphere whose every cascade holds at least 2^19 rays (about 512^2
 * and up) fills the GPU alone: it runs through its plan's own solve (the
 * per-cascade launches of rcx_formal_solve) in the same sequence. Cascade 0
 * writes J directly. The sequence of launches is captured into a HIP graph
 * and replayed, re-captured when the input or output pointers change. */
typedef struct rcx_batch rcx_batch;

/* n_atm atmospheres with grids[a] and n_wave[a] wavelengths. p as for
 * rcx_plan_create, with n_cascades = 0 (automatic per atmosphere), c0_dirs =
 * 4, n_incl = 1 and no flag but RCX_FLAG_CHECK_INPUT (RCX_E_UNSUPPORTED
 * otherwise). Allocates every buffer. */
int32_t rcx_batch_create(int32_t n_atm, const rcx_grid* grids, const int32_t* n_wave, const rcx_params* p,
                         rcx_batch** out);
/* Sparse atmosphere atm of the batch (Sec. 3.5): its plan flags the cells
 * as rcx_plan_set_active_host does (NULL = dense again); the batched solve
 * then marches only its flagged probes' rays, empties its unflagged cells
 * and writes J = 0 there. Rebuilds the task list (and the graph) on the next
 * solve. RCX_E_INVALID for a null batch or atm outside [0, n_atm). */
int32_t rcx_batch_set_active_host(rcx_batch* s, int32_t atm, const uint8_t* active_host);
/* Launch order of every atmosphere's cascades with >= 256 directions, as
 * rcx_plan_set_order: groups of tile_probes x tile_probes probes x
 * tile_dirs directions (default 4 x 4 x 32), or tile_probes = 0 for
 * probe-major order. Results do not depend on it. Waits for the device. */
int32_t rcx_batch_set_order(rcx_batch* b, int32_t tile_probes, int32_t tile_dirs);
/* Enqueue through the captured graph (1, default) or by direct launches (0). */
int32_t rcx_batch_set_graph(rcx_batch* b, int32_t enable);
/* chi_host[a], eta_host[a], J_host[a]: host arrays of n_atm device pointers
 * to [n_wave[a]][nz][nx] float32, as for rcx_formal_solve; the pointers are
 * recorded in the graph and must stay valid while they are in use.
 * Enqueues on the stream without synchronising when the pointers are those
 * of the previous call (a replay of the captured graph); new pointers first
 * synchronise the stream (the work list and the graph that a solve still in
 * flight reads are then rebuilt). rcx_batch_set_order, _set_graph,
 * _set_active_host and _destroy wait for the device to finish. With
 * RCX_FLAG_CHECK_INPUT every call checks chi and eta first (synchronising).
 * Errors: RCX_E_INVALID (null arguments); RCX_E_NONFINITE; RCX_E_HIP. */
int32_t rcx_batch_solve(rcx_batch* b, const float* const* chi_host, const float* const* eta_host,
                        float* const* J_host, hipStream_t stream);
/* Work summed over atmospheres and wavelengths (rcx_work semantics). */
int32_t rcx_batch_work(const rcx_batch* b, int64_t* rays_nonempty_host, int64_t* cell_steps_host);
/* Kernel launches one solve enqueues, from the work list the last solve
 * built (both 0 before the first solve): *march_host march launches (each
 * the next cascade of every active chain), *all_host those plus the field
 * preparation and masking launches (the input check not counted). */
int32_t rcx_batch_launches(const rcx_batch* b, int32_t* march_host, int32_t* all_host);
/* Time each candidate launch order (tile_probes, tile_dirs) in {(0, -),
 * (2, 32), (4, 16), (4, 32), (4, 64), (8, 32)} (rcx_batch_set_order) on
 * these inputs and keep the fastest: *best_host = tile_probes * 1000 +
 * tile_dirs. cache_path (or NULL): a text file of JSON lines keyed by the
 * batch's shapes; a hit skips timing, a miss appends the result. */
int32_t rcx_batch_autotune(rcx_batch* b, const float* const* chi_host, const float* const* eta_host,
                           float* const* J_host, const char* cache_path, int32_t* best_host, hipStream_t stream);
int32_t rcx_batch_destroy(rcx_batch* b);

/* ================================================================ non-LTE
 * The non-LTE iteration of Sec. 3.3: opacities and emissivities from level
 * populations, the radiance-cascades formal solution per wavelength with
 * Doppler-shifted Voigt lines evaluated per ray step (Sec. 3.2), the
 * diagonal cascade-0 operator and the "same-preconditioning" MALI rates
 * (Rybicki & Hummer 1992, as adapted in Sec. 3.3), and the per-cell rate
 * matrix Gamma solved in FP64 with its diagonal from conservation.
 *
 * Model: one atom, levels 0..n_levels-1 with the last level the continuum
 * (ionised stage); every wavelength belongs to exactly one transition (its
 * governing transition, Sec. 3.3), wavelengths are grouped by transition in
 * the order lines then continua; no background opacity; angular
 * quadrature 1/N_0 per cascade-0 direction, flatland or with the
 * inclinations of rcx_params.n_incl; free-space boundary; electron density
 * fixed unless charge conservation is on. */

#define RCX_NLTE_MAX_LEVELS 6
#define RCX_NLTE_MAX_LINES 8
#define RCX_NLTE_MAX_CONTS 4

/* Atomic model (host struct). Energies in eV from the ground level;
 * statistical weights; lines (lower, upper, rest wavelength [nm], oscillator
 * strength f); bound-free continua (lower, upper = n_levels-1, edge
 * wavelength [nm], cross-section at the edge [m^2], scaling as lambda^3
 * below the edge); atomic mass [amu]; collisional de-excitation coefficients
 * q_coll [m^3/s] per transition (lines first, then continua): the downward
 * rate is n_e q (T / 1e4 K)^-1/2, the upward one follows by detailed
 * balance. Natural damping of a line is the sum of the Einstein A of all
 * lines leaving its upper and its lower level. */
typedef struct {
    int32_t n_levels, n_lines, n_conts, pad_;
    double E_eV[RCX_NLTE_MAX_LEVELS];
    double g[RCX_NLTE_MAX_LEVELS];
    double mass_amu;
    int32_t line_lower[RCX_NLTE_MAX_LINES], line_upper[RCX_NLTE_MAX_LINES];
    double line_lambda_nm[RCX_NLTE_MAX_LINES], line_f[RCX_NLTE_MAX_LINES];
    int32_t cont_lower[RCX_NLTE_MAX_CONTS], cont_upper[RCX_NLTE_MAX_CONTS];
    double cont_edge_nm[RCX_NLTE_MAX_CONTS], cont_alpha0[RCX_NLTE_MAX_CONTS];
    double q_coll[RCX_NLTE_MAX_LINES + RCX_NLTE_MAX_CONTS];
} rcx_atom;

typedef struct rcx_nlte rcx_nlte;

/* Create a non-LTE solver for grid g (voxel_scale in metres) and the
 * cascade parameters p, with n_wave wavelengths: lambda_nm_host[n_wave],
 * trans_host[n_wave] (transition index of each wavelength, grouped and
 * ordered as described above) and dnu_host[n_wave] (frequency quadrature
 * weights of the rate integrals, Hz). All host arrays are copied.
 * p->storage = RCX_STORE_F16_SCALED stores cascades >= 1 of every
 * formal solution as the 16-bit codes of RCX_STORE_F16_SCALED, the exponent
 * offset of each wavelength from its largest source function (lines:
 * S_line; continua: eta/chi); cascade 0, the rates and the rate matrix stay
 * FP32/FP64.
 * p: c0_dirs = 4, flags 0 or RCX_FLAG_CHECK_INPUT; n_incl as for
 * rcx_plan_create (Sec. 3.1: every inclination m marches the flatland rays
 * with the path per projected cell 1/sin(theta_m) and sin(theta_m) of the
 * in-plane velocity along them, in Psi* the path through the cell
 * l / sin(theta_m); J and the rate coefficients are the sums over m with the
 * Gauss-Radau weights; the paper iterates with 8).
 * Errors: RCX_E_INVALID (nulls, sizes, ungrouped or out-of-range
 * transitions, a wavelength outside its continuum's edge);
 * RCX_E_UNSUPPORTED (more levels/lines/continua than the maxima);
 * RCX_E_NOMEM; RCX_E_HIP. */
int32_t rcx_nlte_create(const rcx_grid* g, const rcx_params* p, const rcx_atom* atom, int32_t n_wave,
                        const double* lambda_nm_host, const int32_t* trans_host, const double* dnu_host,
                        rcx_nlte** out);

/* Atmosphere (device arrays, [nz][nx]): temperature T [K], electron
 * density ne [m^-3], total atom density ntot [m^-3] (all levels incl. the
 * ionised stage), velocity vel [2][nz][nx] float32 (vx, vz) [m/s]. Computes
 * on the device in FP64 the Saha-Boltzmann populations, collisional rates,
 * thermal widths and damping, and fills the Voigt table H(a, x) in FP64
 * (Fourier-integral form of the Voigt function, Gauss-Legendre panels) for
 * the damping range present. Synchronises the stream once (damping range).
 * With RCX_FLAG_CHECK_INPUT (given to rcx_nlte_create) T, ne and ntot must
 * be finite and positive and vel finite, else RCX_E_NONFINITE and nothing
 * changes. */
int32_t rcx_nlte_set_atmosphere(rcx_nlte* s, const double* T, const double* ne, const double* ntot,
                                const float* vel, hipStream_t stream);

/* LTE (Saha-Boltzmann) populations [n_levels][nz][nx] float64 (device). */
int32_t rcx_nlte_lte_populations(rcx_nlte* s, double* pops, hipStream_t stream);

/* One formal solution at populations pops [n_levels][nz][nx] (device,
 * float64): opacity synthesis, every cascade top-down per wavelength batch,
 * and at cascade 0 the preconditioned rate coefficients. rates (device,
 * float32, [n_trans][2][nz][nx]) receives, per transition t, the upward
 * coefficient (multiplies n_lower) and the downward coefficient (multiplies
 * n_upper):
 *   up   = sum_{lambda,k} W w_k V_ij I_eff,
 *   down = sum_{lambda,k} W w_k [V_ji I_eff + U_ji (1 - chi_t Psi*)],
 *   I_eff = I - Psi* eta_t,  Psi* = (1 - e^{-chi l_k}) / chi,
 * with W = 4 pi dnu / (h nu), w_k = 1/N_0, l_k the distance from the cell
 * centre to its edge along direction k, chi_t and eta_t the transition's own
 * opacity and emissivity at pops. J (device float32 [n_wave][nz][nx]) may
 * be NULL. */
int32_t rcx_nlte_formal_solve_rates(rcx_nlte* s, const double* pops, float* rates, float* J,
                                    hipStream_t stream);

/* Statistical equilibrium (Sec. 3.3): per cell, Gamma[j][i] = upward rate
 * i->j plus collisions, Gamma[i][j] = downward, diagonal = minus the column
 * sum (FP64), the row of the most populated level replaced by sum n = ntot,
 * solved with partial pivoting in FP64; pops_inout updated in place.
 * *max_rel_change_host = max over cells and levels of |n_new - n_old| /
 * n_new (synchronises the stream). */
int32_t rcx_nlte_stat_eq(rcx_nlte* s, const float* rates, double* pops_inout,
                         double* max_rel_change_host, hipStream_t stream);

/* The iteration of Sec. 3.3 from pops_inout until the max relative change
 * drops below tol or max_iter iterations: formal solution with rates,
 * statistical equilibrium, repeat (the paper's plain iteration; with
 * rcx_nlte_set_acceleration, Ng acceleration after the equilibrium step).
 * Returns RCX_OK when converged, RCX_W_NOT_CONVERGED when max_iter was
 * reached. *iters_host and *last_change_host report the iterations run and
 * the last change (of the equilibrium step, before any extrapolation).
 * Synchronises the stream once per iteration (8 bytes), and once more per
 * Ng step. */
int32_t rcx_nlte_iterate(rcx_nlte* s, double* pops_inout, int32_t max_iter, double tol,
                         int32_t* iters_host, double* last_change_host, hipStream_t stream);

/* Launch orders of the solver's marches: rcx_autotune on the solver's own
 * plan (its formal solve of 16 wavelengths timed for each candidate order,
 * cache_path as there). The line and continuum marches take the chosen
 * orders too; every result is bitwise the same under any order (each ray's
 * arithmetic does not depend on where it runs). Synchronises the stream.
 * Errors: as rcx_autotune. */
int32_t rcx_nlte_autotune(rcx_nlte* s, const char* cache_path, hipStream_t stream);

/* Kernel timing for measurement: when enabled, every march launch of the
 * formal solution (rcx_nlte_formal_solve_rates, rcx_nlte_iterate) records
 * two HIP events on its stream. rcx_nlte_get_timing synchronises on them
 * and returns, for the line batches [0] and the continuum batches [1]: the
 * summed kernel time in ms, the launch count, and the cell steps x
 * wavelengths those launches marched (the dense per-cascade counts of
 * rcx_plan_work; per inclination); it then drops the records. Enabling
 * counts the plan's work first (host loop over every ray). Errors:
 * RCX_E_INVALID (null arguments); RCX_E_HIP. */
int32_t rcx_nlte_set_timing(rcx_nlte* s, int32_t enable);
int32_t rcx_nlte_get_timing(rcx_nlte* s, double* ms_host, int64_t* launches_host, int64_t* steps_host);

/* Ng acceleration of rcx_nlte_iterate (not used by the paper; off by
 * default): order M in [1, 3] (0 = off) extrapolates from the last M + 2
 * iterates, x = (1 - sum c_j) x_0 + sum c_j x_j with c the least-squares
 * solution of sum w (d_0 - sum_j c_j (d_0 - d_j))^2, d_k = x_k - x_{k+1},
 * w = 1/x_0^2 (Ng 1974; Auer 1987), first after `delay` iterations, then
 * every `period`; the iterate history restarts after each extrapolation and
 * at this call. Allocates (M_max + 2) x n_levels x ncell FP64 of device
 * memory on first use. RCX_E_INVALID for order outside [0, 3], delay < 0
 * or period < 1. */
int32_t rcx_nlte_set_acceleration(rcx_nlte* s, int32_t order, int32_t delay, int32_t period);

/* Emergent spectra (Sec. 3.9) at populations pops [n_levels][nz][nx]
 * (device, FP64): the beam of rcx_emergent (light direction (wx, wz), ray j
 * at offset j + 1/2 - n_rays/2 cells along (-wz, wx) from the domain
 * centre), traced through the opacities and emissivities synthesised from
 * pops, with the line profiles Doppler-shifted along the rays as in the
 * formal solution. I [n_wave][n_rays] (device, float32, caller-owned);
 * unflagged cells of a sparse solver are empty. Uses the solver's field
 * buffers (not concurrently with another call on it). RCX_E_INVALID for
 * null arguments, n_rays <= 0, a zero direction or before
 * rcx_nlte_set_atmosphere. */
int32_t rcx_nlte_emergent(rcx_nlte* s, const double* pops, double wx, double wz, int32_t n_rays, float* I,
                          hipStream_t stream);

/* Charge conservation (Sec. 3.3; off by default): after each equilibrium
 * step of rcx_nlte_stat_eq / rcx_nlte_iterate, one Newton-Raphson step per
 * cell on the populations and the electron density, with the equations
 * Gamma(n_e) n = 0 (one row replaced by particle conservation, the most
 * populated level's after the equilibrium step) and n_e = n_c (the
 * continuum level: this atom, taken as hydrogen, is the only electron
 * donor). dGamma/dn_e takes the rates proportional to n_e (collisional
 * downward, bound-bound collisional upward, radiative recombination)
 * divided by n_e; the other rates are held. The step is skipped in a cell
 * where it would make a population or n_e non-positive. The solver's n_e
 * (initially the one given to rcx_nlte_set_atmosphere) is updated in place,
 * and the LTE populations, collisional rates and continuum LTE ratios are
 * recomputed from it; the reported change includes |dn_e| / n_e. Setting the
 * atmosphere again restores the given n_e. */
int32_t rcx_nlte_set_charge_conservation(rcx_nlte* s, int32_t enable);

/* Sparse non-LTE solve (Sec. 3.5): cells with T < t_cut (the paper's
 * temperature flag, typically 250 kK) are flagged, and the solver's plan is
 * given them as by rcx_plan_set_active_host (their bilinear parents flagged
 * up to the top cascade; only flagged probes' rays are marched). Unflagged
 * cells are transparent with no emission, their rates (and J) are 0 and
 * their populations and n_e are held by the equilibrium and conservation
 * steps; the change covers the flagged cells. t_cut <= 0 clears the flags.
 * Uses the atmosphere as set (call again after setting a new one); copies T
 * to the host (synchronous). level_active_host (nullable) receives the
 * flagged probes per cascade. */
int32_t rcx_nlte_set_temperature_cut(rcx_nlte* s, double t_cut, int64_t* level_active_host);

/* Pressure conservation (Sec. 3.3; needs charge conservation, else
 * RCX_E_INVALID): after each charge step the hydrogen density becomes
 * n_Htot = P/(kT) - n_e, holding the gas pressure (A_tot n_Htot + n_e) k T
 * of the atmosphere as set (A_tot = 1: this atom is the only species), and
 * every population is scaled with it; the change includes |dn_Htot| /
 * n_Htot. */
int32_t rcx_nlte_set_pressure_conservation(rcx_nlte* s, int32_t enable);

/* Starting n_e from the collisional rates alone (Sec. 3.3): n_iter
 * equilibrium + charge steps with the radiative rates set to zero, from LTE
 * at the current n_e; leaves the solver's n_e (and the LTE populations,
 * collisional rates and the held pressure) at the result. Synchronous;
 * allocates and frees one populations-sized temporary. RCX_E_INVALID for a
 * null solver, n_iter < 1, or before rcx_nlte_set_atmosphere. */
int32_t rcx_nlte_collisional_ne(rcx_nlte* s, int32_t n_iter, hipStream_t stream);

/* The solver's current electron density [ncell] (device, FP64) into ne
 * (device, caller-owned), enqueued on the stream. RCX_E_INVALID for a null
 * argument or before rcx_nlte_set_atmosphere. */
int32_t rcx_nlte_get_ne(rcx_nlte* s, double* ne, hipStream_t stream);

/* Line profile of the march (the Voigt function H(a, x) of Sec. 3.3's line
 * opacity), chosen at rcx_nlte_set_atmosphere:
 *   RCX_PROFILE_AUTO   the expansion about a = 0 when every cell has damping
 *                      a <= 5e-3 (H = e^{-x^2} (1 + a^2 (1 - 2x^2))
 *                      - (2a/sqrt(pi)) (1 - 2x F(x)), F Dawson's function
 *                      from a one-row LDS table; relative error below 7e-6),
 *                      else the compact table;
 *   RCX_PROFILE_TABLE  always the compact (a, x) table.
 * Takes effect at the next rcx_nlte_set_atmosphere. RCX_E_INVALID for
 * another mode. */
#define RCX_PROFILE_AUTO 0
#define RCX_PROFILE_TABLE 1
int32_t rcx_nlte_set_line_profile(rcx_nlte* s, int32_t mode);

/* Evaluate the device Voigt table (bilinear in (a, |x|), asymptotic series
 * beyond its x range) at n points: a, x, out device float32 arrays. For
 * checking the table against a reference. */
int32_t rcx_nlte_voigt_eval(rcx_nlte* s, int32_t n, const float* a, const float* x, float* out,
                            hipStream_t stream);
/* The same for the profile the line march uses (rcx_nlte_set_line_profile):
 * the expansion about a = 0, or the compact table (cubic Hermite in x on
 * [0, 8] at spacing 1/32, linear in a on at most 9 nodes over the
 * atmosphere's damping range, filled in FP64 from the Fourier integrals of
 * H and of the Faraday-Voigt function); every march workgroup copies its
 * table into LDS; the same asymptotic series beyond x = 8. With the table,
 * a is clamped to the atmosphere's damping range. */
int32_t rcx_nlte_voigt_eval_march(rcx_nlte* s, int32_t n, const float* a, const float* x, float* out,
                                  hipStream_t stream);

/* Number of transitions and of levels of the solver's atom. */
int32_t rcx_nlte_dims(const rcx_nlte* s, int32_t* n_levels_host, int32_t* n_trans_host);

/* Release the solver. NULL is accepted. */
int32_t rcx_nlte_destroy(rcx_nlte* s);

/* ===================================================== learned warm start
 * A small multilayer perceptron x [B][n_in] -> (Linear, SiLU) x depth ->
 * Linear -> y [B][n_out], trained by Adam on an MSE loss with BF16 MFMA
 * products (FP32 accumulation) and FP32 master weights. It predicts
 * warm-start level populations for the non-LTE iteration; the plain
 * iteration from its prediction still decides convergence.
 * Parameters are one flat FP32 array, layer by layer: W [fan_in][fan_out]
 * row-major, then b [fan_out]. Initial values come from the caller. */
typedef struct rcx_mlp rcx_mlp;

/* Create a network for batches up to max_batch. Supports 1 <= n_in <= 16,
 * 1 <= n_out <= 64, 1 <= depth <= 16, width a multiple of 64 in [64, 512]
 * (RCX_E_UNSUPPORTED otherwise). Parameters start at zero. */
int32_t rcx_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t max_batch, rcx_mlp** out);
int32_t rcx_mlp_n_params(const rcx_mlp* m, int64_t* n_host);
/* Copy parameters in/out (host arrays of rcx_mlp_n_params floats; both
 * synchronise the device). set_params also resets the Adam moments. */
int32_t rcx_mlp_set_params(rcx_mlp* m, const float* flat_host, int64_t n);
int32_t rcx_mlp_get_params(const rcx_mlp* m, float* flat_host, int64_t n);
/* Inference: x [batch][n_in], y [batch][n_out] (device FP32); any batch size
 * (processed in chunks of max_batch). */
int32_t rcx_mlp_forward(rcx_mlp* m, const float* x, float* y, int32_t batch, hipStream_t stream);
/* Loss (mean squared error over samples and outputs, to *loss_host) and its
 * gradient with respect to the flat parameters (grad: device FP32, may be
 * NULL). batch <= max_batch. Synchronises the stream. */
int32_t rcx_mlp_gradients(rcx_mlp* m, const float* x, const float* y_ref, int32_t batch, float* grad,
                          float* loss_host, hipStream_t stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) at
 * learning rate lr on a batch; *loss_host gets the loss before the step. */
int32_t rcx_mlp_train_step(rcx_mlp* m, const float* x, const float* y_ref, int32_t batch, float lr,
                           float* loss_host, hipStream_t stream);
int32_t rcx_mlp_destroy(rcx_mlp* m);

/* Warm-start features of every cell at populations pops (device FP64):
 * one formal solution with J, then feat [nz*nx][6] (device FP32) =
 * {log10 T, log10 ne, |v| [km/s], log10 chi_0 (line 0's centre opacity
 * [1/m]), log10 Jbar_0, log10 Jbar_1} with Jbar_t the profile-weighted mean
 * intensity of line t; each standardised as (f - mean)/std with
 * norm_host[2][6] = {means, stds} (NULL: no standardisation). Synchronises. */
int32_t rcx_nlte_features(rcx_nlte* s, const double* pops, const float* norm_host, float* feat, hipStream_t stream);
/* Log departure coefficients, the warm start's targets:
 * out [nz*nx][n_levels] (device FP32) = (log10(n_l / n_l^LTE) - mean_l)/std_l
 * with n^LTE the Saha-Boltzmann populations of the atmosphere,
 * norm_host[2][n_levels] (NULL: none). Synchronises. */
int32_t rcx_nlte_log_departures(rcx_nlte* s, const double* pops, const float* norm_host, float* out,
                                hipStream_t stream);
/* Populations from a prediction of the warm start's targets:
 * y [nz*nx][n_levels] (device FP32, standardised log10 departure
 * coefficients), targ_norm_host[2][n_levels] = {means, stds} (host, stds
 * positive); pops_out [n_levels][nz][nx] (device FP64) receives
 * n_l = ntot b_l n_l^LTE / sum_m b_m n_m^LTE, log10 b_l = y_l std_l + mean_l
 * (exponents above 30 are clamped), n^LTE the Saha-Boltzmann populations at
 * the solver's current n_e. The last step of rcx_nlte_warm_start.
 * Synchronises. RCX_E_INVALID for null arguments, non-finite norms or
 * non-positive stds, or before rcx_nlte_set_atmosphere. */
int32_t rcx_nlte_pops_from_prediction(rcx_nlte* s, const float* y, const float* targ_norm_host, double* pops_out,
                                      hipStream_t stream);
/* Learned warm start: LTE populations, one formal solution, features,
 * network inference, and populations n_l = ntot b_l n_l^LTE / sum_m b_m n_m^LTE
 * with log10 b the de-standardised prediction (targ_norm_host[2][n_levels]);
 * pops_out [n_levels][nz][nx] device FP64. The plain iteration started
 * from it still decides convergence. Synchronises. */
int32_t rcx_nlte_warm_start(rcx_nlte* s, rcx_mlp* net, const float* feat_norm_host, const float* targ_norm_host,
                            double* pops_out, hipStream_t stream);


/* Static description of a status code. */
const char* rcx_error_string(int32_t code);

/* Copy the calling thread's last error message into buf (always
 * NUL-terminated when n > 0). Returns the last status code. */
int32_t rcx_last_error(char* buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* RCX_H */
